// tfft_kernels.hpp -- batched C2C FFT kernels with fused two-side ABFT (gfx950).
//
// Structure (TurboFFT Sec. 3.1, Fig. 3, re-designed for CDNA4):
//   * a "slot" is the set of P = Ns/E lanes that transform one (sub-)signal of
//     length Ns per transaction, E elements per lane held in registers;
//   * lane t of a slot holds elements t + P*r (r < E) before and after every
//     stage, so global loads/stores and LDS reads are unit-stride across lanes;
//   * stage s (radix R, L = product of the earlier radices) is a Stockham
//     autosort step: butterfly beta = t + i*P reads elements beta + j*Ns/R,
//     multiplies by w_{LR}^{j k} (k = beta mod L, from a precomputed table,
//     Sec. 3.1: no trigonometric functions in the kernel), applies the radix-R
//     DFT in registers and writes output j to g*L*R + k + j*L (g = beta div L);
//   * stages exchange data through LDS (Sec. 3.2); a slot runs T transactions
//     back to back (Sec. 4.3 multi-transaction).  In a launch of G slots'
//     worth of groups, transaction b of group g takes signal g + b G, so the
//     workgroups running at one time stream neighbouring signals, as with
//     one transaction each (consecutive signals per group would put every
//     concurrent workgroup in its own region of memory; ragged batches, whose
//     workspace is laid out by groups, keep consecutive signals).
// Three geometries share that machinery:
//   * Single : one whole signal per slot; slots of at most a wavefront sit
//     side by side in a wave (lane = slot*P + t) and synchronise with
//     wavefront fences; LDS rows of 128 bytes carry one pad element, which
//     keeps strided stores conflict-free and every address a base register
//     plus a compile-time offset;
//   * ColPass: pass A of N = N1*N2, column FFTs of length N1 (stride N2),
//     C adjacent columns per workgroup (lane = t*C + c), so every global
//     access moves C*S contiguous bytes and the LDS tile [m][c] is
//     conflict-free without padding (Sec. 3.2: lanes of a wave own different
//     sub-signals);
//   * RowPass: pass B, row FFTs of length N2 of the pass-A result multiplied
//     by w_N^{n2 k1}, C adjacent rows per workgroup, outputs written at
//     k1 + N1*k2 (the reorganised last-stage store of Sec. 5.1.2, coalesced
//     over the C rows).
//
// Addressing: a transaction's elements sit at a wave-uniform base plus r
// times a uniform stride plus a 32-bit lane offset, so directly addressed
// launches load (and store 8-byte elements) through raw buffer descriptors:
// one vector offset per lane, the strides in scalar registers.
//
// Two-side ABFT (Sec. 4.1-4.3), per slot and group of T transactions, e_k =
// w_M^k (M = 3, or 5 when 3 | Ns) and a = e^T W of the sub-length:
//   per transaction b: p_b = a^T x_b (input; each lane reads its E entries
//   of a with the inputs, from LDS where the workgroup stages a, else from
//   the cached table), q_b = e^T y_b (output, M bucket sums);
//   group close: D0 = sum q_b - sum p_b detects, D1 = sum (b+1)(q_b - p_b)
//   locates (location encoding), c = W x_s - Y e corrects the located
//   signal (delayed batched correction).  The right-side sums x_s = X e and
//   Y e are formed on the error path only, from the group's intact inputs
//   and stored outputs (in place, where the inputs are overwritten, x_s is
//   accumulated in registers during the group instead).
// Single-pass checking kernels with one signal per workgroup can run
// resident: as many workgroups as the device holds, e^T W staged in LDS
// once, a loop over the signal groups (kResident).
// In the row pass the left vector becomes a_n * w_N^{n k1} applied to the raw
// loaded values and x_s sums the raw values, so the inter-pass twiddle
// multiply is covered as well; all transactions of a row-pass group share
// the row k1 (they run over consecutive signals).
#pragma once

#include "tfft_device.hpp"

namespace tfft {

struct FtCounts {   // mirrors tfft_ft_counts in the public header
    unsigned long long detected, corrected, rebuilt, uncorrectable, last_signal;
    unsigned long long calib;          // calibration: max |D0| / tau (bits of a double)
    unsigned long long sched_errors;   // ragged launches whose waits gave up
    unsigned long long fallback;       // detections located by re-encoding the group
};

// kColPass3 / kRowPass3: the second and third pass of a three-pass
// transform N = N1 N2 N3 (M = N2 N3), see Geo.  Kind 3 labels the ragged
// persistent launches in the launch-timing log.
enum Kind { kSingle = 0, kColPass = 1, kRowPass = 2, kColPass3 = 4, kRowPass3 = 5 };

// Kernel arguments shared by all transform kernels.
// Per-call arguments: direction, scaling, counters and the injection hook.
template <class R> struct KCall {
    int conj_in;          // 1: conjugate loaded values (inverse direction, first pass)
    int conj_out;         // 1: conjugate stored values (inverse direction, last pass)
    R scale;              // applied to every stored value
    int stats;            // 1: record max |D0| / tau over groups (calibration)
    FtCounts* counts;     // device counters (ABFT only)
    long long inj_signal; // signal to corrupt (-1: none)
    long long inj_signal2;// a second signal hit the same way (-1: none)
    long long inj_elem;   // element index in this kernel's numbering (see Geo::inj_r)
    int inj_part;         // 0 real, 1 imaginary
    int inj_bit;          // bit to flip
    int inj_stage;        // radix stage after which the value is hit (the last: the output)
};

// Arguments of one launch (a plain launch passes them as its kernel argument;
// the persistent ragged kernel reads the per-class part from device memory).
template <class V> struct KArgs : KCall<typename RealOf<V>::type> {
    using R = typename RealOf<V>::type;
    const V* tw;          // stage twiddle tables of the sub-length, concatenated
    const V* left;        // e^T W of the sub-length (ABFT only)
    const V* thr_tab;     // thread-level ABFT: e^T W_R and e1^T W_R per radix (see ThreadGuard)
    const V* tw_hi;       // row pass: w_N^m = tw_hi[m >> tw_bits] * tw_lo[m & mask]
    const V* tw_lo;
    int tw_bits;
    long long batch;      // number of signals
    long long N;          // full transform length (signal stride in elements)
    int N1, N2;           // two-pass split, N = N1 * N2
    // Three-pass transforms (N = N1 N2 N3, M = N2 N3): column pass B runs
    // over rows of length M (a.N = M, a.N2 = N3) and multiplies element
    // n2 N3 + n3 of row k1 by w_N^{k1 (n2 N3 + n3)} at load (p3_n1 = N1,
    // full-length table in tw_hi / tw_lo); row pass C runs over (signal,
    // k2) pairs (p3_n2 = N2, p3_M = M, a.N = N, a.N1 = N1), multiplies by
    // w_M^{k2 n3} (tw_hi / tw_lo of length M) and writes k1 + N1 (k2 + N2 k3).
    int p3_n1, p3_n2;
    long long p3_M;
    int T;                // transactions (signals) per slot
    long long sig_base;   // global index of local signal 0 (counters only)
    R thr_ku;             // thread-level ABFT: kappa * u
    R tau_coef;           // kappa * u * sqrt(Ns s), s = log2 Ns (+ 3 with an inter-pass
                          // twiddle); tau = tau_coef * sqrt(nu)
    R cap;                // magnitude cap: larger outputs mark their signal corrupted
    int gran;             // detection granularity: 0 once per group of T transactions
                          // (location by D1/D0), 1 per transaction (note and continue)
    int x_intact;         // 1: inputs can be re-read on the error path
    int tiles;            // workgroups per signal group (tile geometries)
    long long nblk;       // workgroups' worth of work of the launch (resident
                          // kernels loop over it; others launch that many)
    // Indirection (ragged batches, kernels built with IND): element offset of
    // local signal s in x and in y, and its global index for counters and
    // injection.  Without IND, signal s starts at s * N and its global index
    // is sig_base + s.
    const long long* in_tab;
    const long long* out_tab;
    const long long* id_tab;
    // Left vector in cotangent form (single passes that read it from the
    // cached table): with w_M w_N^n = exp(-i theta_n),
    // a_n = c2 (1 - i cot(theta_n / 2)), c2 = (1 - w_M^N) / 2, so
    // p = c2 (sum_n x_n - i sum_n cot_n x_n) needs one real table value per
    // element.  cot holds them lane by lane in runs of 16 bytes: value (t, r)
    // at ((r / G) P + t) G + r % G, G = 16 / sizeof(R).
    const R* cot;
    V cot_c2;
};

// Compile-time plan: kind, sub-length Ns, E elements per lane, WC = waves per
// workgroup (single geometry) or sub-signals per workgroup (tile
// geometries), padded LDS row of 2^B elements (single geometry), stage
// radices Rs...
template <int KIND_, int Ns_, int E_, int WC_, int B_, int... Rs> struct Plan {
    static constexpr int KIND = KIND_;
    static constexpr int Ns = Ns_;
    static constexpr int E = E_;
    static constexpr int P = Ns / E;                           // lanes per slot
    static constexpr bool TILE = KIND != kSingle;
    static constexpr bool IS_COL = KIND == kColPass || KIND == kColPass3;
    static constexpr bool IS_ROW = KIND == kRowPass || KIND == kRowPass3;
    // a per-element twiddle at load, folded into the left vector
    static constexpr bool HAS_TW = KIND == kRowPass || KIND == kColPass3 || KIND == kRowPass3;
    static constexpr int C = TILE ? WC_ : 1;                    // sub-signals per tile
    static constexpr int THREADS = TILE ? P * C : (P > kWave ? P : WC_ * kWave);
    static constexpr bool MULTI_WAVE = THREADS > kWave && (TILE || P > kWave);
    static constexpr int WAVES = THREADS >= kWave ? THREADS / kWave : 1;
    static constexpr int SPW = (!TILE && P <= kWave) ? kWave / P : 1;   // slots per wave
    static constexpr int SLOTS = TILE ? C : (P > kWave ? 1 : WAVES * SPW);
    static constexpr int B = B_;
    // a single pass of more than one wave per signal with WC = 1: the
    // streaming form, which reads e^T W from the cached table instead of
    // staging it in LDS, so that two workgroups share a CU
    static constexpr bool STREAM = !TILE && P > kWave && WC_ == 1;
    static constexpr int LDS_DATA = TILE ? Ns * C : padded_size<B_>(P > kWave ? Ns : WAVES * SPW * Ns);
    static constexpr int M = (Ns % 3 == 0) ? 5 : 3;            // encoding period
    static_assert(Ns % E == 0, "E must divide Ns");
    static_assert(((Rs * ...) == Ns), "radices must multiply to Ns");
    static_assert(((E % Rs == 0) && ...), "every radix must divide E");
    static_assert(THREADS <= 1024, "workgroup too large");
    static_assert(!TILE || THREADS % kWave == 0, "tile workgroups are whole waves");
    static_assert(!TILE || (kWave % C == 0), "tile width divides a wave");
    static_assert(TILE || (P > kWave ? P % kWave == 0 : kWave % P == 0), "slot must tile waves");
    static_assert(TILE || Ns % (1 << B_) == 0, "slot regions start on a padding block");
};

// Conditional negation without a branch: XOR with a wave-uniform sign mask
// (a branch on the flag would make the loads of the values complete first).
__device__ __forceinline__ float xor_sign(float v, unsigned long long m) {
    return __uint_as_float(__float_as_uint(v) ^ (unsigned)(m >> 32));
}
__device__ __forceinline__ double xor_sign(double v, unsigned long long m) {
    return __longlong_as_double(__double_as_longlong(v) ^ (long long)m);
}
// the sign bit of a double, whose high word is that of a float
__device__ __forceinline__ unsigned long long sign_mask(int on) { return on ? 0x8000000000000000ull : 0ull; }

// Bit flip of one component (fault injection, Sec. 5.3 protocol).
__device__ __forceinline__ float flip_bit(float v, int bit) {
    return __uint_as_float(__float_as_uint(v) ^ (1u << bit));
}
__device__ __forceinline__ double flip_bit(double v, int bit) {
    return __longlong_as_double(__double_as_longlong(v) ^ (1ll << bit));
}

// ---------------------------------------------------------------------------
// LDS index maps.
// ---------------------------------------------------------------------------
constexpr bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

// step(d) is the index distance from position m to m + d when no block
// boundary of the map falls between them other than those d itself crosses;
// SPLIT<L, R> says that this holds for the positions base + j L (j < R) of
// every Stockham butterfly and for t + P r (t < P, P = L) of every lane, so
// that one index per butterfly (or lane) plus immediate offsets addresses
// them all.
template <int B> struct LdsPad {   // one signal per region, one pad element per 2^B
    int off;                       // region start, a multiple of 2^B
    __device__ __forceinline__ int operator()(int m) const { return pad_idx<B>(off + m); }
    static __device__ __forceinline__ constexpr int step(int d) { return d + (d >> B); }
    // Powers of two L, R: a butterfly's positions lie in one aligned block of
    // L R positions plus an offset k < L, so base mod 2^B and j L mod 2^B
    // never add up past 2^B (and likewise t + P r with t < P).
    template <int L, int R> static constexpr bool SPLIT = pow2(L) && pow2(R);
};
template <int C> struct LdsCol {    // tile [m][c]: C sub-signals interleaved
    int c;
    __device__ __forceinline__ int operator()(int m) const { return m * C + c; }
    static __device__ __forceinline__ constexpr int step(int d) { return d * C; }
    template <int L, int R> static constexpr bool SPLIT = true;
};

// ---------------------------------------------------------------------------
// One Stockham stage.  LAST: results stay in registers (output layout),
// otherwise they go to LDS at their autosorted positions.
// ---------------------------------------------------------------------------
// BF guards each radix-R DFT of the stage (thread-level ABFT; NoGuard: none).
struct NoGuard {
    template <int R, class V> __device__ __forceinline__ void before(const V (&)[R]) {}
    template <int R, class V> __device__ __forceinline__ void after(V (&)[R], int, int) {}
};
template <class V, int E, int P, int R, int L, bool LAST, int S, class LI, class BF>
__device__ __forceinline__ void stockham_stage(V (&reg)[E], const V* __restrict__ tw_s, int t,
                                               V* __restrict__ lds, const LI& li, BF& bf) {
    constexpr int NB = E / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        // unsigned: t is never negative, and L is a power of two on most
        // stages, where % and / are then a mask and a shift
        const unsigned beta = (unsigned)t + (unsigned)(i * P);
        const int k = (int)(beta % (unsigned)L);
        V v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = reg[i + j * NB];
        if constexpr (L > 1) {
            const V* w = tw_s + k * R;
#pragma unroll
            for (int j = 1; j < R; ++j) v[j] = cmul(v[j], w[j]);
        }
        bf.template before<R>(v);
        dft<R>(v);
        bf.template after<R>(v, S, i);
        if constexpr (LAST) {
#pragma unroll
            for (int j = 0; j < R; ++j) reg[i + j * NB] = v[j];
        } else {
            const int base = (int)(beta / (unsigned)L) * (L * R) + k;
            if constexpr (LI::template SPLIT<L, R>) {
                V* const at = lds + li(base);
#pragma unroll
                for (int j = 0; j < R; ++j) at[LI::step(j * L)] = v[j];
            } else {
#pragma unroll
                for (int j = 0; j < R; ++j) lds[li(base + j * L)] = v[j];
            }
        }
    }
}

// All stages of one in-slot FFT.  reg holds elements t + P*r on entry and the
// transform's outputs t + P*r on exit.  Stage s's table holds L_s * R_s
// entries and the tables follow each other.  hook(s, reg) runs after stage s
// (S counts the stages), on the values t + P*r of the intermediate sequence
// the stage produced (the fault-injection point; a no-op outside tests).
struct NoHook {
    template <class A> __device__ __forceinline__ void operator()(int, A&) const {}
};
template <class V, int E, int P, bool BLOCK, class LI, class H, class BF, int S, int L, int R, int... Rest>
__device__ __forceinline__ void slot_fft(V (&reg)[E], const V* __restrict__ tw, int t,
                                         V* __restrict__ lds, const LI& li, H& hook, BF& bf) {
    constexpr bool LAST = sizeof...(Rest) == 0;
    stockham_stage<V, E, P, R, L, LAST, S>(reg, tw, t, lds, li, bf);
    if constexpr (!LAST) {
        lds_sync<BLOCK>();
        if constexpr (LI::template SPLIT<P, 1>) {
            const V* const at = lds + li(t);
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r] = at[LI::step(P * r)];
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r] = lds[li(t + P * r)];
        }
        lds_sync<BLOCK>();
        hook(S, reg);
        slot_fft<V, E, P, BLOCK, LI, H, BF, S + 1, L * R, Rest...>(reg, tw + L * R, t, lds, li, hook, bf);
    } else {
        hook(S, reg);
    }
}

// w_M^j for the encoding vector e_k = w_M^k, w_M = exp(-2 pi i / M)
template <class V, int M> __device__ __forceinline__ V wM(int j) {
    using R = typename RealOf<V>::type;
    j %= M;
    if constexpr (M == 3) {
        if (j == 0) return V{(R)1, (R)0};
        if (j == 1) return V{(R)-0.5, (R)(-TFFT_SQRT3_2)};
        return V{(R)-0.5, (R)TFFT_SQRT3_2};
    } else {
        // cos/sin of 2 pi j / 5
        const R c1 = (R)0.30901699437494742410229341718281905886436044959939;
        const R s1 = (R)0.95105651629515357211643933337938214340569863846464;
        const R c2 = (R)-0.80901699437494742410229341718281905886436044959939;
        const R s2 = (R)0.58778525229247312916870595463907276859765243764315;
        switch (j) {
            case 0: return V{(R)1, (R)0};
            case 1: return V{c1, -s1};
            case 2: return V{c2, -s2};
            case 3: return V{c2, s2};
            default: return V{c1, s1};
        }
    }
}

// Thread-level two-side ABFT (Sec. 4.2, thread level): every radix-R DFT a
// lane computes in registers is checked on its own.  Before it, p = a^T v
// and p1 = a1^T v with a = e^T W_R and a1 = e1^T W_R (e_k = w_3^k,
// e1_k = (k + 1) w_3^k; host table, radix R at offset 2 (R - 2), a then a1)
// and nu = |v|^2; after it, q = e^T v and q1 = e1^T v.  |q - p| above
// kappa u sqrt(R (log2 R + 3)) sqrt(nu) flags the DFT; its faulty output
// k* = round(Re((q1 - p1) / (q - p))) - 1 is repaired by subtracting
// (q - p) / e_{k*}; a difference beyond 32 |v| (or not finite) marks the
// largest output, which is rebuilt from the left checksum
// (e_{k*} y_{k*} = p - the others).  The test hook flips output j of the first DFT of one
// lane at one stage, between the DFT and its check.
template <class V> struct ThreadGuard {
    using R = typename RealOf<V>::type;
    const V* tab;
    R kappa_u;
    FtCounts* counts;
    int inj_stage, inj_j, inj_part, inj_bit;   // inj_stage < 0: no flip in this lane
    long long sig;
    V p, p1;
    R nu;
    template <int RR> __device__ __forceinline__ void before(const V (&v)[RR]) {
        const V* a = tab + 2 * (RR - 2);
        p = V{0, 0};
        p1 = V{0, 0};
        nu = 0;
#pragma unroll
        for (int j = 0; j < RR; ++j) {
            p = cmac(p, a[j], v[j]);
            p1 = cmac(p1, a[RR + j], v[j]);
            nu = fmad(v[j].x, v[j].x, fmad(v[j].y, v[j].y, nu));
        }
    }
    template <int RR> __device__ __forceinline__ void after(V (&v)[RR], int stage, int i) {
        if (inj_stage == stage && i == 0) {
#pragma unroll
            for (int j = 0; j < RR; ++j)
                if (j == inj_j % RR) {
                    if (inj_part == 0) v[j].x = flip_bit(v[j].x, inj_bit);
                    else v[j].y = flip_bit(v[j].y, inj_bit);
                }
        }
        V q = V{0, 0}, q1 = V{0, 0};
#pragma unroll
        for (int k = 0; k < RR; ++k) {
            const V ek = wM<V, 3>(k);
            const V t = cmul(ek, v[k]);
            q = cadd(q, t);
            q1 = V{fmad((R)(k + 1), t.x, q1.x), fmad((R)(k + 1), t.y, q1.y)};
        }
        // rounding steps: log2 R for the DFT, three for the checksum products
        constexpr int LG = RR == 2 ? 1 : RR == 4 ? 2 : RR == 8 ? 3 : 4;
        const R tau = kappa_u * (R)__builtin_sqrt((R)(RR * (LG + 3))) * __builtin_sqrt(nu);
        const V d = csub(q, p);
        // |d| scaled by its larger component, so that a large finite
        // difference does not overflow to infinity
        const R ax = __builtin_fabs(d.x), ay = __builtin_fabs(d.y);
        const bool fin = ax < (R)INFINITY && ay < (R)INFINITY;
        const R m = ax > ay ? ax : ay;
        R d0 = (R)INFINITY;
        if (fin) d0 = m > (R)0 ? m * __builtin_sqrt((d.x / m) * (d.x / m) + (d.y / m) * (d.y / m)) : (R)0;
        if (!(d0 <= tau)) {
            // locate: Re(d1 / d) = Re(d1 conj(d / |d|)) / |d|; a non-finite
            // difference: the non-finite output, else the largest one
            const V d1 = csub(q1, p1);
            int ks = -1;
            // An error up to a few times the DFT's inputs is subtracted (its
            // rounding stays at the data's scale); a larger or non-finite one
            // would leave its own rounding behind: the largest output, which
            // carries it, is rebuilt instead.
            if (fin && d0 <= (R)32 * __builtin_sqrt(nu)) {
                const R re = (d1.x * (d.x / d0) + d1.y * (d.y / d0)) / d0;
                if (re == re && re > (R)0.5 && re < (R)RR + (R)0.5) ks = (int)__builtin_floor(re + (R)0.5) - 1;
            }
            const bool add = ks >= 0;
            if (!add) {
                // a NaN counts as the largest (and stays chosen)
                R big = (R)-1;
#pragma unroll
                for (int k = 0; k < RR; ++k) {
                    R mk = __builtin_fabs(v[k].x) + __builtin_fabs(v[k].y);
                    if (!(mk < (R)INFINITY)) mk = (R)INFINITY;
                    if (mk > big) {
                        big = mk;
                        ks = k;
                    }
                }
            }
            bool ok = false;
#pragma unroll
            for (int k = 0; k < RR; ++k)
                if (k == ks) {
                    const V ek = wM<V, 3>(k);
                    if (add) {
                        // v_k -= d / e_k = d conj(e_k)  (|e_k| = 1)
                        v[k] = csub(v[k], cmul(d, V{ek.x, -ek.y}));
                    } else {
                        // rebuild from the left checksum: e_k v_k = p - sum of the others
                        V o = p;
#pragma unroll
                        for (int m = 0; m < RR; ++m)
                            if (m != k) o = csub(o, cmul(wM<V, 3>(m), v[m]));
                        v[k] = cmul(o, V{ek.x, -ek.y});
                    }
                    ok = true;
                }
            atomicAdd(&counts->detected, 1ull);
            atomicAdd(!ok ? &counts->uncorrectable : (add ? &counts->corrected : &counts->rebuilt), 1ull);
            atomicExch(&counts->last_signal, (unsigned long long)sig);
        }
    }
};

// sum_r w_M^{(P r) mod M} v[r]: e^T v for a lane whose positions are t + P r,
// up to the lane factor w_M^{t mod M} applied by the caller.
template <class V, int E, int P, int M> __device__ __forceinline__ V encode_out(const V (&v)[E]) {
    V bucket[M];
#pragma unroll
    for (int m = 0; m < M; ++m) bucket[m] = V{0, 0};
#pragma unroll
    for (int r = 0; r < E; ++r) bucket[(P * r) % M] = cadd(bucket[(P * r) % M], v[r]);
    V acc = bucket[0];
#pragma unroll
    for (int m = 1; m < M; ++m) acc = cmac(acc, bucket[m], wM<V, M>(m));
    return acc;
}

template <class R> __device__ __forceinline__ bool cfin(R x, R y, R cap) {
    return finite_le(x, cap) && finite_le(y, cap);
}

// ---------------------------------------------------------------------------
// Geometry: lane -> (slot, t), addressing, reductions over a slot.
// ---------------------------------------------------------------------------
template <class V, class PL, bool IND> struct Geo {
    using R = typename RealOf<V>::type;
    static constexpr int E = PL::E, P = PL::P, Ns = PL::Ns, C = PL::C;
    static constexpr bool BLOCK = PL::MULTI_WAVE;
    int t;               // position in the slot
    int slot;            // slot within the workgroup (column / row of a tile)
    long long sig0;      // signal of transaction 0
    long long sig_step;  // signal stride between transactions
    int line;            // tiles: column n2 (pass A) or row k1 (pass B)
    int lds_off;         // single: start of the slot's LDS region
    int par = 0;         // which half of the reduction scratch the next reduce uses
    int tid;             // lane in the workgroup
    int tile = 0;        // tiles: tile index within the signal group
    long long sig_u0;    // wave-uniform signal of transaction 0 (slot 0 of the wave)
    unsigned lane_in;    // this lane's element offset within a transaction's input
    unsigned lane_out;   // and within its output
    V tw_base{(R)1, (R)0};       // passes with a twiddle: this lane's w^{k (b + D t)}
    const V* tw_step = nullptr;  // and the LDS table of the steps w^{k D P r}

    __device__ __forceinline__ Geo(const KArgs<V>& a, long long block, long long nblocks, int tid_)
        : tid(tid_) {
        if constexpr (PL::KIND == kSingle) {
            const int lane = tid % kWave, wave = tid / kWave;
            if constexpr (P > kWave) {
                t = tid;
                slot = 0;
                lds_off = 0;
                if constexpr (IND) {
                    sig0 = block * a.T;
                    sig_step = 1;
                } else {
                    sig0 = block;
                    sig_step = nblocks;
                }
                sig_u0 = sig0;
                lane_in = (unsigned)t;
            } else {
                const int sigma = lane / P;
                t = lane % P;
                slot = wave * PL::SPW + sigma;
                lds_off = slot * Ns;
                const long long wave_u = __builtin_amdgcn_readfirstlane(wave);
                if constexpr (IND) {
                    sig_u0 = (block * PL::WAVES + wave_u) * a.T * PL::SPW;
                    sig_step = PL::SPW;
                } else {
                    sig_u0 = (block * PL::WAVES + wave_u) * PL::SPW;
                    sig_step = nblocks * PL::WAVES * PL::SPW;
                }
                sig0 = sig_u0 + sigma;
                lane_in = (unsigned)sigma * (unsigned)a.N + (unsigned)t;
            }
            lane_out = lane_in;
            line = 0;
        } else {
            t = tid / C;
            slot = tid % C;
            lds_off = 0;
            // workgroups are dealt round-robin to the 8 XCDs; renumber them so
            // each XCD (and its L2) walks a contiguous range of tiles, where
            // neighbouring tiles share cache lines
            long long bid = block;
            const long long G = nblocks;
            if (!IND && (G & 7) == 0) bid = (bid & 7) * (G >> 3) + (bid >> 3);
            const long long tl = bid % a.tiles;   // tiles of one signal group are consecutive
            const long long grp = bid / a.tiles;
            tile = (int)tl;
            line = (int)(tl * C + slot);
            if constexpr (IND) {
                sig0 = grp * a.T;
                sig_step = 1;
            } else {
                sig0 = grp;
                sig_step = G / a.tiles;   // signal groups in the launch
            }
            sig_u0 = sig0;
            if constexpr (PL::IS_COL) {
                lane_in = (unsigned)t * (unsigned)a.N2 + (unsigned)slot;
                lane_out = lane_in;
            } else if constexpr (PL::KIND == kRowPass) {
                lane_in = (unsigned)slot * (unsigned)a.N2 + (unsigned)t;
                lane_out = (unsigned)slot + (unsigned)a.N1 * (unsigned)t;
            } else {   // kRowPass3: rows k1 at stride M, outputs k1 + N1 N2 k3
                lane_in = (unsigned)slot * (unsigned)a.p3_M + (unsigned)t;
                lane_out = (unsigned)slot + (unsigned)a.N1 * (unsigned)a.p3_n2 * (unsigned)t;
            }
        }
    }
    // Transaction b's elements t + P r sit at a wave-uniform element offset
    // (in_uni / out_uni) plus r times a uniform stride (in_step / out_step)
    // plus this lane's 32-bit offset (lane_in / lane_out): loads and stores
    // then take a scalar base and one vector offset shared by all E elements.
    // Lane offsets stay below 2^32 bytes: at most a tile's span of a signal.
    // three-pass row pass: signal s is the pair (b, k2) = (s / N2, s % N2);
    // its row k1 starts at b N + k2 N3 + k1 M, its outputs at b N + k2 N1 + k1
    __device__ __forceinline__ static long long p3_in_base(const KArgs<V>& a, long long s) {
        return (s / a.p3_n2) * a.N + (s % a.p3_n2) * (long long)Ns;
    }
    __device__ __forceinline__ static long long p3_out_base(const KArgs<V>& a, long long s) {
        return (s / a.p3_n2) * a.N + (s % a.p3_n2) * (long long)a.N1;
    }
    __device__ __forceinline__ long long in_uni(const KArgs<V>& a, int b) const {
        const long long su = sig_u0 + (long long)b * sig_step;
        if constexpr (PL::KIND == kSingle) return su * a.N;
        else if constexpr (PL::IS_COL) return su * a.N + (long long)tile * C;
        else if constexpr (PL::KIND == kRowPass) return su * a.N + (long long)tile * C * a.N2;
        else return p3_in_base(a, su) + (long long)tile * C * a.p3_M;
    }
    __device__ __forceinline__ long long out_uni(const KArgs<V>& a, int b) const {
        const long long su = sig_u0 + (long long)b * sig_step;
        if constexpr (PL::KIND == kSingle) return su * a.N;
        else if constexpr (PL::KIND == kRowPass3) return p3_out_base(a, su) + (long long)tile * C;
        else return su * a.N + (long long)tile * C;
    }
    __device__ __forceinline__ long long in_step(const KArgs<V>& a) const {
        if constexpr (PL::IS_COL) return (long long)P * a.N2;
        else return P;
    }
    __device__ __forceinline__ long long out_step(const KArgs<V>& a) const {
        if constexpr (PL::KIND == kSingle) return P;
        else if constexpr (PL::IS_COL) return (long long)P * a.N2;
        else if constexpr (PL::KIND == kRowPass) return (long long)P * a.N1;
        else return (long long)P * a.N1 * a.p3_n2;
    }
    __device__ __forceinline__ long long sig(int b) const { return sig0 + (long long)b * sig_step; }
    // element offsets of input element m / output element k of signal s
    __device__ __forceinline__ long long in_base(const KArgs<V>& a, long long s) const {
        if constexpr (IND) return a.in_tab[s];
        else if constexpr (PL::KIND == kRowPass3) return p3_in_base(a, s);
        else return s * a.N;
    }
    __device__ __forceinline__ long long out_base(const KArgs<V>& a, long long s) const {
        if constexpr (IND) return a.out_tab[s];
        else if constexpr (PL::KIND == kRowPass3) return p3_out_base(a, s);
        else return s * a.N;
    }
    __device__ __forceinline__ long long gid(const KArgs<V>& a, long long s) const {
        if constexpr (IND) return a.id_tab[s];
        else return a.sig_base + s;
    }
    // the caller's signal a fault of local signal s is reported against: the
    // passes of a three-pass transform number rows (b, k1) or pairs (b, k2)
    __device__ __forceinline__ long long rid(const KArgs<V>& a, long long s) const {
        if constexpr (PL::KIND == kColPass3) return gid(a, s) / a.p3_n1;
        else if constexpr (PL::KIND == kRowPass3) return gid(a, s) / a.p3_n2;
        else return gid(a, s);
    }
    __device__ __forceinline__ long long in_off(const KArgs<V>& a, long long s, int m) const {
        if constexpr (PL::KIND == kSingle) return in_base(a, s) + m;
        else if constexpr (PL::IS_COL) return in_base(a, s) + (long long)m * a.N2 + line;
        else if constexpr (PL::KIND == kRowPass) return in_base(a, s) + (long long)line * a.N2 + m;
        else return in_base(a, s) + (long long)line * a.p3_M + m;
    }
    __device__ __forceinline__ long long out_off(const KArgs<V>& a, long long s, int k) const {
        if constexpr (PL::KIND == kSingle) return out_base(a, s) + k;
        else if constexpr (PL::IS_COL) return out_base(a, s) + (long long)k * a.N2 + line;
        else if constexpr (PL::KIND == kRowPass) return out_base(a, s) + line + (long long)a.N1 * k;
        else return out_base(a, s) + line + (long long)a.N1 * a.p3_n2 * k;
    }
    // which of this lane's values t + P r is the injected one: r, or -1 (test
    // hook).  inj_elem numbers a value of position k of a sub-sequence as k
    // (single pass), k N2 + n2 (column n2 of a column pass) or n1 + N1 k
    // (row n1 of a row pass), the layouts the passes store; k is the
    // position in the sequence the chosen stage produces.
    __device__ __forceinline__ int inj_r(const KArgs<V>& a, const KCall<typename RealOf<V>::type>& kc) const {
        long long k = -1;   // index of the target in this slot's numbering
        if constexpr (PL::KIND == kSingle) {
            k = kc.inj_elem;
        } else if constexpr (PL::IS_COL) {
            if (kc.inj_elem % a.N2 == line) k = kc.inj_elem / a.N2;
        } else {
            if (kc.inj_elem % a.N1 == line) k = kc.inj_elem / a.N1;
        }
        if (k < t || k >= Ns || (k - t) % P != 0) return -1;
        return (int)((k - t) / P);
    }
    __device__ __forceinline__ auto lidx() const {
        if constexpr (PL::KIND == kSingle) return LdsPad<PL::B>{lds_off};
        else return LdsCol<C>{slot};
    }
    // row pass: w_N^{n k1} for sub-signal element n (two table values, one product)
    // w_N^m from the two-level table (m < N)
    __device__ __forceinline__ static V twiddle_at(const KArgs<V>& a, unsigned m) {
        const V hi = a.tw_hi[m >> a.tw_bits];
        const V lo = a.tw_lo[m & ((1u << a.tw_bits) - 1u)];
        return cmul(hi, lo);
    }
    // Row pass: build w_N^{P r k1} for the C rows k1 of this tile and r < E
    // in LDS (shared by every lane of a row), and this lane's w_N^{t k1}.
    // The inter-pass twiddle of element t + P r is then their product: one
    // LDS read and one multiply instead of two table gathers per element.
    __device__ __forceinline__ void twiddle_setup(const KArgs<V>& a, V* steps) {
        if constexpr (PL::KIND == kRowPass) {
            for (int i = tid; i < C * E; i += PL::THREADS) {
                const int c = i / E, r = i % E;
                const unsigned k1 = (unsigned)(tile * C + c);
                steps[i] = twiddle_at(a, (unsigned)P * (unsigned)r * k1);   // P r k1 < N
            }
            tw_base = twiddle_at(a, (unsigned)t * (unsigned)line);          // t k1 < N
            tw_step = steps;
        } else if constexpr (PL::KIND == kColPass3 || PL::KIND == kRowPass3) {
            // Three-pass passes run one signal per workgroup (groups of one
            // transaction), whose k (k1 = s mod N1 or k2 = s mod N2) every
            // lane shares: w^{k (b + D t)} w^{k D P r} with D = N3 (pass 1,
            // b = n3 = line, table of N) or D = 1 (pass 2, b = 0, table of M);
            // both exponents stay below the table's length.
            constexpr bool P1 = PL::KIND == kColPass3;
            const unsigned k = (unsigned)(sig0 % (P1 ? a.p3_n1 : a.p3_n2));
            const unsigned D = P1 ? (unsigned)a.N2 : 1u;
            for (int i = tid; i < E; i += PL::THREADS) steps[i] = twiddle_at(a, k * D * (unsigned)P * (unsigned)i);
            tw_base = twiddle_at(a, k * ((P1 ? (unsigned)line : 0u) + D * (unsigned)t));
            tw_step = steps;
        }
    }
    // inter-pass twiddle of element t + P r of local signal s (1 where a
    // pass has none); the LDS steps must be visible (barrier after
    // twiddle_setup).  A three-pass pass's steps belong to the workgroup's
    // one signal: s is that signal.
    __device__ __forceinline__ V twiddle(const KArgs<V>& a, long long s, int r) const {
        (void)a;
        (void)s;
        if constexpr (PL::KIND == kRowPass) {
            return cmul(tw_base, tw_step[slot * E + r]);
        } else if constexpr (PL::KIND == kColPass3 || PL::KIND == kRowPass3) {
            return cmul(tw_base, tw_step[r]);
        } else {
            return V{(R)1, (R)0};
        }
    }

    // reduce K values over the slot with Op; the result is bit-identical on
    // every lane of the slot (XOR butterflies, then one ordered pass over the
    // per-wave partials in LDS).  scratch holds 2 * K * WAVES * C values of T.
    template <class Op, int K, class T> __device__ __forceinline__ void reduce(T (&v)[K], T* scratch) {
        if constexpr (PL::KIND == kSingle) {
            constexpr int W = P < kWave ? P : kWave;
#pragma unroll
            for (int i = 0; i < K; ++i) v[i] = xor_reduce<1, W, Op>(v[i]);
            if constexpr (P > kWave) {
                // two alternating halves: a half is rewritten only after the
                // barrier of the next reduction, when all its readers are done
                const int wave = tid / kWave, lane = tid % kWave;
                T* sc = scratch + par * (K * PL::WAVES);
                par ^= 1;
                if (lane == 0) {
#pragma unroll
                    for (int i = 0; i < K; ++i) sc[i * PL::WAVES + wave] = v[i];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    T s = sc[i * PL::WAVES];
#pragma unroll
                    for (int w = 1; w < PL::WAVES; ++w) s = Op::f(s, sc[i * PL::WAVES + w]);
                    v[i] = s;
                }
            }
        } else {
            // lanes t*C + c: XOR over the t bits inside a wave, then across waves
            constexpr int TW = (kWave / C) < P ? (kWave / C) : P;   // t values per wave
#pragma unroll
            for (int i = 0; i < K; ++i) v[i] = xor_reduce<C, C * TW, Op>(v[i]);
            if constexpr (PL::MULTI_WAVE) {
                const int wave = tid / kWave, lane = tid % kWave;
                T* sc = scratch + par * (K * PL::WAVES * C);
                par ^= 1;
                if (lane < C) {
#pragma unroll
                    for (int i = 0; i < K; ++i) sc[(i * PL::WAVES + wave) * C + lane] = v[i];
                }
                __syncthreads();
#pragma unroll
                for (int i = 0; i < K; ++i) {
                    T s = sc[(i * PL::WAVES) * C + slot];
#pragma unroll
                    for (int w = 1; w < PL::WAVES; ++w) s = Op::f(s, sc[(i * PL::WAVES + w) * C + slot]);
                    v[i] = s;
                }
            }
        }
    }
    // any lane of the synchronisation domain (wave or workgroup), for flags
    // that are identical on every lane of a slot (decisions taken from
    // reduced values).  A workgroup that synchronises as a whole holds one
    // slot, or tiles whose waves each carry lanes of every slot, so every
    // wave sees every slot's flag and its own vote is the workgroup's: no
    // barrier is needed, and all waves take the same branch.
    __device__ __forceinline__ bool domain_any(bool f) const {
        static_assert(!BLOCK || PL::SLOTS == 1 || PL::TILE, "a wave must see every slot of its workgroup");
        return __any(f ? 1 : 0) != 0;
    }

    // ---- per-transaction checking ----
    // The lanes of a slot that share a wave (TXW of them) reduce a
    // transaction's values with cross-lane exchanges; lane tx_tl() == b of
    // that wave part keeps transaction b's partial, so a group of up to
    // TX_MAX transactions leaves one partial per lane and no array indexed
    // by b.  Slots spanning TX_PARTS waves add the parts through LDS once
    // per group.
    static constexpr bool SINGLE = PL::KIND == kSingle;
    static constexpr int TXW = SINGLE ? (P < kWave ? P : kWave) : kWave / C;
    static constexpr int TX_MAX = TXW < 16 ? TXW : 16;
    static constexpr int TX_PARTS = SINGLE ? (P > kWave ? P / kWave : 1) : (PL::MULTI_WAVE ? PL::WAVES : 1);
    __device__ __forceinline__ int tx_tl() const {
        if constexpr (SINGLE) return P > kWave ? tid % kWave : t;
        else return (tid % kWave) / C;
    }
    // lane of this wave holding transaction b's values for this slot
    __device__ __forceinline__ int tx_lane(int b) const {
        if constexpr (SINGLE) return P > kWave ? b : (tid % kWave) - t + b;
        else return b * C + slot;
    }
    template <class T> __device__ __forceinline__ T tx_wave_sum(T v) const {
        if constexpr (SINGLE) return xor_reduce<1, TXW, OpAdd>(v);
        else return xor_reduce<C, kWave, OpAdd>(v);
    }
    // add the wave parts of the kept partials (K values per lane): every
    // lane tx_tl() < T of every wave ends with the slot's totals, summed in
    // the same order everywhere
    template <int K, class T> __device__ __forceinline__ void tx_parts_sum(T (&v)[K], int T_, T* txr) const {
        if constexpr (TX_PARTS > 1) {
            const int tl = tx_tl();
            const int part = tid / kWave;   // wave = part of the slot
            auto at = [&](int k, int pr) -> T* {
                return txr + (((k * TX_MAX + tl) * TX_PARTS + pr) * C + (SINGLE ? 0 : slot));
            };
            const bool mine = tl < T_ && tl < TX_MAX;
            if (mine) {
#pragma unroll
                for (int k = 0; k < K; ++k) *at(k, part) = v[k];
            }
            __syncthreads();
            if (mine) {
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    T acc = *at(k, 0);
#pragma unroll
                    for (int pr = 1; pr < TX_PARTS; ++pr) acc = acc + *at(k, pr);
                    v[k] = acc;
                }
            }
            // the space may be the exchange buffer, which the next group
            // writes next
            __syncthreads();
        }
    }
    // bit b set when lane tx_lane(b) of this wave has f set (b < T_)
    __device__ __forceinline__ unsigned tx_mask(bool f, int T_) const {
        const unsigned long long bal = __ballot(f ? 1 : 0);
        if constexpr (SINGLE) {
            const int first = P > kWave ? 0 : (tid % kWave) - t;
            return (unsigned)(bal >> first) & (T_ >= 32 ? 0xffffffffu : ((1u << T_) - 1u));
        } else {
            unsigned m = 0;
            for (int b = 0; b < T_; ++b) m |= (unsigned)((bal >> (b * C + slot)) & 1ull) << b;
            return m;
        }
    }
};

// ---------------------------------------------------------------------------
// The transform kernel.  FT: 0 off, 1 detect (one-side check with location),
// 2 correct (two-side check, location and delayed batched correction; the
// right-side input sum is formed again from the intact inputs on the error
// path), 3 correct in place (the right-side input sum X e stays in registers
// through the group, because the outputs overwrite the inputs).
// ---------------------------------------------------------------------------
// Resident checking kernels: single-pass plans whose workgroup holds one
// signal per transaction read all Ns entries of e^T W per signal, as many
// bytes again as the signal itself.  Their workgroups stay resident instead,
// stage e^T W in LDS once and loop over signal groups (directly addressed
// launches only; the ragged kernel has its own persistent loop).  The loop
// costs the kernel 12-26 more registers, which loses an occupancy step on
// some plans: residency is kept where it measured faster (complex float:
// 8 elements per lane, or 8192 points and up; complex double: 4096 points
// and up).
template <class V, class PL, int FT, bool IND> constexpr bool kResident =
    FT != 0 && !IND && PL::KIND == kSingle && PL::SLOTS == 1 && !PL::STREAM &&
    (sizeof(V) == 8 ? (PL::E == 8 || PL::Ns >= 8192) : PL::Ns >= 4096);

// LDS of one workgroup of a plan: exchange buffer, then reduction scratch
template <class V, class PL, int FT, bool IND = false> struct Smem {
    using R = typename RealOf<V>::type;
    static constexpr int NRED = 6;
    static constexpr int RED = FT ? 2 * (PL::TILE ? PL::C : 1) * PL::WAVES * NRED : 1;
    // row pass: the C x E inter-pass twiddle steps of the workgroup's rows;
    // three-pass passes: the E steps of the workgroup's one signal
    static constexpr int TWS = PL::KIND == kRowPass ? PL::C * PL::E : (PL::HAS_TW ? PL::E : 0);
    // per-transaction checking: wave parts of the kept partials (3 values)
    using G = Geo<V, PL, IND>;
    static constexpr int TXR = (FT != 0 && G::TX_PARTS > 1) ? 3 * G::TX_MAX * G::TX_PARTS * (PL::TILE ? PL::C : 1) : 0;
    // The kept partials are exchanged at the end of a group, when the
    // exchange buffer is idle (the last exchange of the group's last
    // transaction has passed its closing barrier, and a barrier follows the
    // partials' reads): they share its space, so per-transaction checking
    // costs no LDS.  (Single precision only: the double-precision tiles,
    // which check per group by default, keep their measured occupancy.)
    static constexpr bool TXR_ALIAS = sizeof(R) == 4 && TXR * (int)sizeof(R) <= PL::LDS_DATA * (int)sizeof(V);
    static constexpr int REST = PL::LDS_DATA * (int)sizeof(V) + TWS * (int)sizeof(V) +
                                (RED + (TXR_ALIAS ? 0 : TXR)) * (int)sizeof(R);
    // ABFT: the left vector e^T W staged once per workgroup where several
    // signals share it and it is small (column tiles; single-pass groups of
    // up to 2048 points); row passes keep reading the cached table, which
    // costs them no registers and saves the staging
    // (and only where it costs no workgroup per CU: a column tile of 1024 or
    // 2048 points would otherwise drop from two to one; resident kernels
    // always stage it)
    static constexpr int CU_LDS = 160 * 1024;
    static constexpr int WG_CAP = PL::WAVES >= 16 ? 1 : 16 / PL::WAVES;   // four waves per SIMD
    static constexpr int wg_fit(int bytes) { return CU_LDS / bytes < WG_CAP ? CU_LDS / bytes : WG_CAP; }
    static constexpr bool AW_FITS = wg_fit(REST + PL::Ns * (int)sizeof(V)) == wg_fit(REST);
    static constexpr bool AW_LDS =
        FT != 0 && (kResident<V, PL, FT, IND> ||
                    ((PL::TILE || (PL::KIND == kSingle && PL::SLOTS >= 2 && PL::Ns <= 2048)) && AW_FITS));
    static constexpr int AW = AW_LDS ? PL::Ns : 0;
    static constexpr int TWS_OFF = PL::LDS_DATA * (int)sizeof(V);
    static constexpr int AW_OFF = TWS_OFF + TWS * (int)sizeof(V);
    static constexpr int RED_OFF = AW_OFF + AW * (int)sizeof(V);
    static constexpr int TXR_OFF = TXR_ALIAS ? 0 : RED_OFF + RED * (int)sizeof(R);
    static constexpr int BYTES = RED_OFF + RED * (int)sizeof(R) + (TXR_ALIAS ? 0 : TXR * (int)sizeof(R));
};

// Single passes that read e^T W from the cached table (not staged in LDS)
// read it in its cotangent form (KArgs::cot): half the bytes, and one 16-byte
// load per 4 (fp32) or 2 (fp64) elements instead of one load per element.
template <class V, class PL, int FT, bool IND> constexpr bool kCotLeft =
    FT != 0 && !IND && PL::KIND == kSingle && !Smem<V, PL, FT, IND>::AW_LDS;

// Buffers that other workgroups of the same launch read back (the persistent
// ragged kernel's workspace) are accessed coherently at device scope: each
// XCD has its own L2, and a plain store may sit there unseen by the others.
// COH bit 0: stores to y (and reads of y back) are coherent; bit 1: loads
// from x are coherent.  Relaxed device-scope atomics give exactly that per
// access, without whole-cache write-back or invalidation.
template <class V> __device__ __forceinline__ V ld_coh(const V* p) {
    static_assert(sizeof(V) % 8 == 0, "complex elements are whole 8-byte words");
    unsigned long long w[sizeof(V) / 8];
    unsigned long long* q = reinterpret_cast<unsigned long long*>(const_cast<V*>(p));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(V) / 8); ++i)
        w[i] = __hip_atomic_load(q + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    V v;
    __builtin_memcpy(&v, w, sizeof(V));
    return v;
}
template <class V> __device__ __forceinline__ void st_coh(V* p, const V& v) {
    unsigned long long w[sizeof(V) / 8];
    __builtin_memcpy(w, &v, sizeof(V));
    unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(V) / 8); ++i)
        __hip_atomic_store(q + i, w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <int COH, class V> __device__ __forceinline__ V ld_x(const V* x, long long i) {
    if constexpr ((COH & 2) != 0) return ld_coh(x + i);
    else return x[i];
}
template <int COH, class V> __device__ __forceinline__ V ld_y(const V* y, long long i) {
    if constexpr ((COH & 1) != 0) return ld_coh(y + i);
    else return y[i];
}
template <int COH, class V> __device__ __forceinline__ void st_y(V* y, long long i, const V& v) {
    if constexpr ((COH & 1) != 0) st_coh(y + i, v);
    else y[i] = v;
}
// Raw buffer access: a wave-uniform descriptor (base address in scalar
// registers), one 32-bit vector offset shared by all elements of a lane and
// a 32-bit scalar offset per element.  A flat pointer would need a 64-bit
// vector address per element, since the element strides exceed the 4 KiB
// immediate offset range.  Descriptor word 3: 32-bit data format (raw
// accesses on this architecture must not use the invalid format); the
// record count is the maximum, so no access is range-clamped.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* p) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, -1, 0x00020000);
}
template <class V> __device__ __forceinline__ V buf_load(__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
    V v;
    if constexpr (sizeof(V) == 8) {
        const auto q = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
        __builtin_memcpy(&v, &q, 8);
    } else {
        static_assert(sizeof(V) == 16, "complex float or double");
        const auto q = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)voff, (int)soff, 0);
        __builtin_memcpy(&v, &q, 16);
    }
    return v;
}
template <class V> __device__ __forceinline__ void buf_store(const V& v, __amdgpu_buffer_rsrc_t rs, unsigned voff,
                                                             unsigned soff) {
    static_assert(sizeof(V) == 8, "8-byte elements only");
    unsigned __attribute__((ext_vector_type(2))) q;
    __builtin_memcpy(&q, &v, 8);
    __builtin_amdgcn_raw_buffer_store_b64(q, rs, (int)voff, (int)soff, 0);
}

// One workgroup's share of a transform: block `block` of `nblocks`.
template <class V, class PL, int FT, bool IND, int COH, bool TL, int... Rs>
__device__ __forceinline__ void fft_body(const V* __restrict__ x, V* __restrict__ y, const KArgs<V>& a,
                                         const KCall<typename RealOf<V>::type>& kc, long long block,
                                         long long nblocks, char* smem) {
    using R = typename RealOf<V>::type;
    constexpr int E = PL::E, P = PL::P, M = PL::M, Ns = PL::Ns;
    constexpr bool BLOCK = PL::MULTI_WAVE;
    V* lds = reinterpret_cast<V*>(smem);
    R* red = reinterpret_cast<R*>(smem + Smem<V, PL, FT, IND>::RED_OFF);

    // An opaque copy of the lane index: a persistent caller runs this body in
    // a loop, and nothing derived from the lane may be hoisted out of it.
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    Geo<V, PL, IND> g(a, block, nblocks, tid);
    // The left vector is read where each element is encoded: from LDS where
    // one copy serves several lines or signals of the workgroup (and LDS
    // reads need no address registers), from the cached table otherwise.
    // Signals addressed directly (not through the ragged tables, and not
    // shared with other workgroups of the launch) move through raw buffers.
    constexpr bool kBufIO = !IND && COH == 0;
    // Stores of 16-byte elements stay flat.  A buffer store of more than 8
    // bytes reads its data registers after issue, and with a register as
    // scalar offset the compiler lets the next instruction overwrite them
    // (seen as complex-double outputs corrupted in groups of four lanes,
    // with clean checksums: the registers held the right values); two
    // 8-byte stores instead cost more than the flat store saves.
    constexpr bool kBufStore = kBufIO && sizeof(V) == 8;
    constexpr bool kCot = kCotLeft<V, PL, FT, IND> && kBufIO;
    constexpr int CG = 16 / (int)sizeof(R);   // cotangent values per 16-byte load
    static_assert(!kCot || E % CG == 0, "whole 16-byte runs of the cotangent table");
    const V* left = a.left;
    const auto left_rs = buf_rsrc(a.left);
    const auto cot_rs = buf_rsrc(a.cot);
    if constexpr (Smem<V, PL, FT, IND>::AW_LDS) {
        V* awl = reinterpret_cast<V*>(smem + Smem<V, PL, FT, IND>::AW_OFF);
        if constexpr (!kResident<V, PL, FT, IND>) {   // resident kernels staged it once
            for (int i = tid; i < Ns; i += PL::THREADS) awl[i] = a.left[i];
        }
        left = awl;
    }
    if constexpr (PL::HAS_TW)
        g.twiddle_setup(a, reinterpret_cast<V*>(smem + Smem<V, PL, FT, IND>::TWS_OFF));
    // these tables are written by some waves and read by all: a workgroup
    // barrier whenever the workgroup has more than one wave (sub-wave slots
    // otherwise only synchronise within their wave)
    if constexpr (PL::HAS_TW || (Smem<V, PL, FT, IND>::AW_LDS && !kResident<V, PL, FT, IND>))
        lds_sync<(PL::THREADS > kWave)>();
    const auto li = g.lidx();
    constexpr bool KEEP_XS = FT == 3;   // in place: inputs are gone after the store
    const int t = g.t;

    // This lane's share of the left vector e^T W (always the same positions)
    // is loaded with each transaction's inputs and dies at the encoding, so it
    // holds no registers through the butterflies; repeats hit the cache.

    V reg[E];
    V xs[KEEP_XS ? E : 1];
    V ps = V{0, 0}, pw = V{0, 0};   // sum_b p_b, sum_b (b+1) p_b
    V qs = V{0, 0}, qw = V{0, 0};   // sum_b q_b, sum_b (b+1) q_b
    R nu = 0;                        // input energy of the group
    unsigned nfmask = 0;             // transactions with a non-finite / oversized output
    // per-transaction checking: this lane's kept partial, the slot's
    // q_b - p_b (D0 of transaction b = tx_tl()) and input energy nu_b
    R txd[3] = {0, 0, 0};
    const bool per_tx = FT != 0 && a.gran != 0;
    if constexpr (KEEP_XS) {
#pragma unroll
        for (int r = 0; r < E; ++r) xs[r] = V{0, 0};
    }

    for (int b = 0; b < a.T; ++b) {
        const long long s = g.sig(b);
        const bool valid = s < a.batch;
        // Opaque copies of the lane's coordinates: address arithmetic is
        // recomputed inside each transaction instead of being hoisted into
        // dozens of loop-invariant registers.
        int t = g.t;
        asm volatile("" : "+v"(t));
        auto li = g.lidx();
        asm volatile("" : "+v"(li));
        // this lane's share of e^T W: single-pass plans request it before
        // the inputs, so that the two loads overlap (they meet in the
        // encode); tiles read it there, which keeps the row pass (where it
        // also meets the inter-pass twiddle) within fewer registers
        auto left_at = [&](int r) -> V {
            if constexpr (Smem<V, PL, FT, IND>::AW_LDS || !kBufIO) return left[t + P * r];
            else return buf_load<V>(left_rs, (unsigned)t * (unsigned)sizeof(V), (unsigned)(P * r * (int)sizeof(V)));
        };
        constexpr bool kAwEarly = FT != 0 && PL::KIND == kSingle && kBufIO && !kCot;
        V aw[kAwEarly ? E : 1];
        if constexpr (kAwEarly) {
#pragma unroll
            for (int r = 0; r < E; ++r) aw[r] = left_at(r);
        }
        R cw[kCot ? E : 1];
        if constexpr (kCot) {
#pragma unroll
            for (int j = 0; j < E / CG; ++j) {
                const auto q = __builtin_amdgcn_raw_buffer_load_b128(cot_rs, (int)((unsigned)t * 16u),
                                                                      j * P * 16, 0);
                __builtin_memcpy(&cw[j * CG], &q, 16);
            }
        }
        if (valid) {
            if constexpr (kBufIO) {
                const auto rs = buf_rsrc(x + g.in_uni(a, b));
                const unsigned st = (unsigned)(g.in_step(a) * (long long)sizeof(V));
                const unsigned lo = g.lane_in * (unsigned)sizeof(V);
#pragma unroll
                for (int r = 0; r < E; ++r) reg[r] = buf_load<V>(rs, lo, st * (unsigned)r);
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) reg[r] = ld_x<COH>(x, g.in_off(a, s, t + P * r));
            }
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r] = V{0, 0};
        }
        if constexpr (kBufIO) {
            const unsigned long long cm = sign_mask(kc.conj_in);
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r].y = xor_sign(reg[r].y, cm);
        } else if (kc.conj_in) {
            // the persistent kernel holds every plan in one function: a
            // branch here costs it fewer registers than the mask
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r].y = -reg[r].y;
        }
        V p = V{0, 0};
        R nub = 0;   // input energy of this transaction
        {
            const R wb = (R)(b + 1);
            V cs = V{0, 0};   // cotangent form: sum of the values, sum of cot_n x_n in p
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const V z = reg[r];   // raw loaded value
                V tw = V{(R)1, (R)0};
                if constexpr (PL::HAS_TW) {
                    tw = g.twiddle(a, s, r);
                    reg[r] = cmul(z, tw);
                }
                if constexpr (FT != 0) {
                    if constexpr (kCot) {
                        cs = cadd(cs, z);
                        p = V{fmad(cw[r], z.x, p.x), fmad(cw[r], z.y, p.y)};
                    } else {
                        V av;
                        if constexpr (kAwEarly) av = aw[r];
                        else av = left_at(r);
                        if constexpr (PL::HAS_TW) av = cmul(av, tw);
                        p = cmac(p, av, z);
                    }
                    nub = fmad(z.x, z.x, fmad(z.y, z.y, nub));
                    if constexpr (KEEP_XS) xs[r] = cadd(xs[r], z);
                }
            }
            // p = c2 (S - i C), S = sum x_n, C = sum cot_n x_n
            if constexpr (kCot) p = cmul(a.cot_c2, V{cs.x + p.y, cs.y - p.x});
            if constexpr (FT != 0) {
                if (!per_tx) {
                    ps = cadd(ps, p);
                    pw = V{fmad(wb, p.x, pw.x), fmad(wb, p.y, pw.y)};
                    nu = nu + nub;
                }
            }
        }

        // test hook: one bit flip in the value of position inj_elem after
        // radix stage inj_stage (a uniform branch on kernel arguments)
        auto inject = [&](int stage, V (&rg)[E]) {
            if (kc.inj_signal >= 0 && kc.inj_stage == stage && valid &&
                (g.gid(a, s) == kc.inj_signal || g.gid(a, s) == kc.inj_signal2)) {
                const int rh = g.inj_r(a, kc);
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    if (r == rh) {
                        if (kc.inj_part == 0) rg[r].x = flip_bit(rg[r].x, kc.inj_bit);
                        else rg[r].y = flip_bit(rg[r].y, kc.inj_bit);
                    }
                }
            }
        };
        if constexpr (TL) {
            ThreadGuard<V> tg;
            tg.tab = a.thr_tab;
            tg.kappa_u = a.thr_ku;
            tg.counts = kc.counts;
            tg.sig = g.gid(a, s);
            tg.inj_stage = (kc.inj_signal >= 0 && valid && (tg.sig == kc.inj_signal || tg.sig == kc.inj_signal2) &&
                            (long long)t == kc.inj_elem % P) ? kc.inj_stage : -1;
            tg.inj_j = (int)((kc.inj_elem / P) & 15);
            tg.inj_part = kc.inj_part;
            tg.inj_bit = kc.inj_bit;
            NoHook nh;
            slot_fft<V, E, P, BLOCK, decltype(li), NoHook, ThreadGuard<V>, 0, 1, Rs...>(reg, a.tw, t, lds, li, nh, tg);
        } else {
            NoGuard ng;
            slot_fft<V, E, P, BLOCK, decltype(li), decltype(inject), NoGuard, 0, 1, Rs...>(reg, a.tw, t, lds, li,
                                                                                        inject, ng);
        }

        if constexpr (FT != 0) {
            const V q = encode_out<V, E, P, M>(reg);
            if (per_tx) {
                // check of transaction b (Sec. 4.1, note and continue): the
                // slot's q_b - p_b and nu_b, reduced over the lanes of this
                // wave and kept by lane b; the decision is taken for all
                // transactions of the group at its end
                int tt = g.t;
                asm volatile("" : "+v"(tt));
                const V lf = wM<V, M>(tt % M);
                const V d = csub(cmul(lf, q), p);
                const R w0 = g.tx_wave_sum(d.x), w1 = g.tx_wave_sum(d.y), w2 = g.tx_wave_sum(nub);
                if (g.tx_tl() == b) {
                    txd[0] = w0;
                    txd[1] = w1;
                    txd[2] = w2;
                }
            } else {
                const R wb = (R)(b + 1);
                qs = cadd(qs, q);
                qw = V{fmad(wb, q.x, qw.x), fmad(wb, q.y, qw.y)};
                if (!cfin(q.x, q.y, a.cap)) nfmask |= 1u << b;
            }
        }

        if (valid) {
            const auto rs = buf_rsrc(y + g.out_uni(a, b));
            const unsigned st = (unsigned)(g.out_step(a) * (long long)sizeof(V));
            const unsigned lo = g.lane_out * (unsigned)sizeof(V);
            // conjugation folded into the scale of the imaginary part
            // (-a * s and a * -s round alike)
            const R sy = kc.conj_out ? -kc.scale : kc.scale;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const V v = reg[r];
                const V o = V{v.x * kc.scale, v.y * sy};
                if constexpr (kBufStore) buf_store<V>(o, rs, lo, st * (unsigned)r);
                else st_y<COH>(y, g.out_off(a, s, t + P * r), o);
            }
        }
    }

    if constexpr (FT != 0) {
        // The group close decides and corrects; its arithmetic never reaches
        // a fault-free output, so the compiler may fuse freely here.
#pragma clang fp contract(fast)
        const V lanef = wM<V, M>(t % M);   // e_{t + P r} = w_M^t w_M^{P r}

        // ---- delayed batched correction (Sec. 4.1, Eq. 5) ----
        // Correct transaction bstar of this slot from the right-side sums of
        // transactions [0, upto): c = W x_s - Y e, with x_s = X e summed from
        // the intact inputs (in registers when in place) and Y e from the
        // stored outputs (HBM, where transactions corrected earlier in the
        // group already hold their repaired values).  act: 0 nothing for this
        // slot, 1 add c when it is finite and small, else rebuild, 2 rebuild
        // y_b* = W x_s - sum_{b != b*} y_b.  The repair is accepted when
        // |e^T c + dref| <= tau_v (c explains the discrepancy) or, for a
        // rebuild, when the rebuilt values are finite.  Called by the whole
        // synchronisation domain together (it exchanges through LDS).
        const Geo<V, PL, IND>& g0 = g;
        auto correct = [&](int act, int bstar, int upto, V dref, R tau_v, R nu_sum) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            // opaque coordinates: called in a loop, nothing derived from the
            // lane or the group may be hoisted out of it (the 64-bit addresses
            // of every element would then stay live through the loop)
            Geo<V, PL, IND> g = g0;
            asm volatile("" : "+v"(g.t), "+v"(g.sig0), "+v"(g.lds_off), "+v"(g.line), "+v"(g.slot),
                              "+v"(g.tile), "+v"(g.tw_base.x), "+v"(g.tw_base.y));
            const int t = g.t;
            const auto li = g.lidx();
            const V lanef = wM<V, M>(t % M);
            const long long sstar = g.sig(bstar < 0 ? 0 : bstar);
            // loops run over the whole group (a uniform bound) and skip the
            // transactions past upto, which may differ between the slots of a wave
            int nvalid = 0;
            for (int b = 0; b < a.T; ++b) nvalid += (b < upto && g.sig(b) < a.batch) ? 1 : 0;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                V acc = V{0, 0};
                if constexpr (KEEP_XS) {
                    acc = xs[r];
                } else {
                    for (int b = 0; b < a.T; ++b) {
                        const long long sb = g.sig(b);
                        if (b >= upto || sb >= a.batch) continue;
                        V xv = ld_x<COH>(x, g.in_off(a, sb, t + P * r));
                        if (kc.conj_in) xv.y = -xv.y;
                        acc = cadd(acc, xv);
                    }
                }
                // every transaction of a group shares the twiddle (row pass:
                // same rows; three-pass passes run one transaction per group)
                if constexpr (PL::HAS_TW) acc = cmul(acc, g.twiddle(a, g.sig(0), r));
                reg[r] = acc;
            }
            NoHook nohook;
            NoGuard ng;
            slot_fft<V, E, P, BLOCK, decltype(li), NoHook, NoGuard, 0, 1, Rs...>(reg, a.tw, t, lds, li, nohook, ng);   // W x_s
            // c = W x_s - Y e, element by element, Y e summed from the stored
            // outputs (internal domain); skip: leave out b*
            auto corr_elem = [&](int r, int skip) -> V {
                V acc = reg[r];
                for (int b = 0; b < a.T; ++b) {
                    const long long sb = g.sig(b);
                    if (b >= upto || sb >= a.batch || b == skip) continue;
                    V yv = ld_y<COH>(y, g.out_off(a, sb, t + P * r));
                    if (kc.conj_out) yv.y = -yv.y;
                    acc = V{acc.x - yv.x / kc.scale, acc.y - yv.y / kc.scale};
                }
                return acc;
            };
            const R yrms2 = (R)Ns * nu_sum / (R)(nvalid > 0 ? nvalid : 1);
            bool cf = true, small = true;
            V bucket[M];
#pragma unroll
            for (int m = 0; m < M; ++m) bucket[m] = V{0, 0};
#pragma unroll
            for (int r = 0; r < E; ++r) {
                const V c = corr_elem(r, -1);
                cf = cf && cfin(c.x, c.y, a.cap);
                small = small && (c.x * c.x + c.y * c.y) <= yrms2;
                bucket[(P * r) % M] = cadd(bucket[(P * r) % M], c);
            }
            V ec = bucket[0];
#pragma unroll
            for (int m = 1; m < M; ++m) ec = cadd(ec, cmul(bucket[m], wM<V, M>(m)));
            ec = cmul(lanef, ec);
            R w4[4] = {ec.x, ec.y, cf ? (R)0 : (R)1, small ? (R)0 : (R)1};
            g.template reduce<OpAdd>(w4, red);
            // additive only when c is finite and no larger than one signal's
            // rms output norm; otherwise rebuild from the other outputs
            if (act == 1 && !(w4[2] == (R)0 && w4[3] == (R)0)) act = 2;
            bool ok = true;
            if (act == 1) {
                const R vx = w4[0] + dref.x, vy = w4[1] + dref.y;
                ok = __builtin_sqrt(vx * vx + vy * vy) <= tau_v;
            }
            bool rebuilt_ok = true;
            if (act == 1 && ok) {
                // y_b* += scale * cj(c)
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    V cc = corr_elem(r, -1);
                    if (kc.conj_out) cc.y = -cc.y;
                    const long long o = g.out_off(a, sstar, t + P * r);
                    const V old = ld_y<COH>(y, o);
                    st_y<COH>(y, o, V{old.x + kc.scale * cc.x, old.y + kc.scale * cc.y});
                }
            } else if (act == 2) {
                // y_b* = scale * cj(W x_s - sum_{b != b*} y_b)
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    V vv = corr_elem(r, bstar);
                    if (kc.conj_out) vv.y = -vv.y;
                    vv = V{kc.scale * vv.x, kc.scale * vv.y};
                    rebuilt_ok = rebuilt_ok && cfin(vv.x, vv.y, a.cap);
                    st_y<COH>(y, g.out_off(a, sstar, t + P * r), vv);
                }
            }
            unsigned badv[1] = {(act == 2 && !rebuilt_ok) ? 1u : 0u};
            g.template reduce<OpOr>(badv, reinterpret_cast<unsigned*>(red));
            if (act == 2 && badv[0] != 0u) ok = false;
            if ((act == 1 || act == 2) && t == 0) {
                atomicAdd(&kc.counts->detected, 1ull);
                if (!ok) atomicAdd(&kc.counts->uncorrectable, 1ull);
                else if (act == 1) atomicAdd(&kc.counts->corrected, 1ull);
                else atomicAdd(&kc.counts->rebuilt, 1ull);
                atomicExch(&kc.counts->last_signal, (unsigned long long)g.rid(a, sstar));
            }
            // the next correction of this group re-reads these outputs
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        };

        // Pending repairs, from whichever granularity is in use; one call site
        // below serves both, so the correction is compiled once.
        unsigned Fr = 0u;              // per transaction: faulty transactions not yet repaired
        int gact = 0, gb = -1;         // per group: 1 add / 2 rebuild, and the located signal
        V gD0 = V{0, 0};
        R gtau = 0, gnu = 0;
        if (per_tx) {
            // ---- per-transaction decisions, taken at the end of the group ----
            R* txr = reinterpret_cast<R*>(smem + Smem<V, PL, FT, IND>::TXR_OFF);
            // the host limits T to what the plan keeps; never read past it
            const int Tq = a.T < Geo<V, PL, IND>::TX_MAX ? a.T : Geo<V, PL, IND>::TX_MAX;
            g.template tx_parts_sum<3>(txd, Tq, txr);
            const int tl = g.tx_tl();
            // lane tl (< T) holds transaction tl's D0 = q - p and nu
            const R tau_b = a.tau_coef * __builtin_sqrt(txd[2]);
            const bool checked = tl < Tq && (txd[2] == txd[2]) && txd[2] < (R)INFINITY;
            const R d0 = __builtin_sqrt(txd[0] * txd[0] + txd[1] * txd[1]);
            const bool bad = checked && !(d0 <= tau_b);
            if (kc.stats && checked && !bad && tau_b > (R)0 && g.sig(tl) < a.batch) {
                const double q = (double)d0 / (double)tau_b;
                atomicMax(&kc.counts->calib, (unsigned long long)__double_as_longlong(q));
            }
            const unsigned F = g.tx_mask(bad, Tq);   // faulty transactions of this slot
            if constexpr (FT == 1) {
                if (t == 0) {
                    for (unsigned f = F; f != 0u; f &= f - 1u) {
                        atomicAdd(&kc.counts->detected, 1ull);
                        atomicExch(&kc.counts->last_signal,
                                   (unsigned long long)g.rid(a, g.sig(__builtin_ctz(f))));
                    }
                }
            } else {
                // in place, x_s holds the whole group's inputs: a lone fault
                // is repaired from it, two or more are not separable
                const int nbad = __builtin_popcount(F);
                const bool lone = !KEEP_XS || nbad <= 1;
                if (!lone && t == 0) {
                    atomicAdd(&kc.counts->detected, (unsigned long long)nbad);
                    atomicAdd(&kc.counts->uncorrectable, (unsigned long long)nbad);
                }
                Fr = lone ? F : 0u;
            }
        } else {
            // ---- group close: reduce the checksum differences over the slot ----
            const V dd0 = csub(cmul(lanef, qs), ps);   // this lane's share of D0
            const V dd1 = csub(cmul(lanef, qw), pw);   // and of D1
            const R nfc = (R)__builtin_popcount(nfmask);
            V D0, D1;
            R nu_s, nf_count;
            if (a.T == 1) {   // one transaction: D1 = D0, no location needed
                R v[4] = {dd0.x, dd0.y, nu, nfc};
                g.template reduce<OpAdd>(v, red);
                D0 = V{v[0], v[1]};
                D1 = D0;
                nu_s = v[2];
                nf_count = v[3];
            } else {
                R v[6] = {dd0.x, dd0.y, dd1.x, dd1.y, nu, nfc};
                g.template reduce<OpAdd>(v, red);
                D0 = V{v[0], v[1]};
                D1 = V{v[2], v[3]};
                nu_s = v[4];
                nf_count = v[5];
            }
            unsigned nf = 0;
            if (nf_count > (R)0) {   // rare: which transactions held a non-finite output
                unsigned nfv[1] = {nfmask};
                g.template reduce<OpOr>(nfv, reinterpret_cast<unsigned*>(red));
                nf = nfv[0];
            }

            // decision, identical on every lane of the slot:
            // 0 clean or unchecked, 1 add the correction, 2 rebuild, 3 uncorrectable
            int action = 0, bstar = -1;
            const R tau = a.tau_coef * __builtin_sqrt(nu_s);
            const bool checked = (nu_s == nu_s) && nu_s < (R)INFINITY;
            const R d0 = __builtin_sqrt(D0.x * D0.x + D0.y * D0.y);
            if (checked) {
                if (nf != 0) {
                    if ((nf & (nf - 1)) != 0) action = 3;
                    else { bstar = __builtin_ctz(nf); action = 2; }
                } else if (!(d0 <= tau)) {
                    const R den = D0.x * D0.x + D0.y * D0.y;
                    const R rr = (D1.x * D0.x + D1.y * D0.y) / den;
                    const R ri = (D1.y * D0.x - D1.x * D0.y) / den;
                    const R rnd = __builtin_rint(rr);
                    const R dx = rr - rnd;
                    const bool ok = rnd >= (R)1 && rnd <= (R)a.T && (dx * dx + ri * ri) <= (R)0.0625 &&
                                    g.sig((int)rnd - 1) < a.batch;
                    if (ok) { bstar = (int)rnd - 1; action = 1; }
                    else action = 3;
                }
            }
            if (kc.stats && checked && nf == 0 && t == 0 && tau > (R)0) {
                // calibration: largest |D0| / tau seen (non-negative doubles order as integers)
                const double q = (double)d0 / (double)tau;
                atomicMax(&kc.counts->calib, (unsigned long long)__double_as_longlong(q));
            }

            // Location fallback on the error path: when D1/D0 is not an index (an
            // error just above the threshold, where location noise dominates) and
            // the inputs are intact, re-encode every signal of the group and take
            // the one whose own checksums disagree most.
            if (g.domain_any(action == 3 && nf == 0 && a.x_intact)) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                R best = (R)-1;
                int bbest = -1;
                for (int b = 0; b < a.T; ++b) {
                    const long long sb = g.sig(b);
                    const bool vb = sb < a.batch;
                    V p = V{0, 0};
                    V bucket[M];
#pragma unroll
                    for (int m = 0; m < M; ++m) bucket[m] = V{0, 0};
                    if (vb) {
#pragma unroll
                        for (int r = 0; r < E; ++r) {
                            V xv = ld_x<COH>(x, g.in_off(a, sb, t + P * r));
                            if (kc.conj_in) xv.y = -xv.y;
                            V av = left[t + P * r];
                            if constexpr (PL::HAS_TW) av = cmul(av, g.twiddle(a, sb, r));
                            p = cadd(p, cmul(av, xv));
                            V yv = ld_y<COH>(y, g.out_off(a, sb, t + P * r));
                            if (kc.conj_out) yv.y = -yv.y;
                            bucket[(P * r) % M] = cadd(bucket[(P * r) % M], V{yv.x / kc.scale, yv.y / kc.scale});
                        }
                    }
                    V q = bucket[0];
#pragma unroll
                    for (int m = 1; m < M; ++m) q = cadd(q, cmul(bucket[m], wM<V, M>(m)));
                    q = cmul(lanef, q);
                    R d[2] = {q.x - p.x, q.y - p.y};
                    g.template reduce<OpAdd>(d, red);
                    const R m2 = d[0] * d[0] + d[1] * d[1];
                    if (vb && m2 > best) { best = m2; bbest = b; }
                }
                if (action == 3 && nf == 0 && bbest >= 0) {
                    bstar = bbest;
                    action = 1;
                    if (t == 0) atomicAdd(&kc.counts->fallback, 1ull);
                }
            }
            const long long sstar = g.sig(bstar < 0 ? 0 : bstar);

            if constexpr (FT == 1) {
                if (action != 0 && t == 0) {
                    atomicAdd(&kc.counts->detected, 1ull);
                    if (action == 3) atomicAdd(&kc.counts->uncorrectable, 1ull);
                    else atomicExch(&kc.counts->last_signal, (unsigned long long)g.rid(a, sstar));
                }
            } else {
                if (action == 1 || action == 2) {
                    gact = action;
                    gb = bstar;
                    gD0 = D0;
                    gtau = tau;
                    gnu = nu_s;
                }
                if (action == 3 && t == 0) {
                    atomicAdd(&kc.counts->detected, 1ull);
                    atomicAdd(&kc.counts->uncorrectable, 1ull);
                }
            }
        }

        if constexpr (FT != 1) {
            // Repairs, oldest first.  Per transaction (note and continue), a
            // faulty transaction is corrected from the sums of the
            // transactions before the next faulty one, or of the whole group;
            // per group, the located signal from the whole group's sums.  (The
            // guard keeps the loop's set-up off the fault-free path.)
            if (g.domain_any(Fr != 0u || gact != 0)) do {
                int act = 0, bstar = -1, upto = a.T;
                V dref = V{0, 0};
                R tau_v = 0, nu_sum = 0;
                if (Fr != 0u) {
                    bstar = __builtin_ctz(Fr);
                    Fr &= Fr - 1u;
                    upto = Fr ? (int)__builtin_ctz(Fr) : a.T;
                    dref = V{__shfl(txd[0], g.tx_lane(bstar)), __shfl(txd[1], g.tx_lane(bstar))};
                    for (int b = 0; b < a.T; ++b) {
                        const R nb = __shfl(txd[2], g.tx_lane(b));
                        if (b < upto && nb == nb && nb < (R)INFINITY) nu_sum += nb;
                    }
                    // c carries the rounding of every signal in the sums
                    tau_v = a.tau_coef * __builtin_sqrt(nu_sum);
                    act = 1;
                } else if (gact != 0) {
                    act = gact;
                    bstar = gb;
                    dref = gD0;
                    tau_v = gtau;
                    nu_sum = gnu;
                    gact = 0;
                }
                correct(act, bstar, upto, dref, tau_v, nu_sum);
            } while (g.domain_any(Fr != 0u));
        }
    }
}

// Occupancy the checking tile and streaming single-pass kernels are held
// to: what their LDS allows, at most four waves per SIMD (three in place).  The error path (correction) needs more registers
// than the transform; without the floor the compiler lowers the occupancy of
// the whole kernel for it and then spends the registers in the hot loop too.
// With it, the error path spills instead, which costs nothing when no fault
// occurs.
template <class V, class PL, int FT, bool IND> struct Occupancy {
    static constexpr int LDS_PER_CU = 160 * 1024;
    static constexpr int WG_PER_CU = LDS_PER_CU / Smem<V, PL, FT, IND>::BYTES;
    static constexpr int LDS_WAVES = WG_PER_CU * PL::WAVES / 4;   // per SIMD
    // in place, the right-side input sum stays in registers through the group
    static constexpr int CAP = FT == 3 ? 3 : 4;
    static constexpr int WAVES = FT == 0 || !(PL::TILE || PL::STREAM) ? 1 : (LDS_WAVES < 1 ? 1 : (LDS_WAVES > CAP ? CAP : LDS_WAVES));
};

// FT = 4: thread-level ABFT only (the workgroup-level checks of FT 0).
template <int FT> constexpr int kGroupFt = FT == 4 ? 0 : FT;

template <class V, class PL, int FT, bool IND, int... Rs>
__global__ __launch_bounds__(PL::THREADS)
__attribute__((amdgpu_waves_per_eu(Occupancy<V, PL, kGroupFt<FT>, IND>::WAVES)))
void k_fft(const V* __restrict__ x, V* __restrict__ y, KArgs<V> a) {
    constexpr int GF = kGroupFt<FT>;
    constexpr bool TL = FT == 4;
    static_assert(Smem<V, PL, GF, IND>::BYTES <= 160 * 1024, "LDS of a workgroup exceeds a CU's");
    static_assert(!kResident<V, PL, GF, IND> || Smem<V, PL, GF, IND>::AW_LDS, "resident kernels stage e^T W");
    __shared__ __align__(16) char smem[Smem<V, PL, GF, IND>::BYTES];
    if constexpr (kResident<V, PL, GF, IND>) {
        // e^T W into LDS once; every exchange and reduction of the first
        // group passes a workgroup barrier before it is read
        V* awl = reinterpret_cast<V*>(smem + Smem<V, PL, GF, IND>::AW_OFF);
        for (int i = threadIdx.x; i < PL::Ns; i += PL::THREADS) awl[i] = a.left[i];
        __syncthreads();
        for (long long g = blockIdx.x; g < a.nblk; g += gridDim.x)
            fft_body<V, PL, GF, IND, 0, TL, Rs...>(x, y, a, a, g, a.nblk, smem);
    } else {
        fft_body<V, PL, GF, IND, 0, TL, Rs...>(x, y, a, a, blockIdx.x, gridDim.x, smem);
    }
}

}  // namespace tfft
