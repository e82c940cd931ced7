// tfft_kernels.hpp -- batched C2C FFT kernels with fused two-side ABFT (gfx950).
//
// Structure (TurboFFT Sec. 3.1, Fig. 3, re-designed for CDNA4):
//   * a "slot" is the set of P = N/E lanes that transform one signal per
//     transaction, E elements per lane held in registers;
//   * lane t of a slot holds elements t + P*r (r < E) before and after every
//     stage, so HBM loads/stores and LDS reads are unit-stride across lanes;
//   * stage s (radix R, L = product of the earlier radices) is a Stockham
//     autosort step: butterfly beta = t + i*P reads elements beta + j*N/R,
//     multiplies by w_{LR}^{j k} (k = beta mod L, from a precomputed table,
//     Sec. 3.1 "avoid FP64 trigonometric functions"), applies the radix-R DFT
//     in registers and writes output j to g*L*R + k + j*L (g = beta div L);
//   * stages exchange data through LDS with an XOR swizzle instead of padding
//     (Sec. 3.2); slots of at most one wavefront synchronise with wavefront
//     fences only, larger slots use workgroup barriers;
//   * a slot runs T transactions back to back (Sec. 4.3 multi-transaction).
//
// Two-side ABFT (Sec. 4.1-4.3), per slot and group of T transactions:
//   right side  x_s = sum_b x_b,  y_s = sum_b y_b          (X e_c, Y e_c)
//   location    xw_s = sum_b (b+1) x_b,  q_b = e^T y_b      (e_3 weights)
//   left side   s_in = (e^T W) x_s, l_in = (e^T W) xw_s,
//               s_out = e^T y_s,   l_out = sum_b (b+1) q_b
//   D0 = s_out - s_in detects, D1/D0 - 1 locates, c = W x_s - y_s corrects.
// Linearity lets the left encoding of the inputs run once per group on the
// right-side sums instead of once per element; e_k = w_M^k takes only M
// values, so e^T y needs M bucket sums per lane and no table.
#pragma once

#include "tfft_device.hpp"

namespace tfft {

struct FtCounts {   // mirrors tfft_ft_counts in the public header
    unsigned long long detected, corrected, rebuilt, uncorrectable, last_signal, reserved[3];
};

// Kernel arguments shared by all transform kernels.
template <class V> struct KArgs {
    using R = typename RealOf<V>::type;
    const V* tw;          // stage twiddle tables, concatenated
    const V* left;        // e^T W for the transform length (ABFT only)
    long long batch;      // number of signals
    int T;                // transactions (signals) per slot
    int conj;             // 1: conjugate on load and store (inverse direction)
    R scale;              // applied to every stored value
    R tau_coef;           // kappa * u * sqrt(N log2 N); tau = tau_coef * sqrt(nu)
    R cap;                // magnitude cap: larger outputs mark their signal corrupted
    FtCounts* counts;     // device counters (ABFT only)
    long long inj_signal; // signal to corrupt (-1: none)
    int inj_elem;         // output element index
    int inj_part;         // 0 real, 1 imaginary
    int inj_bit;          // bit to flip
    int stats;            // 1: record max |D0| / tau over groups (calibration)
    int x_intact;         // 1: out of place, inputs can be re-read on the error path
};

// Compile-time plan: length N, E elements per lane, WPB waves per workgroup,
// swizzle row 2^B, stage radices Rs...
template <int N_, int E_, int WPB_, int B_, int... Rs> struct Plan {
    static constexpr int N = N_;
    static constexpr int E = E_;
    static constexpr int P = N / E;                       // lanes per slot
    static constexpr bool MULTI_WAVE = P > kWave;         // slot spans waves
    static constexpr int WPB = MULTI_WAVE ? P / kWave : WPB_;
    static constexpr int THREADS = WPB * kWave;
    static constexpr int SPW = MULTI_WAVE ? 1 : kWave / P;  // slots per wave
    static constexpr int SLOTS = MULTI_WAVE ? 1 : WPB * SPW; // slots per workgroup
    static constexpr int B = B_;
    static constexpr int LDS_ELEMS = MULTI_WAVE ? N : WPB * SPW * N;
    static constexpr int M = (N % 3 == 0) ? 5 : 3;         // encoding period
    static_assert(N % E == 0, "E must divide N");
    static_assert(MULTI_WAVE ? (P % kWave == 0) : (kWave % P == 0), "slot must tile waves");
    static_assert(((Rs * ...) == N), "radices must multiply to N");
    static_assert(((E % Rs == 0) && ...), "every radix must divide E");
};

// Bit flip of one component (fault injection, Sec. 5.3 protocol).
__device__ __forceinline__ float flip_bit(float v, int bit) {
    return __uint_as_float(__float_as_uint(v) ^ (1u << bit));
}
__device__ __forceinline__ double flip_bit(double v, int bit) {
    return __longlong_as_double(__double_as_longlong(v) ^ (1ll << bit));
}

// ---------------------------------------------------------------------------
// One Stockham stage.  LAST: results stay in registers (output layout),
// otherwise they go to LDS at their autosorted positions.
// ---------------------------------------------------------------------------
template <class V, int E, int P, int N, int R, int L, bool LAST, int B>
__device__ __forceinline__ void stockham_stage(V (&reg)[E], const V* __restrict__ tw_s, int t,
                                               V* __restrict__ lds, int lds_off) {
    constexpr int NB = E / R;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int beta = t + i * P;
        const int k = beta % L;
        V v[R];
#pragma unroll
        for (int j = 0; j < R; ++j) v[j] = reg[i + j * NB];
        if constexpr (L > 1) {
            const V* w = tw_s + k * R;
#pragma unroll
            for (int j = 1; j < R; ++j) v[j] = cmul(v[j], w[j]);
        }
        dft<R>(v);
        if constexpr (LAST) {
#pragma unroll
            for (int j = 0; j < R; ++j) reg[i + j * NB] = v[j];
        } else {
            const int base = lds_off + (beta / L) * (L * R) + k;
#pragma unroll
            for (int j = 0; j < R; ++j) lds[swz<B>(base + j * L)] = v[j];
        }
    }
}

// All stages of one in-slot FFT.  reg holds elements t + P*r on entry and the
// transform's outputs t + P*r on exit.
template <class V, int E, int P, int N, int B, bool BLOCK, int L, int R, int... Rest>
__device__ __forceinline__ void slot_fft(V (&reg)[E], const V* __restrict__ tw, int t,
                                         V* __restrict__ lds, int lds_off) {
    constexpr bool LAST = sizeof...(Rest) == 0;
    stockham_stage<V, E, P, N, R, L, LAST, B>(reg, tw, t, lds, lds_off);
    if constexpr (!LAST) {
        lds_sync<BLOCK>();
#pragma unroll
        for (int r = 0; r < E; ++r) reg[r] = lds[swz<B>(lds_off + t + P * r)];
        lds_sync<BLOCK>();
        // the next stage's table follows this one: L*R entries
        slot_fft<V, E, P, N, B, BLOCK, L * R, Rest...>(reg, tw + L * R, t, lds, lds_off);
    }
}

template <class V, class PL, int... Rs> struct SlotFFT {
    __device__ __forceinline__ static void run(V (&reg)[PL::E], const V* tw, int t, V* lds,
                                               int lds_off) {
        // stage 0 has L = 1 and reads no twiddles; its table slot holds R0 entries
        slot_fft<V, PL::E, PL::P, PL::N, PL::B, PL::MULTI_WAVE, 1, Rs...>(reg, tw, t, lds, lds_off);
    }
};

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
    for (int m = 1; m < M; ++m) acc = cadd(acc, cmul(bucket[m], wM<V, M>(m)));
    return acc;
}

// Reduce K values (sum) over one slot.  Single-wave slots use lane shuffles
// (an XOR butterfly leaves bit-identical results on every lane); multi-wave
// slots add one pass through LDS, which the caller must not be using.
template <class PL, class R, int K>
__device__ __forceinline__ void slot_sum(R (&v)[K], R* scratch /* K * WPB */) {
    if constexpr (!PL::MULTI_WAVE) {
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = group_sum<PL::P>(v[i]);
    } else {
#pragma unroll
        for (int i = 0; i < K; ++i) v[i] = group_sum<kWave>(v[i]);
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int i = 0; i < K; ++i) scratch[i * PL::WPB + wave] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < K; ++i) {
            R s = 0;
#pragma unroll
            for (int w = 0; w < PL::WPB; ++w) s += scratch[i * PL::WPB + w];
            v[i] = s;
        }
        __syncthreads();
    }
}

template <class PL> __device__ __forceinline__ unsigned slot_or(unsigned v, unsigned* scratch) {
    if constexpr (!PL::MULTI_WAVE) {
        return group_or<PL::P>(v);
    } else {
        v = group_or<kWave>(v);
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        __syncthreads();
        if (lane == 0) scratch[wave] = v;
        __syncthreads();
        unsigned o = 0;
#pragma unroll
        for (int w = 0; w < PL::WPB; ++w) o |= scratch[w];
        __syncthreads();
        return o;
    }
}

template <class PL, class R> __device__ __forceinline__ R slot_max(R v, R* scratch) {
    if constexpr (!PL::MULTI_WAVE) {
        return group_max<PL::P>(v);
    } else {
        v = group_max<kWave>(v);
        const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        __syncthreads();
        if (lane == 0) scratch[wave] = v;
        __syncthreads();
        R m = scratch[0];
#pragma unroll
        for (int w = 1; w < PL::WPB; ++w) m = (scratch[w] > m || scratch[w] != scratch[w]) ? scratch[w] : m;
        __syncthreads();
        return m;
    }
}

// Is any lane of the synchronisation domain flagging?  Multi-wave slots take
// their decisions from workgroup-wide reductions, so the flag is uniform.
template <class PL> __device__ __forceinline__ bool domain_any(bool f) {
    if constexpr (!PL::MULTI_WAVE) return __any(f) != 0;
    else return f;
}

template <class R> __device__ __forceinline__ bool cfin(R x, R y, R cap) {
    return finite_le(x, cap) && finite_le(y, cap);
}

// ---------------------------------------------------------------------------
// Single-pass batched kernel.  FT: 0 off, 1 detect (one-side check plus
// location), 2 correct (two-side, delayed batched correction at group close).
// ---------------------------------------------------------------------------
template <class V, class PL, int FT, int... Rs>
__global__ __launch_bounds__(PL::THREADS) void k_single(const V* __restrict__ x, V* __restrict__ y,
                                                        KArgs<V> a) {
    using R = typename RealOf<V>::type;
    constexpr int N = PL::N, E = PL::E, P = PL::P, M = PL::M;
    __shared__ V lds[PL::LDS_ELEMS];

    const int lane = threadIdx.x % kWave;
    const int wave = threadIdx.x / kWave;
    int t, lds_off;
    long long sig0;      // signal of transaction 0
    long long sig_step;  // signal stride between transactions
    if constexpr (PL::MULTI_WAVE) {
        t = threadIdx.x;
        lds_off = 0;
        sig0 = (long long)blockIdx.x * a.T;
        sig_step = 1;
    } else {
        const int sigma = lane / P;
        t = lane % P;
        lds_off = (wave * PL::SPW + sigma) * N;
        sig0 = ((long long)blockIdx.x * PL::WPB + wave) * a.T * PL::SPW + sigma;
        sig_step = PL::SPW;
    }

    V reg[E];
    V xs[FT ? E : 1], xw[FT ? E : 1], ys[FT == 2 ? E : 1];
    V lq = V{0, 0};        // sum_b (b+1) q_b
    V sq = V{0, 0};        // sum_b q_b
    R nu = 0;              // input energy
    unsigned nfmask = 0;   // transactions with a non-finite / oversized output
    if constexpr (FT != 0) {
#pragma unroll
        for (int r = 0; r < E; ++r) xs[r] = xw[r] = V{0, 0};
    }
    if constexpr (FT == 2) {
#pragma unroll
        for (int r = 0; r < E; ++r) ys[r] = V{0, 0};
    }

    for (int b = 0; b < a.T; ++b) {
        const long long sig = sig0 + (long long)b * sig_step;
        const bool valid = sig < a.batch;
        const V* xin = x + sig * N;
        if (valid) {
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r] = xin[t + P * r];
        } else {
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r] = V{0, 0};
        }
        if (a.conj) {
#pragma unroll
            for (int r = 0; r < E; ++r) reg[r].y = -reg[r].y;
        }
        if constexpr (FT != 0) {
            const R wb = (R)(b + 1);
#pragma unroll
            for (int r = 0; r < E; ++r) {
                xs[r] = cadd(xs[r], reg[r]);
                xw[r] = V{xw[r].x + wb * reg[r].x, xw[r].y + wb * reg[r].y};
                nu += reg[r].x * reg[r].x + reg[r].y * reg[r].y;
            }
        }

        SlotFFT<V, PL, Rs...>::run(reg, a.tw, t, lds, lds_off);

        if (sig == a.inj_signal) {   // test hook: one bit flip in one output value
#pragma unroll
            for (int r = 0; r < E; ++r) {
                if (t + P * r == a.inj_elem) {
                    if (a.inj_part == 0) reg[r].x = flip_bit(reg[r].x, a.inj_bit);
                    else reg[r].y = flip_bit(reg[r].y, a.inj_bit);
                }
            }
        }

        if constexpr (FT != 0) {
            const V q = encode_out<V, E, P, M>(reg);
            const R wb = (R)(b + 1);
            sq = cadd(sq, q);
            lq = V{lq.x + wb * q.x, lq.y + wb * q.y};
            if (!cfin(q.x, q.y, a.cap)) nfmask |= 1u << b;
        }
        if constexpr (FT == 2) {
#pragma unroll
            for (int r = 0; r < E; ++r) ys[r] = cadd(ys[r], reg[r]);
        }

        if (valid) {
            V* yout = y + sig * N;
#pragma unroll
            for (int r = 0; r < E; ++r) {
                V v = reg[r];
                if (a.conj) v.y = -v.y;
                yout[t + P * r] = V{v.x * a.scale, v.y * a.scale};
            }
        }
    }

    if constexpr (FT != 0) {
        // ---- group close: left-side checksums from the right-side sums ----
        __shared__ R red[9 * PL::WPB];
        V sin_ = V{0, 0}, lin = V{0, 0};
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const V av = a.left[t + P * r];
            sin_ = cadd(sin_, cmul(av, xs[r]));
            lin = cadd(lin, cmul(av, xw[r]));
        }
        const V lanef = wM<V, M>(t % M);   // e_{t + P r} = w_M^t w_M^{P r}
        const V sout = cmul(lanef, sq);
        const V lout = cmul(lanef, lq);
        R v[9] = {sin_.x, sin_.y, lin.x, lin.y, sout.x, sout.y, lout.x, lout.y, nu};
        slot_sum<PL>(v, red);
        const unsigned nf = slot_or<PL>(nfmask, reinterpret_cast<unsigned*>(red));

        // decision, identical on every lane of the slot:
        // 0 clean or unchecked, 1 add the correction, 2 rebuild, 3 uncorrectable
        int action = 0, bstar = -1;
        const V D0 = V{v[4] - v[0], v[5] - v[1]};
        const V D1 = V{v[6] - v[2], v[7] - v[3]};
        const R nu_s = v[8];
        const R tau = a.tau_coef * __builtin_sqrt(nu_s);
        const bool checked = (nu_s == nu_s) && nu_s < (R)INFINITY;
        if (checked) {
            if (nf != 0) {
                if ((nf & (nf - 1)) != 0) action = 3;
                else { bstar = __builtin_ctz(nf); action = 2; }
            } else if (!(__builtin_sqrt(D0.x * D0.x + D0.y * D0.y) <= tau)) {
                const R den = D0.x * D0.x + D0.y * D0.y;
                const R rr = (D1.x * D0.x + D1.y * D0.y) / den;
                const R ri = (D1.y * D0.x - D1.x * D0.y) / den;
                const R rnd = __builtin_rint(rr);
                const R dx = rr - rnd;
                const bool ok = rnd >= (R)1 && rnd <= (R)a.T && (dx * dx + ri * ri) <= (R)0.0625 &&
                                (sig0 + (long long)((int)rnd - 1) * sig_step) < a.batch;
                if (ok) { bstar = (int)rnd - 1; action = 1; }
                else action = 3;
            }
        }
        if (a.stats && checked && nf == 0 && t == 0 && tau > (R)0) {
            // calibration: largest |D0| / tau seen (non-negative doubles order as integers)
            const double q = (double)__builtin_sqrt(D0.x * D0.x + D0.y * D0.y) / (double)tau;
            atomicMax(&a.counts->reserved[0], (unsigned long long)__double_as_longlong(q));
        }
        // Location fallback on the error path: when D1/D0 is not an index (an
        // error just above the threshold, where location noise dominates) and
        // the inputs are intact, re-encode every signal of the group and take
        // the one whose own checksums disagree most.
        if (domain_any<PL>(action == 3 && nf == 0 && a.x_intact)) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            R best = (R)-1;
            int bbest = -1;
            for (int b = 0; b < a.T; ++b) {
                const long long sb = sig0 + (long long)b * sig_step;
                const bool vb = sb < a.batch;
                V p = V{0, 0}, qv[E];
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    V xv = vb ? x[sb * N + t + P * r] : V{0, 0};
                    if (a.conj) xv.y = -xv.y;
                    p = cadd(p, cmul(a.left[t + P * r], xv));
                    V yv = vb ? y[sb * N + t + P * r] : V{0, 0};
                    if (a.conj) yv.y = -yv.y;
                    qv[r] = V{yv.x / a.scale, yv.y / a.scale};
                }
                const V q = cmul(lanef, encode_out<V, E, P, M>(qv));
                R d[2] = {q.x - p.x, q.y - p.y};
                slot_sum<PL>(d, red);
                const R m = d[0] * d[0] + d[1] * d[1];
                if (vb && m > best) { best = m; bbest = b; }
            }
            if (action == 3 && nf == 0 && bbest >= 0) { bstar = bbest; action = 1; }
        }
        const long long sstar = sig0 + (long long)(bstar < 0 ? 0 : bstar) * sig_step;

        if constexpr (FT == 1) {
            if (action != 0 && t == 0) {
                atomicAdd(&a.counts->detected, 1ull);
                if (action == 3) atomicAdd(&a.counts->uncorrectable, 1ull);
                else atomicExch(&a.counts->last_signal, (unsigned long long)sstar);
            }
        } else {
            if (domain_any<PL>(action == 1 || action == 2)) {
                // ---- delayed batched correction: W x_s on the slot's lanes ----
                SlotFFT<V, PL, Rs...>::run(xs, a.tw, t, lds, lds_off);   // xs := W x_s
                R cm = 0;
                bool cf = true;
                V cvec[E];
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    cvec[r] = csub(xs[r], ys[r]);   // c = W x_s - y_s
                    cf = cf && cfin(cvec[r].x, cvec[r].y, a.cap);
                    const R m2 = cvec[r].x * cvec[r].x + cvec[r].y * cvec[r].y;
                    cm = m2 > cm ? m2 : cm;
                }
                const V ec = cmul(lanef, encode_out<V, E, P, M>(cvec));
                R w3[3] = {ec.x, ec.y, cf ? (R)0 : (R)1};
                slot_sum<PL>(w3, red);
                const R cmx = slot_max<PL>(cm, red);
                // additive only when c is finite and no larger than one signal's
                // rms output norm; otherwise rebuild from the other outputs
                const R yrms2 = (R)N * nu_s / (R)a.T;
                if (action == 1 && !(w3[2] == (R)0 && cmx <= yrms2)) action = 2;
                bool ok = true;
                if (action == 1) {
                    const R vx = w3[0] + D0.x, vy = w3[1] + D0.y;
                    ok = __builtin_sqrt(vx * vx + vy * vy) <= tau;
                }
                // make this lane's earlier stores visible to its own reloads
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                bool rebuilt_ok = true;
                if (action == 1 && ok) {
                    V* yo = y + sstar * N;
#pragma unroll
                    for (int r = 0; r < E; ++r) {
                        V cc = cvec[r];
                        if (a.conj) cc.y = -cc.y;
                        const V old = yo[t + P * r];
                        yo[t + P * r] = V{old.x + a.scale * cc.x, old.y + a.scale * cc.y};
                    }
                } else if (action == 2) {
                    // stored domain: y_b* = scale * cj(W x_s) - sum_{b != b*} y_b
#pragma unroll
                    for (int r = 0; r < E; ++r) {
                        V vv = xs[r];
                        if (a.conj) vv.y = -vv.y;
                        cvec[r] = V{a.scale * vv.x, a.scale * vv.y};
                    }
                    for (int b = 0; b < a.T; ++b) {
                        const long long sb = sig0 + (long long)b * sig_step;
                        if (b == bstar || sb >= a.batch) continue;
                        const V* yb = y + sb * N;
#pragma unroll
                        for (int r = 0; r < E; ++r) cvec[r] = csub(cvec[r], yb[t + P * r]);
                    }
                    V* yo = y + sstar * N;
#pragma unroll
                    for (int r = 0; r < E; ++r) {
                        rebuilt_ok = rebuilt_ok && cfin(cvec[r].x, cvec[r].y, a.cap);
                        yo[t + P * r] = cvec[r];
                    }
                }
                const unsigned bad =
                    slot_or<PL>((action == 2 && !rebuilt_ok) ? 1u : 0u, reinterpret_cast<unsigned*>(red));
                if (action == 2 && bad) ok = false;
                if ((action == 1 || action == 2) && t == 0) {
                    atomicAdd(&a.counts->detected, 1ull);
                    if (!ok) atomicAdd(&a.counts->uncorrectable, 1ull);
                    else if (action == 1) atomicAdd(&a.counts->corrected, 1ull);
                    else atomicAdd(&a.counts->rebuilt, 1ull);
                    atomicExch(&a.counts->last_signal, (unsigned long long)sstar);
                }
            }
            if (action == 3 && t == 0) {
                atomicAdd(&a.counts->detected, 1ull);
                atomicAdd(&a.counts->uncorrectable, 1ull);
            }
        }
    }
}

}  // namespace tfft
