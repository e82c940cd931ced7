// tfft_device.hpp -- device building blocks for the batched C2C FFT on gfx950.
//
// Complex arithmetic on float2/double2, the in-register small DFTs used as
// radix-R butterflies (TurboFFT Sec. 3.1: thread-level radix-n macro kernels),
// padded LDS addressing (Sec. 3.2), and wavefront reductions for the ABFT
// checksums (Sec. 4.2).
//
// Contraction is explicit: every fused multiply-add of the transform is
// written as one (fmad) and the compiler forms no others, so that the
// arithmetic of a plan does not depend on the code around it; the checking
// kernels then store exactly the plain kernels' outputs.
//
// Every transform here is the forward DFT  y_k = sum_n x_n w^{kn},
// w = exp(-2 pi i / R)  (Sec. 2.2); the inverse is obtained by the caller by
// conjugating on load and on store.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#pragma clang fp contract(off)

namespace tfft {

constexpr int kWave = 64;

__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R> struct Vec;
template <> struct Vec<float>  { using type = float2; };
template <> struct Vec<double> { using type = double2; };

template <class V> struct RealOf;
template <> struct RealOf<float2>  { using type = float; };
template <> struct RealOf<double2> { using type = double; };

template <class V> __device__ __forceinline__ V cadd(V a, V b) { return V{a.x + b.x, a.y + b.y}; }
template <class V> __device__ __forceinline__ V csub(V a, V b) { return V{a.x - b.x, a.y - b.y}; }
template <class V> __device__ __forceinline__ V cmul(V a, V b) {
    return V{fmad(a.x, b.x, -(a.y * b.y)), fmad(a.x, b.y, a.y * b.x)};
}
// acc + a b
template <class V> __device__ __forceinline__ V cmac(V acc, V a, V b) {
    return V{fmad(a.x, b.x, fmad(-a.y, b.y, acc.x)), fmad(a.x, b.y, fmad(a.y, b.x, acc.y))};
}
// multiply by -i and +i
template <class V> __device__ __forceinline__ V mul_mi(V a) { return V{a.y, -a.x}; }
template <class V> __device__ __forceinline__ V mul_pi(V a) { return V{-a.y, a.x}; }
template <class V, class R> __device__ __forceinline__ V cscale(V a, R s) { return V{a.x * s, a.y * s}; }
template <class V> __device__ __forceinline__ V cconj(V a) { return V{a.x, -a.y}; }

// multiply by (c - i s), i.e. by exp(-i theta) with c = cos theta, s = sin theta
template <class V, class R> __device__ __forceinline__ V mul_cis(V a, R c, R s) {
    return V{fmad(a.x, c, a.y * s), fmad(a.y, c, -(a.x * s))};
}

// ---------------------------------------------------------------------------
// Small forward DFTs, natural order in and out.
// ---------------------------------------------------------------------------
#define TFFT_SQRT1_2 0.70710678118654752440084436210484903928483593768847
#define TFFT_COS_PI8 0.92387953251128675612818318939678828682241662586364
#define TFFT_SIN_PI8 0.38268343236508977172845998403039886676134456248563
#define TFFT_SQRT3_2 0.86602540378443864676372317075293618347140262690519

template <class V> __device__ __forceinline__ void dft2(V& a, V& b) {
    V t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// y = [a+s, a - s/2 - i(sqrt3/2)d, a - s/2 + i(sqrt3/2)d], s = b+c, d = b-c
template <class V> __device__ __forceinline__ void dft3(V& a, V& b, V& c) {
    using R = typename RealOf<V>::type;
    constexpr R h = (R)TFFT_SQRT3_2;
    V s = cadd(b, c);
    V d = csub(b, c);
    V t = V{fmad((R)-0.5, s.x, a.x), fmad((R)-0.5, s.y, a.y)};
    a = cadd(a, s);
    // t -/+ i (sqrt3/2) d
    b = V{fmad(h, d.y, t.x), fmad(-h, d.x, t.y)};
    c = V{fmad(-h, d.y, t.x), fmad(h, d.x, t.y)};
}

template <class V> __device__ __forceinline__ void dft4(V& a0, V& a1, V& a2, V& a3) {
    V t0 = cadd(a0, a2), t1 = csub(a0, a2);
    V t2 = cadd(a1, a3), t3 = mul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// multiply by w16^m = exp(-2 pi i m / 16), m known at compile time
template <int m, class V> __device__ __forceinline__ V w16(V a) {
    using R = typename RealOf<V>::type;
    constexpr int mm = m & 15;
    if constexpr (mm == 0) return a;
    else if constexpr (mm == 4) return mul_mi(a);
    else if constexpr (mm == 8) return V{-a.x, -a.y};
    else if constexpr (mm == 12) return mul_pi(a);
    else if constexpr (mm == 2) return V{(R)TFFT_SQRT1_2 * (a.x + a.y), (R)TFFT_SQRT1_2 * (a.y - a.x)};
    else if constexpr (mm == 6) return V{(R)TFFT_SQRT1_2 * (a.y - a.x), (R)(-TFFT_SQRT1_2) * (a.x + a.y)};
    else if constexpr (mm == 1) return mul_cis(a, (R)TFFT_COS_PI8, (R)TFFT_SIN_PI8);
    else if constexpr (mm == 3) return mul_cis(a, (R)TFFT_SIN_PI8, (R)TFFT_COS_PI8);
    else if constexpr (mm == 9) return mul_cis(a, (R)(-TFFT_COS_PI8), (R)(-TFFT_SIN_PI8));
    else {
        static_assert(mm == 0 || mm == 1 || mm == 2 || mm == 3 || mm == 4 || mm == 6 || mm == 8 ||
                          mm == 9 || mm == 12,
                      "unused w16 power");
        return a;
    }
}

template <class V> __device__ __forceinline__ void dft8(V (&v)[8]) {
    using R = typename RealOf<V>::type;
    constexpr R K = (R)TFFT_SQRT1_2;
    dft4(v[0], v[2], v[4], v[6]);
    dft4(v[1], v[3], v[5], v[7]);
    // y_k = E_k + w8^k O_k, y_{k+4} = E_k - w8^k O_k  (E_k in v[2k], O_k in v[2k+1]);
    // w8 O = K (O.x + O.y, O.y - O.x) and w8^3 O = K (O.y - O.x, -(O.x + O.y)),
    // the factor K fused into the butterfly
    const V e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6], o0 = v[1];
    const V o2 = mul_mi(v[5]);
    const R s1 = v[3].x + v[3].y, d1 = v[3].y - v[3].x;
    const R s3 = v[7].x + v[7].y, d3 = v[7].y - v[7].x;
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = V{fmad(K, s1, e1.x), fmad(K, d1, e1.y)};
    v[5] = V{fmad(-K, s1, e1.x), fmad(-K, d1, e1.y)};
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = V{fmad(K, d3, e3.x), fmad(-K, s3, e3.y)};
    v[7] = V{fmad(-K, d3, e3.x), fmad(K, s3, e3.y)};
}

// dft4 of (a0, a1, a2, a3) from its two half sums: t0 = a0 + a2,
// t1 = a0 - a2, t2 = a1 + a3, t3 = -i (a1 - a3)
template <class V> __device__ __forceinline__ void dft4_tail(V& a0, V& a1, V& a2, V& a3, V t0, V t1, V t2, V t3) {
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// 16 = 4 x 4: n = 4 n1 + n2, k = k1 + 4 k2
template <class V> __device__ __forceinline__ void dft16(V (&v)[16]) {
    using R = typename RealOf<V>::type;
    constexpr R K = (R)TFFT_SQRT1_2;
    dft4(v[0], v[4], v[8], v[12]);
    dft4(v[1], v[5], v[9], v[13]);
    dft4(v[2], v[6], v[10], v[14]);
    dft4(v[3], v[7], v[11], v[15]);
    // v[n2 + 4 k1] *= w16^{n2 k1}, then a 4-point DFT over n2 per k1; the
    // factor K of w16^2 and w16^6 (K (x + y, y - x), K (y - x, -(x + y)))
    // is fused into the first additions
    dft4(v[0], v[1], v[2], v[3]);
    {   // k1 = 1: w16^1, w16^2, w16^3
        const V a1 = w16<1>(v[5]), a3 = w16<3>(v[7]);
        const R s = v[6].x + v[6].y, d = v[6].y - v[6].x;
        const V a0 = v[4];
        const V t0 = V{fmad(K, s, a0.x), fmad(K, d, a0.y)};
        const V t1 = V{fmad(-K, s, a0.x), fmad(-K, d, a0.y)};
        dft4_tail(v[4], v[5], v[6], v[7], t0, t1, cadd(a1, a3), mul_mi(csub(a1, a3)));
    }
    {   // k1 = 2: w16^2, w16^4, w16^6
        const R s1 = v[9].x + v[9].y, d1 = v[9].y - v[9].x;
        const R s3 = v[11].x + v[11].y, d3 = v[11].y - v[11].x;
        const V a0 = v[8], a2 = mul_mi(v[10]);
        // a1 + a3 = K (s1 + d3, d1 - s3); -i (a1 - a3) = K (d1 + s3, d3 - s1)
        const V t2 = V{K * (s1 + d3), K * (d1 - s3)};
        const V t3 = V{K * (d1 + s3), K * (d3 - s1)};
        dft4_tail(v[8], v[9], v[10], v[11], cadd(a0, a2), csub(a0, a2), t2, t3);
    }
    {   // k1 = 3: w16^3, w16^6, w16^9
        const V a1 = w16<3>(v[13]), a3 = w16<9>(v[15]);
        const R s = v[14].x + v[14].y, d = v[14].y - v[14].x;
        const V a0 = v[12];
        const V t0 = V{fmad(K, d, a0.x), fmad(-K, s, a0.y)};
        const V t1 = V{fmad(-K, d, a0.x), fmad(K, s, a0.y)};
        dft4_tail(v[12], v[13], v[14], v[15], t0, t1, cadd(a1, a3), mul_mi(csub(a1, a3)));
    }
    // group k1 holds y[k1 + 4 k2] in v[4 k1 + k2]: transpose the 4x4 index
    V t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[i];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
        for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[4 * k1 + k2];
}

template <int R, class V> __device__ __forceinline__ void dft(V (&v)[R]) {
    if constexpr (R == 1) {
    } else if constexpr (R == 2) dft2(v[0], v[1]);
    else if constexpr (R == 3) dft3(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8(v);
    else if constexpr (R == 16) dft16(v);
    else static_assert(R == 2, "unsupported radix");
}

// ---------------------------------------------------------------------------
// Synchronisation of LDS exchanges.
// ---------------------------------------------------------------------------
// Within one wavefront LDS operations execute in order, so a wavefront-scope
// fence plus a code-motion barrier is enough between a store and a load.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool BLOCK> __device__ __forceinline__ void lds_sync() {
    if constexpr (BLOCK) __syncthreads();
    else wave_lds_sync();
}

// Padded LDS index: one spare element after every 2^B elements (a 128-byte
// row), so that lanes writing with a stride of 2^B elements hit distinct
// banks.  Strides that are multiples of 2^B stay compile-time offsets.
template <int B> __device__ __forceinline__ int pad_idx(int g) { return g + (g >> B); }
template <int B> constexpr int padded_size(int n) { return n + (n >> B) + 1; }

// ---------------------------------------------------------------------------
// Cross-lane exchange v[lane ^ X] inside a wave, on the VALU where possible:
// DPP quad permutes for X = 1, 2; ds_swizzle (bit-mask mode, no LDS memory
// access) for X = 4, 8, 16; ds_bpermute only for X = 32.
// ---------------------------------------------------------------------------
template <int X> __device__ __forceinline__ int xor_lane_i32(int v) {
    static_assert(X == 1 || X == 2 || X == 4 || X == 8 || X == 16 || X == 32, "xor offset");
    if constexpr (X == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    else if constexpr (X == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false); // quad_perm [2,3,0,1]
    else if constexpr (X < 32) return __builtin_amdgcn_ds_swizzle(v, (X << 10) | 0x1F);  // lane ^ X within 32
    else return __builtin_amdgcn_ds_bpermute((int)((__lane_id() ^ 32u) << 2), v);
}
template <int X> __device__ __forceinline__ float xor_lane(float v) {
    return __int_as_float(xor_lane_i32<X>(__float_as_int(v)));
}
template <int X> __device__ __forceinline__ double xor_lane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = xor_lane_i32<X>((int)(b & 0xffffffffll));
    const int hi = xor_lane_i32<X>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int X> __device__ __forceinline__ unsigned xor_lane(unsigned v) {
    return (unsigned)xor_lane_i32<X>((int)v);
}

// v op v[lane ^ X] for X = FROM, 2 FROM, ..., < TO (powers of two).  Every
// step pairs two lanes that combine the same two values, so all lanes of a
// group end with bit-identical results.
template <int FROM, int TO, class Op, class T> __device__ __forceinline__ T xor_reduce(T v) {
    if constexpr (FROM < TO) {
        v = Op::f(v, xor_lane<FROM>(v));
        return xor_reduce<FROM * 2, TO, Op>(v);
    } else {
        return v;
    }
}

struct OpAdd {
    template <class T> __device__ __forceinline__ static T f(T a, T b) { return a + b; }
};
struct OpOr {
    __device__ __forceinline__ static unsigned f(unsigned a, unsigned b) { return a | b; }
};

template <class T> __device__ __forceinline__ bool finite_le(T v, T cap) {
    return __builtin_fabs(v) <= cap;   // false for NaN and +-Inf
}

}  // namespace tfft
