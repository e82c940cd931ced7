// tfft_offline.hpp -- host interface of the offline (unfused) ABFT kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace tfft {

constexpr int kOfflineT = 16;   // signals per right-side sum of the offline scheme

struct OfflineArgs {
    const void* x;     // inputs (batch x N)
    void* y;           // outputs
    long long N, batch;
    const void* left;  // a = e^T W of length N (the library's table)
    int M;             // encoding period (3, or 5 when 3 | N)
    int conj;          // inverse direction: conjugate in and out
    double scale;      // output scale
    double tau_coef;   // kappa u sqrt(N log2 N)
    void* cs;          // 2 * batch complex double: p, then q
    void* nu;          // batch doubles
    void* xs;          // ceil(batch / kOfflineT) x N complex: right-side sums, transformed in place
    void* flags;       // batch ints
    void* counts;      // tfft_ft_counts (device)
};

// step 0: input pass; 1: output pass and check; 2: fix
template <class V> hipError_t offline_launch(const OfflineArgs& o, hipStream_t s, int step);

}  // namespace tfft
