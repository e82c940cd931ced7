// tfft_ragged_plans.hpp -- the plan list for ragged batches (fp32).
//
// Every plan runs 256-lane workgroups so that one persistent kernel can
// execute any of them.  The plans are deliberately light (8 elements per lane
// for 2^k lengths, 12 for 3*2^k lengths, 4 for 1024 and 6 for 1536, where
// 256 lanes must cover one signal): the persistent kernel
// holds all of them in one function, whose register allocation is that of
// the heaviest, and it must keep two workgroups per CU resident.  Lengths
// without a single-pass plan here run as a column pass of length N1 and a
// row pass of length N2 (N = N1 * N2, N1 <= N2, N1 as large as possible,
// each pass's sub-signals per tile dividing the other length).
//
// X(id, kind, Ns, E, WC, B, radices...)   (WC: waves for single plans,
// sub-signals per tile for column / row passes)
#pragma once

#define TFFT_RAGGED_SINGLE_PLANS(X)                          \
    X(0, kSingle, 64, 8, 4, 4, 8, 8)                         \
    X(1, kSingle, 128, 8, 4, 4, 2, 8, 8)                     \
    X(2, kSingle, 256, 8, 4, 4, 4, 8, 8)                     \
    X(3, kSingle, 512, 8, 4, 4, 8, 8, 8)                     \
    X(4, kSingle, 1024, 4, 4, 4, 4, 4, 4, 4, 4)              \
    X(5, kSingle, 2048, 8, 4, 4, 4, 8, 8, 8)                 \
    X(6, kSingle, 192, 12, 4, 4, 3, 4, 4, 4)                 \
    X(7, kSingle, 384, 12, 4, 4, 3, 4, 4, 4, 2)              \
    X(8, kSingle, 768, 12, 4, 4, 3, 4, 4, 4, 4)              \
    X(9, kSingle, 1536, 6, 4, 4, 3, 2, 2, 2, 2, 2, 2, 2, 2, 2) \
    X(10, kSingle, 3072, 12, 4, 4, 3, 4, 4, 4, 4, 4)

#define TFFT_RAGGED_TILES_PLANS(X)                   \
    X(11, kColPass, 64, 8, 32, 0, 8, 8)              \
    X(12, kColPass, 96, 12, 32, 0, 3, 4, 4, 2)       \
    X(13, kColPass, 128, 8, 16, 0, 2, 8, 8)          \
    X(14, kColPass, 192, 12, 16, 0, 3, 4, 4, 4)      \
    X(15, kColPass, 256, 8, 8, 0, 4, 8, 8)           \
    X(16, kColPass, 384, 12, 8, 0, 3, 4, 4, 4, 2)    \
    X(17, kRowPass, 64, 8, 32, 0, 8, 8)              \
    X(18, kRowPass, 96, 12, 32, 0, 3, 4, 4, 2)       \
    X(19, kRowPass, 128, 8, 16, 0, 2, 8, 8)          \
    X(20, kRowPass, 192, 12, 16, 0, 3, 4, 4, 4)      \
    X(21, kRowPass, 256, 8, 8, 0, 4, 8, 8)           \
    X(22, kRowPass, 384, 12, 8, 0, 3, 4, 4, 4, 2)    \
    X(23, kRowPass, 512, 8, 4, 0, 8, 8, 8)

#define TFFT_RAGGED_PLANS(X) TFFT_RAGGED_SINGLE_PLANS(X) TFFT_RAGGED_TILES_PLANS(X)

#define TFFT_PLAN_T(id, kind, Ns, E, WC, B, ...) Plan<kind, Ns, E, WC, B, __VA_ARGS__>
