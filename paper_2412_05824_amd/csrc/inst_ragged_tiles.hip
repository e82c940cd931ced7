// Registry entries (k_fft launches with per-signal offset tables) of the ragged tiles plans.
#include "tfft_ragged.hpp"
#include "tfft_ragged_plans.hpp"

namespace tfft {

#define TFFT_CHECK_THREADS(id, kind, Ns, E, WC, B, ...)                                            \
    static_assert(TFFT_PLAN_T(id, kind, Ns, E, WC, B, __VA_ARGS__)::THREADS == kRaggedThreads, \
                  "ragged plan width");
TFFT_RAGGED_TILES_PLANS(TFFT_CHECK_THREADS)
#undef TFFT_CHECK_THREADS

void register_fp32_ragged_tiles(std::vector<KernelEntry>& out) {
#define TFFT_REG(id, kind, Ns, E, WC, B, ...)                                \
    {                                                                         \
        using PL = TFFT_PLAN_T(id, kind, Ns, E, WC, B, __VA_ARGS__);          \
        KernelEntry e0 = make_entry<float2, PL, 0, true, __VA_ARGS__>(0);           \
        KernelEntry e1 = make_entry<float2, PL, 1, true, __VA_ARGS__>(0);           \
        KernelEntry e2 = make_entry<float2, PL, 2, true, __VA_ARGS__>(0);           \
        e0.ragged_id = e1.ragged_id = e2.ragged_id = id;                      \
        out.push_back(e0);                                                    \
        out.push_back(e1);                                                    \
        out.push_back(e2);                                                    \
    }
    TFFT_RAGGED_TILES_PLANS(TFFT_REG)
#undef TFFT_REG
}

}  // namespace tfft
