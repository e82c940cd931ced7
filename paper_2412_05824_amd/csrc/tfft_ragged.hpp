// tfft_ragged.hpp -- one persistent launch for a ragged batch of mixed sizes.
//
// Every plan used for ragged batches has 256-lane workgroups, so one
// persistent kernel can run any of them.  The host turns the list of sizes
// into "classes" (one per size and pass) and a list of work items, ordered
// column passes first, then single-pass groups, then row passes.  Workgroups
// take items from an atomic queue in that order; a row-pass item first waits
// until every column-pass item of its signal has finished (a per-signal
// counter), which always happens because those items were handed out earlier
// and never wait themselves.  The queue and the counters reset themselves at
// the end of the launch, so the launch can be replayed from a captured graph
// without any memset node.
#pragma once

#include "tfft_registry.hpp"

namespace tfft {

constexpr int kRaggedThreads = 256;

struct RClass {
    KArgs<float2> args;      // batch = signals of the class, tables per class
    int plan;                // index into the ragged plan list
    int final_pass;          // 1: writes the transform's output (single or row pass)
    int src_ws, dst_ws;      // 1: read from / write to the workspace instead of x / y
    int nblocks;             // grid of the class
    int tiles;               // workgroups per signal (column/row passes)
    int cnt_base;            // first per-signal counter of this class (-1: none)
    int need;                // row pass: column-pass workgroups per signal to wait for
    int signal_after;        // column pass: 1 = bump the signal's counter when done
    int pair_tiles_b;        // column pass: row-pass workgroups per signal (for resets)
};

struct RItem {
    int cls;
    int blk;
};

struct RQueue {
    unsigned long long next;   // next item to hand out
    unsigned long long done;   // workgroups that have left the loop
};

struct RaggedArgs {
    // per call
    int conj;                  // 1: inverse direction
    int unit_scale;            // 1: scale 1 (else 1 forward, 1/N inverse)
    FtCounts* counts;
    long long inj_signal;      // global signal index (-1: none)
    long long inj_elem;
    int inj_part, inj_bit;
    int stats;
    // per plan
    const RClass* classes;
    const RItem* items;
    long long n_items;
    RQueue* q;
    unsigned* cnt_a;           // per signal: finished column-pass workgroups
    unsigned* cnt_b;           // per signal: row-pass workgroups that saw them all
    float2* ws;                // workspace for the column-pass results
};

using RaggedLaunchFn = hipError_t (*)(const void* x, void* y, const RaggedArgs& ra, int grid,
                                      hipStream_t stream);

// plan list shared by the registry and the persistent kernel (defined in
// inst_ragged.hip)
void register_fp32_ragged(std::vector<KernelEntry>& out);
RaggedLaunchFn ragged_launcher(int ft);
int ragged_max_blocks_per_cu(int ft);

}  // namespace tfft
