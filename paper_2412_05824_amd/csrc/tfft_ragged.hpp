// tfft_ragged.hpp -- one persistent launch for a ragged batch of mixed sizes.
//
// Every plan used for ragged batches has 256-lane workgroups, so one
// persistent kernel can run any of them.  The host turns the list of sizes
// into "classes" (one per size and pass) and a list of work items, ordered
// column passes first, then single-pass groups, then row passes.  Workgroups
// take items from an atomic queue in that order; a row-pass item first waits
// until every column-pass item of its group of signals has finished (a
// per-group counter), which always happens because those items were handed
// out earlier and never wait themselves.  The queue and the counters reset
// themselves at the end of the launch, so the launch can be replayed from a
// captured graph without any memset node.
#pragma once

#include "tfft_registry.hpp"

namespace tfft {

// Default bound on the polls of one wait (a poll is a device-scope load plus
// a short sleep, about a microsecond): far beyond any column pass, so it only
// ends a wait whose counters are out of step.  It sets the error bit, and
// every later wait of the launch gives up at once, so even a broken schedule
// drains the queue in bounded time instead of hanging.  The last workgroup
// out reports the error (counts->sched_errors and the plan's sticky count),
// clears it and zeroes every counter, so the next launch starts in step.
constexpr unsigned kMaxPolls = 1u << 20;

constexpr int kRaggedThreads = 256;
constexpr int kRaggedSlotBytes = 16;   // LDS slot for the item index, ahead of the plan's LDS

struct RClass {
    KArgs<float2> args;      // batch = signals of the class, per-signal offset tables
    int plan;                // index into the ragged plan list
    int final_pass;          // 1: writes the transform's output (single or row pass)
    int src_ws, dst_ws;      // 1: read from / write to the workspace instead of x / y
    int nblocks;             // grid of the class
    int tiles;               // workgroups per group of signals (column / row passes)
    int cnt_base;            // first per-group counter of this class (-1: none)
    int need;                // row pass: column-pass items per group to wait for
    int signal_after;        // column pass: 1 = bump the group's counter when done
    int items_per_group;     // column / row passes: items covering one group
};

// A work item: blocks [blk, blk + nblk) of one class, never straddling two
// groups of signals of a column / row pass.  With a windowed workspace, a
// row-pass item counts itself into its batch (batch >= 0) and a column-pass
// item first waits until wait_need row-pass items of batch wait_batch have
// finished reading the workspace half it is about to overwrite.
struct RItem {
    int cls;
    int blk;
    int nblk;
    int batch;
    int wait_batch;
    int wait_need;
    int pad0, pad1;
};

struct RQueue {
    unsigned long long next;   // next item to hand out
    unsigned long long done;   // workgroups that have left the loop
    unsigned long long err;    // bit 0: a wait of this launch gave up (cleared at its end)
    unsigned long long err_launches;   // launches that ended with err set (sticky)
};

// Device-resident description of one ragged plan, written once by the host.
struct RaggedDesc {
    const RClass* classes;
    const RItem* items;
    long long n_items;
    RQueue* q;
    unsigned* cnt_a;           // per group: finished column-pass workgroups
    unsigned* cnt_b;           // per group: row-pass items past their wait
    unsigned* cnt_r;           // per batch: finished row-pass items (windowed workspace)
    long long n_batches;
    long long n_groups;        // entries of cnt_a and cnt_b
    float2* ws;                // column-pass results of the two-pass signals
};

// Per-launch arguments.
struct RaggedCall {
    const float2* x;
    float2* y;
    FtCounts* counts;
    long long inj_signal;      // global signal index (-1: none)
    long long inj_signal2;     // a second signal hit the same way (-1: none)
    long long inj_elem;
    int inj_part, inj_bit;
    int inj_pass;              // -1 last pass, 0 single / column pass, 1 row pass
    int inj_stage;             // -1 after the last radix stage
    int conj;                  // 1: inverse direction
    int unit_scale;            // 1: scale 1 (else 1 forward, 1/N inverse)
    int stats;
    unsigned max_polls;        // bound of one wait (polls)
    unsigned wait_extra;       // test hook: added to what every wait needs (0)
    int pad;
};

using RaggedLaunchFn = hipError_t (*)(const RaggedCall& c, const RaggedDesc* d, int grid,
                                      hipStream_t stream);

struct RaggedKernel {
    RaggedLaunchFn launch;
    int lds_bytes;        // dynamic LDS per workgroup
    int blocks_per_cu;    // resident workgroups per CU (0: query failed)
};

// registry entries of the ragged plans (k_fft with offset tables: the
// per-size launches) and the persistent kernel per ABFT mode
void register_fp32_ragged_single(std::vector<KernelEntry>& out);
void register_fp32_ragged_tiles(std::vector<KernelEntry>& out);
// waves: 0 = the compiler's register budget, 3 = held to three workgroups per CU
RaggedKernel ragged_kernel_ft0(int waves);
RaggedKernel ragged_kernel_ft1(int waves);
RaggedKernel ragged_kernel_ft2(int waves);

}  // namespace tfft
