// bat_launch.hpp -- host-side launchers for the ahead-of-time kernels in
// bat_kernels.hip (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "bat_device.hpp"

namespace batk {

// ---- batched form: many graphs x many probability vectors in one launch.
// wavefronts per block (one block per CU: LDS-bound): 3 per SIMD while the
// reach words, which persist across a chained block, fit beside the 32
// accumulators in 168 VGPRs, else 2
constexpr int batch_waves(int nmax) { return nmax <= 16 ? 12 : 8; }
// the same for the transposed accumulation (k_batched_dyn_t: one
// accumulator per lane, 118 VGPRs at 16 nodes, about 150 above)
constexpr int batch_waves_t(int nmax) { return nmax <= 16 ? 16 : 12; }
constexpr int kBatchWavesMax = 12;
constexpr int kBatchMaxP = 32;                  // probability vectors per entry
constexpr int kBatchSegLog = 6;                 // iterations per wavefront work unit: 2^f
static_assert(kBatchMaxP == bat::kBatchCols, "partial slot layout of the batched sweeps");
static_assert((1 << kBatchSegLog) <= bat::kBatchQlo, "Q_lo table of the specialised batched sweep");

// One (graph, group of <= 32 probability vectors).  Its work is split into
// items of batch_waves(nmax) * 2^f iterations; items of all entries form one
// queue.
struct BatchEntry {
    bat::u32 m, ubits, f, P;
    bat::u32 n_nodes, s, t, n_relax;
    bat::u32 prog_off;    // into the concatenated relaxation programs (u32s)
    bat::u32 n_groups;    // relaxation groups of 4 per sweep direction
    bat::u32 graph, pv_base;
    bat::u32 chain;       // k: warm-started chains over the k lowest iteration bits (0: none)
    bat::u32 ck_code[6];  // relaxation code of counter bit 11 + b (~0: pruned)
    bat::u64 item_begin, n_items;
    bat::u64 tab_off;     // doubles: P consecutive forward table blocks
};

struct BatchParams {
    const BatchEntry *entries;
    const bat::u64 *item_start;   // [n_entries + 1], ascending
    bat::u32 n_entries, check_every;
    bat::u64 n_items;
    const bat::u32 *prog;         // concatenated relaxation programs (bat::KParams::prog)
    const double *tables;
    double *part;                 // [n_items][kBatchMaxP][2]
    bat::u64 *pcount;             // [n_items]
    unsigned long long *ctr;      // work queue head (zeroed before launch)
};

hipError_t batched_tables(hipStream_t st, const BatchEntry *entries, const bat::u32 *pair_entry,
                          const bat::u32 *pair_pv, const bat::u64 *entry_p_off, const double *p, unsigned n_pairs,
                          double *tables);
// transposed: the kernel with the transposed accumulation (k_batched_dyn_t)
hipError_t batched_sweep(hipStream_t st, unsigned blocks, int nmax, bool transposed, const BatchParams &B);
hipError_t batched_reduce(hipStream_t st, const BatchEntry *entries, unsigned n_entries, const double *part,
                          const bat::u64 *pcount, bat::u32 n_pvec, double *R, bat::u64 *counts);

// ---- multi-state arcs (bat_ms.hip)
constexpr int kMsMaxArcs = 32;     // arc masks and reach sets are 32-bit words
// slots of the kernel instance that sweeps m arcs (the rest padded): 16,
// 20, 24 or 32; up to 20 slots the kernel fits 4 wavefronts per SIMD
constexpr int ms_slots(int m) { return m <= 16 ? 16 : m <= 20 ? 20 : m <= 24 ? 24 : 32; }
constexpr int kMsMaxNodes = 32;
constexpr int kMsMaxStates = 32;   // per arc
constexpr int kMsMaxTable = 1024;  // sum of the arcs' state counts (LDS tables)
constexpr int kMsMaxDemand = 1024;
constexpr int kMsMaxCapacity = 1 << 20;

struct MsParams {
    bat::u64 c_lo, c_hi;   // index range of the mixed-radix counter (slot 0 least significant)
    bat::u64 run;          // consecutive indices per lane in a work item
    bat::u64 n_items;      // wavefront work items: item i covers [c_lo + 64 i run, c_lo + 64 (i+1) run)
    bat::u32 m, n, s, t, d, directed;
    bat::u32 n_table;      // sum of the state counts
    bat::u32 warm;         // 1: slot 0's capacity is nondecreasing in its state
    bat::u32 sig[kMsMaxArcs];  // states of the arc in slot i (sweep position i)
    bat::u32 off[kMsMaxArcs];  // its first table entry
    unsigned char u[kMsMaxArcs], v[kMsMaxArcs];
    const int *cap;        // [n_table] capacity of (slot, state), slot 0's states first
    const double *w;       // [n_table] probability of (arc, state)
    double *part;          // [n_items][2] double-double partials
    bat::u64 *pcount;      // [n_items]
};
hipError_t ms_sweep(hipStream_t st, unsigned blocks, const MsParams &P);

hipError_t build_tables(hipStream_t st, const double *p, const unsigned char *row, bat::u32 m, bat::u32 f,
                        double *T, int *status);
hipError_t sweep_dyn(hipStream_t st, unsigned blocks, bool grad, int nmax, bool directed, const bat::KParams &K);
hipError_t reduce(hipStream_t st, const double *part, const bat::u64 *pcount, bat::u64 n_chunks, bat::u32 ncol,
                  double *res, bat::u64 *count);
// the diagnostic VALU-rate kernel: `blocks` blocks of 256 threads, `iters`
// loop trips of kValuPeakOpsPerTrip VALU instructions each; sink: 64 u32s
constexpr int kValuPeakOpsPerTrip = 16;
hipError_t valu_peak(hipStream_t st, unsigned blocks, bat::u32 iters, bat::u32 *sink);
hipError_t finalize(hipStream_t st, const double *res, const bat::u64 *count, const int *status,
                    const unsigned char *cb_of_arc, bat::u32 m, bool grad, double *R, bat::u64 *cnt, double *dRdp,
                    double *T1, double *T0, int *status_out);

}  // namespace batk
