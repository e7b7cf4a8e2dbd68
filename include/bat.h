/*
 * bat.h -- C ABI of the MI355X (gfx950) library for exact two-terminal
 * reliability of binary-state networks by exhaustive binary-addition-tree
 * enumeration (BAT, Yeh, arXiv 2209.09711).
 *
 * What every entry point computes (Section 3, Eq. 1):
 *
 *   R = sum over all X in {0,1}^m with s ~ t in G(X) of  prod_i q_i(x_i),
 *   q_i(1) = p_i,  q_i(0) = 1 - p_i,
 *
 * where G(X) keeps the arcs a_i with x_i = 1 (Section 2.2) and "s ~ t" is
 * the PLSA connectivity test of Section 3.2 (arcs are undirected).  The
 * feasible-vector count is the number of such X.  The enumeration order is
 * the paper's backward BAT (Section 3.1, Table 2): arc i (0-based) is the
 * coordinate x_{i+1}, the vector with 0-based index c has x_{i+1} = bit
 * (m-1-i) of c (Eq. 2-3), so arc 0 is the most significant coordinate.
 *
 * The gradient entry points add dR/dp_i = T1_i - T0_i, where T1_i (T0_i) is
 * R with p_i replaced by 1 (by 0): Eq. 1 is multilinear in p, so these are
 * the Birnbaum importances.  They come from the same sweep as R (each
 * connectivity verdict is reused), not from extra runs.
 *
 * Conventions for every function:
 *  - Nodes are 0-based ids in [0, n_nodes).  The paper's source 1 and sink n
 *    are passed explicitly as s and t (s != t).
 *  - arcs points to n_arcs pairs (u, v) (bat_arc), undirected.  Self-loops
 *    and parallel arcs are accepted (Eq. 1 is well defined for them; the
 *    paper's assumption of none restricts its benchmarks only).
 *  - p[i] is the working probability of arcs[i]; it must be finite and in
 *    [0, 1].
 *  - Limits: 2 <= n_nodes <= BAT_MAX_NODES, 0 <= n_arcs <= BAT_MAX_ARCS.
 *    m = 0 is one empty, disconnected vector: R = 0, count = 0.
 *  - Return value: BAT_OK (0) or a negative BAT_E* code (and BAT_PENDING
 *    from bat_reliability_checkpointed).  On error the outputs are left
 *    untouched and bat_last_error() describes the failure.
 *  - Ownership: the caller owns every buffer.  The library copies what it
 *    needs during the call and keeps no pointer after it returns (for the
 *    _async functions: after the work queued on the stream has run).
 *  - Threads: calls are re-entrant; synchronous calls run on a per-thread
 *    stream of the current HIP device, _async calls on the stream given.
 *  - Memory: synchronous single-graph calls reuse a device workspace and a
 *    pinned host staging buffer kept per thread and device (grown when a
 *    call needs more, never shrunk; an exiting thread's go to later
 *    threads).  _async calls allocate their workspace on the given stream
 *    and free it there.
 *  - Results are deterministic: the same inputs give bitwise the same R,
 *    count and gradient on every run (fixed-order reductions, no
 *    floating-point atomics).
 */
#ifndef BAT_H
#define BAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BAT_OK 0
#define BAT_EINVAL (-1)  /* bad argument: sizes, node ids, s == t, p outside [0,1] or NaN, NULL */
#define BAT_ETOOBIG (-2) /* n_nodes > BAT_MAX_NODES or n_arcs > BAT_MAX_ARCS */
#define BAT_EDEVICE (-3) /* HIP runtime or JIT compiler error; text in bat_last_error() */
#define BAT_ENOMEM (-4)  /* host or device allocation failed */
#define BAT_EIO (-5)     /* a checkpoint file could not be read, parsed or written */
#define BAT_PENDING 1    /* bat_reliability_checkpointed: chunks remain (not an error) */

#define BAT_MAX_NODES 64
#define BAT_MAX_ARCS 62

typedef struct {
    int32_t u, v;
} bat_arc;

/* Library version string, e.g. "bat-mi355x 0.1.0". */
const char *bat_version(void);

/* Text of the last error raised on the calling thread ("" if none). */
const char *bat_last_error(void);

/*
 * Exact reliability R and feasible-vector count of G(V, E, D_b) between s
 * and t (Eq. 1 over all 2^m vectors).  Host pointers; blocks until done.
 */
int bat_reliability(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                    int32_t s, int32_t t, double *R_out, uint64_t *count_out);

/*
 * As bat_reliability, plus dR/dp (n_arcs doubles) from the same sweep.
 * T1_out and T0_out (n_arcs doubles each, may be NULL) receive T1_i =
 * R|p_i<-1 and T0_i = R|p_i<-0; dRdp_out[i] = T1_i - T0_i.
 */
int bat_reliability_grad(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                         int32_t s, int32_t t, double *R_out, uint64_t *count_out,
                         double *dRdp_out, double *T1_out, double *T0_out);

/*
 * Partial sums over the 0-based backward-order indices [c_lo, c_hi) of the
 * 2^m vectors (c_lo <= c_hi <= 2^m).  The equal divisions of Section 4 (Eq.
 * 6: division i of chi holds indices [(i-1) mu, i mu), mu = 2^m / chi) are
 * such ranges, so a long sweep can be split into checkpointed chunks or
 * shards and the parts added afterwards.  The sum is returned unevaluated
 * as a double-double (*R_hi + *R_lo).  T1_out / T0_out (n_arcs doubles each)
 * may both be NULL (no gradient) or both non-NULL (gradient partials,
 * collapsed to doubles).
 */
int bat_reliability_range(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                          int32_t s, int32_t t, uint64_t c_lo, uint64_t c_hi,
                          double *R_hi, double *R_lo, uint64_t *count_out,
                          double *T1_out, double *T0_out);

/*
 * Variants (flags, OR-ed):
 *   BAT_DIRECTED       arcs are directed, u -> v: f(X) = 1 iff G(X) has a
 *                      directed s -> t path (the "directed path" wording of
 *                      the layered search, Section 3.2).  The paper's own
 *                      results are for the undirected reading.
 *   BAT_FORWARD_ORDER  range indices follow the forward BAT (Section 4.2,
 *                      Eq. 4-5): x_1 is the least significant bit of the
 *                      0-based index, arc i is bit i.  Without it, indices
 *                      follow the backward BAT of Section 3.1 (Eq. 2-3).
 *                      A whole sweep does not depend on the order.
 * Unknown flag bits return BAT_EINVAL.
 */
#define BAT_DIRECTED 1u
#define BAT_FORWARD_ORDER 2u

/*
 * bat_reliability / bat_reliability_grad with flags.  dRdp_out, T1_out and
 * T0_out (n_arcs doubles each) are each nullable; the gradient sweep runs
 * when any of them is set.  Same errors as above.
 */
int bat_reliability_ex(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                       int32_t s, int32_t t, uint32_t flags, double *R_out, uint64_t *count_out,
                       double *dRdp_out, double *T1_out, double *T0_out);

/*
 * bat_reliability_range with flags: [c_lo, c_hi) in the index order the
 * flags select.
 */
int bat_reliability_range_ex(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                             int32_t s, int32_t t, uint32_t flags, uint64_t c_lo, uint64_t c_hi,
                             double *R_hi, double *R_lo, uint64_t *count_out,
                             double *T1_out, double *T0_out);

/*
 * A whole sweep, as bat_reliability_ex, run in chunks of about
 * 2^chunk_log2 vectors each (0 <= chunk_log2 <= BAT_MAX_ARCS; chunk_log2 >=
 * n_arcs gives one chunk), each chunk one call's worth of work.  The whole
 * sweep's work items (blocks of the counter, the way a single call would
 * cut it) are dealt out into J = 2^(n_arcs - chunk_log2) parts (fewer if
 * the sweep has fewer work items): part j holds the blocks whose index is
 * j modulo J.  So every chunk spans the whole counter, with the same mix
 * of cheap and costly regions as a whole sweep, and runs about as fast per
 * vector.  Contiguous divisions (Eq. 6 of Section 4, as
 * bat_reliability_range computes them) are not used here.  The arc-to-bit
 * order, the work-item size and the chain length are those the whole
 * sweep would take (tuned, else the defaults; with BAT_FORWARD_ORDER, the
 * forward BAT order of Section 4.2).  The first chunk fixes them, and the
 * checkpoint file keeps them, so a resumed sweep uses them too.  Chunks
 * are added in order: R and each T1_i, T0_i as double-doubles, the count
 * exactly.  The result therefore depends on that launch only through
 * rounding, and not at all on how the chunks are spread over calls.
 *
 *   path        NULL, or a checkpoint file.  After each chunk the running
 *               sums are written to path + ".tmp", flushed to disk and
 *               renamed over path (readers see the old file or the new
 *               one, whole).  A later call for the same problem resumes
 *               after the last chunk the file holds; a finished file
 *               returns its result without touching the device.  The file
 *               is text: a format line, a line naming the problem (n_nodes,
 *               n_arcs, s, t, flags, chunk_log2, whether gradient sums are
 *               kept, 64-bit FNV-1a hashes of the arc list and of p's
 *               bytes), the part count, the launch (arc order kind,
 *               work-item size and chain length as bat_last_launch reports
 *               them), the parts done, the count, then R and the per-arc T1
 *               and T0 as hexadecimal floating-point pairs (hi lo).
 *               The caller owns the file; it is kept after the sweep
 *               ends.
 *   max_chunks  run at most this many chunks in this call (< 0: no limit),
 *               so one call's time can be bounded.
 *   dRdp_out, T1_out, T0_out  nullable, n_arcs doubles each; gradient sums
 *               are kept when any is set (and are part of the problem).
 *
 * Returns BAT_OK with every output set once all chunks are done, or
 * BAT_PENDING with the outputs untouched while chunks remain (or when no
 * file exists and max_chunks is 0: nothing has run).  A file naming
 * another problem is BAT_EINVAL and is left as it is; a file that cannot be
 * read, parsed or replaced is BAT_EIO.  Other errors as for
 * bat_reliability_ex; the file then holds the chunks finished before the
 * failing one.  Two calls must not share one file at the same time.
 */
int bat_reliability_checkpointed(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                                 int32_t s, int32_t t, uint32_t flags, int32_t chunk_log2,
                                 const char *path, int64_t max_chunks,
                                 double *R_out, uint64_t *count_out,
                                 double *dRdp_out, double *T1_out, double *T0_out);

/*
 * Many networks, many probability vectors, one persistent launch.
 * Graph g has n_nodes[g] nodes and the arcs arcs[arc_offsets[g] ..
 * arc_offsets[g+1]) (arc_offsets has n_graphs + 1 entries, arc_offsets[0]
 * = 0), source s[g], sink t[g].  Each graph has n_pvec probability vectors:
 * p holds, graph after graph, an n_pvec x m_g row-major block (arc fastest),
 * i.e. graph g's block starts at n_pvec * arc_offsets[g].  One connectivity
 * verdict per state vector serves all n_pvec probability vectors of its
 * graph (in groups of up to 32 per pass over the graph's vectors).  Work
 * items (graph, counter range) are queued largest graph first and taken by
 * one persistent block per compute unit.  Outputs: R_out[g * n_pvec + j]
 * and counts_out[g], host pointers.  Limits per graph as above;
 * 1 <= n_pvec <= BAT_MAX_PVEC.  Blocks until done.
 */
#define BAT_MAX_PVEC 1024
int bat_reliability_batched(int32_t n_graphs, const int32_t *n_nodes, const int32_t *arc_offsets,
                            const bat_arc *arcs, const int32_t *s, const int32_t *t,
                            int32_t n_pvec, const double *p, double *R_out, uint64_t *counts_out);

/*
 * Autotuner for the batched launch: runs this batch (same arguments as
 * bat_reliability_batched, results discarded) with each candidate number
 * of chained iteration bits (0, 3..6) and per-wavefront segment size
 * (2^4..2^6 iterations), then with graph-specialised kernels for the
 * graphs of at least m_max - 4, m_max - 2 or m_max arcs (m_max: the
 * batch's largest arc count; compile time is not counted), and caches the
 * fastest under the batch's structure (graphs, terminals, n_pvec; not p).
 * Each threshold is measured with 3, 2 and 1 side streams
 * ("BAT_BATCH_STREAMS"); a specialised candidate must be 2% faster than
 * the best generic one.  Later batched calls with that structure use the
 * choice while "BAT_AUTOTUNE" is 1 ("BAT_CHAIN_LOG2", "BAT_BATCH_JIT_ARCS"
 * and "BAT_BATCH_STREAMS", when not -1, override its parts).  *best_kernel_ms (may be NULL) receives the
 * best kernel time.
 * Results never depend on the choice beyond floating-point rounding.
 */
int bat_autotune_batched(int32_t n_graphs, const int32_t *n_nodes, const int32_t *arc_offsets,
                         const bat_arc *arcs, const int32_t *s, const int32_t *t, int32_t n_pvec,
                         const double *p, double *best_kernel_ms);

/*
 * Stream-ordered forms for callers that keep p and the results in device
 * memory (e.g. PyTorch tensors).  arcs, n_nodes, s, t are host values; p_dev
 * (n_arcs doubles), R_dev (1 double), count_dev (1 uint64) and, for the
 * gradient form, dRdp_dev / T1_dev / T0_dev (n_arcs doubles each; T1_dev and
 * T0_dev may be NULL) are device pointers on the current device.  stream is
 * a hipStream_t (NULL = the default stream).  The call returns once the
 * work is queued; argument errors that need no device data are returned at
 * once.  p_dev is checked on the device: if any p is outside [0, 1] or NaN,
 * *R_dev is set to NaN and, when status_dev is non-NULL, *status_dev to
 * BAT_EINVAL (else BAT_OK).  Temporary device memory is taken from the
 * stream-ordered allocator and released on the stream.
 */
int bat_reliability_async(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs,
                          const double *p_dev, int32_t s, int32_t t, double *R_dev,
                          uint64_t *count_dev, int32_t *status_dev, void *stream);

int bat_reliability_grad_async(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs,
                               const double *p_dev, int32_t s, int32_t t, double *R_dev,
                               uint64_t *count_dev, double *dRdp_dev, double *T1_dev,
                               double *T0_dev, int32_t *status_dev, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * forward sweep of bat_reliability_async with the same arguments, the same
 * device-side check of p and results within rounding of it (1e-12
 * relative; the count is exact), run without any allocation.
 *
 * Its device workspace is a fixed array of BAT_NOALLOC_SCRATCH_BYTES bytes
 * inside the library, one per GPU, held from the first call on that GPU
 * until the process ends.  The call makes no hipMalloc, hipFree or other
 * device allocation: it runs the ahead-of-time kernels only (never a
 * run-time compiled one, whose module would take device memory), and work
 * items grow until their partial sums fit the array.  A problem whose sums
 * do not fit even then (about 2^53 or more state vectors) returns
 * BAT_ETOOBIG before anything is queued.  Every call's kernels write the
 * parts of the array they read, so no state carries over between calls.
 *
 * All calls on one GPU share its array: calls whose work overlaps on that
 * GPU (other threads, other streams, or queued work of an earlier call
 * still running on another stream) race and give wrong results.  Order
 * them, e.g. by using one stream.
 */
#define BAT_NOALLOC_SCRATCH_BYTES (8u << 20)

int bat_reliability_noalloc(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs,
                            const double *p_dev, int32_t s, int32_t t, double *R_dev,
                            uint64_t *count_dev, int32_t *status_dev, void *stream);

/*
 * Multi-state arcs.  The paper sizes the solution space of arcs with
 * sigma_i states as prod_i sigma_i (Section 4.1) and names multi-state
 * network reliability as the next problem (Section 6) without defining it;
 * these entry points take the multi-state flow network reading:
 *
 *   arc i is in state k (0 <= k < n_states[i]) with probability w_i(k) and
 *   then carries at most capacity_i(k) units of flow, in either direction
 *   (from u to v only with BAT_DIRECTED); a state vector X meets demand d
 *   when the maximum s-t flow is at least d;
 *   R_d = sum over X meeting d of prod_i w_i(x_i), count = their number.
 *
 * With two states of capacity 0 and 1 (w = 1 - p, p) and d = 1 this is the
 * binary problem of Eq. 1.  The vectors are enumerated by the BAT
 * generalised to mixed radix: index c (0-based) is the vector whose
 * coordinates, arc 0 most significant, are the digits of c in the bases
 * n_states[i]; the next vector raises the last coordinate below its top
 * state and returns every later one to state 0 (Rule 1 for sigma_i = 2).
 *
 * Arguments: n_states[n_arcs]; capacity and w hold sum(n_states) entries,
 * arc 0's states first (capacity NULL: state k has capacity k).  Limits:
 * n_nodes <= 32, n_arcs <= 32, 1 <= n_states[i] <= 32, sum(n_states) <=
 * 1024, capacities in [0, 2^20], 1 <= demand <= 1024, prod n_states <=
 * 2^62 (else BAT_ETOOBIG or BAT_EINVAL).  Each w_i(k) must lie in [0, 1];
 * they are used as given (the library does not check that an arc's sum is
 * 1).  flags: 0 or BAT_DIRECTED.  Host pointers; synchronous, on the
 * calling thread's stream; the same workspace rules as bat_reliability.
 *
 * bat_ms_reliability sweeps every vector (in any arc order it likes: R and
 * the count are sums).  With demand 1 to 3 both entry points decide the
 * flow test bit-sliced, up to 32 vectors per word, in a kernel compiled at
 * run time for the graph, its states and capacities (hiprtc, cached like
 * the other graph-specialised kernels; probabilities are run-time data):
 * by max-flow min-cut the flow reaches 1 when t is reachable from s over
 * the arcs of capacity >= 1, 2 when besides no single arc of capacity
 * exactly 1 separates s from t there, and 3 when no single arc of
 * capacity 1 or 2 and no two arcs of capacity 1 do.  Higher demands run
 * the augmenting-path kernel.  bat_ms_reliability_range sweeps indices
 * [c_lo, c_hi) in the order above and returns the partial sum as a
 * double-double (R_hi + R_lo) and its count.
 */
int bat_ms_reliability(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const int32_t *n_states,
                       const int32_t *capacity, const double *w, int32_t s, int32_t t, int32_t demand,
                       uint32_t flags, double *R_out, uint64_t *count_out);

int bat_ms_reliability_range(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs,
                             const int32_t *n_states, const int32_t *capacity, const double *w,
                             int32_t s, int32_t t, int32_t demand, uint32_t flags, uint64_t c_lo,
                             uint64_t c_hi, double *R_hi, double *R_lo, uint64_t *count_out);

/*
 * Tuning and diagnostics.
 *
 * bat_set_option / bat_get_option read and set process-wide knobs (also
 * settable through the environment variable of the same name at load):
 *   "BAT_JIT"          0 = never use graph-specialised kernels, 1 = always,
 *                      2 = automatic (default: when the problem is large)
 *   "BAT_CHUNK_LOG2"   log2 of the enumeration iterations per wavefront
 *                      work item (0 = automatic)
 *   "BAT_SEG_LOG2"     log2 of the iterations per probability segment
 *   "BAT_CHECK_EVERY"  1 = convergence test after every sweep, 2 = after
 *                      every forward+backward pair
 *   "BAT_AUTOTUNE"     1 = let bat_autotune's cached choices apply
 *   "BAT_PERM"         which arcs take the low counter bits in whole-range
 *                      sweeps: -1 = the tuned choice, else kind 3; 0 = the
 *                      paper's order, 1..3 = orders that put arcs near t on
 *                      the in-wavefront bits and pruned or mid-graph arcs on
 *                      the chained iteration bits (R and counts never
 *                      depend on it; the range entry point always uses the
 *                      paper's order)
 *   "BAT_CHAIN_LOG2"   -1 = tuned (else 3), 0 = no warm starts, 3..6: the
 *                      specialised forward sweep visits iterations in blocks
 *                      of 2^k along chains that switch one iteration arc on
 *                      per step, starting each step's closure from the
 *                      previous one (gradient sweeps use at most 4)
 *   "BAT_ITEM_ORDER"   which counter chunk each wavefront work item sweeps:
 *                      -1 or 1 = spread (item i takes chunk i times an odd
 *                      constant, modulo the chunk count, when that count is
 *                      a power of two, so work items running side by side
 *                      cover distant parts of the counter), 0 = counter
 *                      order; R and counts never depend on it beyond
 *                      floating-point rounding
 *   "BAT_MS_RUN"       consecutive state vectors each lane of the
 *                      multi-state augmenting-path sweep decides, and the
 *                      most words each lane of the bit-sliced sweep
 *                      (demand <= 2) steps through (0 = automatic)
 *   "BAT_MS_BITS"      1 (default) = multi-state sweeps with demand 1 to 3
 *                      run the bit-sliced kernel; 0 = always the
 *                      augmenting-path kernel
 *   "BAT_WINDOW_TEST"  1 (default) = the graph-specialised sweeps (R, and
 *                      R with the gradient) test each window of 2048 iterations once, with all
 *                      11 word arcs up, and skips the chained blocks whose
 *                      last iteration cannot connect s and t (none of their
 *                      vectors can); 0 = sweep every block.  Results are
 *                      identical either way
 *   "BAT_BLOCK_WAVES"  wavefronts per block of the graph-specialised
 *                      forward sweep: -1 = tuned (else 4), 1, 2 or 4
 *   "BAT_SUPER_RESTART" graph-specialised forward sweeps of graphs of up to
 *                      28 relevant nodes: 1 = keep each 64-iteration
 *                      super-block's bottom closure in LDS and resume later
 *                      block bottoms from it, 0 = solve block bottoms
 *                      afresh, -1 = tuned (else 0)
 *   "BAT_SIMD_WAVES"   graph-specialised forward sweep: compile it to fit
 *                      this many wavefronts per SIMD (5..8; the compiler
 *                      then keeps fewer registers and may spill), 0 = the
 *                      compiler's own budget, -1 = tuned (else 6)
 *   "BAT_KEEP_BOTTOM"  graph-specialised forward sweep: 1 = keep each
 *                      chained block's bottom closure in registers and
 *                      resume later chain starts from it, 2 = keep it in
 *                      LDS instead, 0 = solve chain starts afresh,
 *                      -1 = tuned (else 1)
 *   "BAT_GRAD_KEEP_BOTTOM" graph-specialised gradient sweep: 2 (default) =
 *                      keep each chained block's bottom closure in LDS and
 *                      resume later chain starts from it, 0 = solve chain
 *                      starts afresh
 *   "BAT_SERIES"       1 (default) = the graph-specialised kernels join two
 *                      arcs in series through a node of degree 2 (other
 *                      than s and t) into one relaxation with the AND of
 *                      their masks, which removes the node; 0 = relax
 *                      every arc.  Results are identical either way
 *   "BAT_BATCH_JIT_ARCS" batched form: graphs with at least this many arcs
 *                      (and at least 2^(11+f) vectors, f the segment size)
 *                      run their own graph-specialised kernel (compiled at
 *                      run time, one per graph and p-vector group, side by
 *                      side as for "BAT_JIT_PROCS"), the rest the generic
 *                      persistent kernel, in the same call; 0 = none,
 *                      -1 (default) = bat_autotune_batched's choice, else none
 *   "BAT_BATCH_STREAMS" side streams (1..4) the specialised batched
 *                      kernels are spread over (each kernel to the
 *                      least-loaded one, largest first), forked from and
 *                      joined to the calling thread's stream, so that
 *                      several run at once; 0 = the thread's stream only;
 *                      -1 (default) = bat_autotune_batched's choice of 1,
 *                      2 or 3, else 3.  With the thread's stream, 3 fill
 *                      the 4 hardware queues HIP gives a process by
 *                      default when no other streams share them
 *   "BAT_BATCH_ACC"    1 (default) = the batched kernels accumulate
 *                      transposed (lane = one p-vector and two of the
 *                      word's bytes; only mixed words read the byte
 *                      tables); 0 = one accumulator per p-vector in every
 *                      lane
 *   "BAT_JIT_PROCS"    how many graph-specialised kernels bat_autotune
 *                      compiles at once, each in a child process running
 *                      the helper program bat_jitc from the library's
 *                      directory (16 by default, at most 64; 0 = compile
 *                      each in this process when first launched).  The
 *                      code objects are those of an in-process compile:
 *                      the helper uses this process's hiprtc library
 *   "BAT_JIT_FLUSH"    setting it to a nonzero value unloads every
 *                      graph-specialised kernel this process compiled or
 *                      loaded (after the current device finishes its work;
 *                      no asynchronous call using one may still be pending
 *                      on another device); reads as 0
 * Unknown keys return BAT_EINVAL.
 *
 * Compiled specialised kernels are also kept on disk across processes:
 * code objects keyed by hashes of the whole kernel source, the target and
 * the compile options, in $BAT_JIT_CACHE_DIR, else
 * $XDG_CACHE_HOME/bat-mi355x, else $HOME/.cache/bat-mi355x.  Set the
 * environment variable BAT_JIT_CACHE=0 to turn this off.  An entry that
 * fails to read or load is recompiled and rewritten.
 */
int bat_set_option(const char *key, int64_t value);
int bat_get_option(const char *key, int64_t *value);

/*
 * Autotuner: times the kernel variants (arc-to-bit order, chain length,
 * work-item size, convergence-test cadence, the specialised forward
 * sweep's launch shape, specialised vs generic kernel) on an evenly spread
 * sample of the counter range of this graph and caches the fastest choice
 * under the graph's structure; a later candidate must be at least 1%
 * faster to replace an earlier one.  The gradient sweep's arc order and
 * chain length are then tuned on their own, starting from the forward's.
 * The candidates' specialised kernels are compiled side by side before
 * they are timed (option "BAT_JIT_PROCS").  Later calls on a graph of the same structure use it
 * while "BAT_AUTOTUNE" is 1.  *best_ns_per_vector (may be NULL) receives the
 * best measured time per state vector.  Results never depend on the choice
 * beyond floating-point rounding; counts never change.
 */
int bat_autotune(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const double *p,
                 int32_t s, int32_t t, double *best_ns_per_vector);

/*
 * Description of the last launch on the calling thread, for benchmarks:
 * kernel time in milliseconds (HIP events around the enumeration kernel on
 * its own stream), the number of state vectors it covered, which kernel ran
 * and the launch choices it ran with.  Returns BAT_EINVAL if nothing ran yet.
 */
typedef struct {
    double kernel_ms;      /* enumeration kernel only */
    double total_ms;       /* tables + enumeration + reduction, device side */
    double jit_ms;         /* graph-specialised kernel compile time (0 if cached / unused) */
    uint64_t vectors;      /* state vectors covered */
    int32_t specialised;   /* 1 if the graph-specialised kernel ran */
    int32_t chunk_log2;    /* work-item size used */
    int32_t n_chunks;      /* wavefront work items */
    int32_t relaxations;   /* arc relaxations per sweep after pruning */
    uint64_t kernel_id;    /* 64-bit hash naming the exact kernel code that ran (the specialised
                              kernel's code object, or the ahead-of-time kernel sources and instance) */
    int32_t perm;          /* arc-to-counter-bit order (as "BAT_PERM"; 4 = forward BAT order; -1 batched) */
    int32_t chain_log2;    /* warm-start chain length used, 0 = none */
    int32_t check_every;   /* convergence-test cadence */
    int32_t item_order;    /* 0 = consecutive work items, 1 = spread */
    int32_t block_waves;   /* wavefronts per block */
    int32_t super_restart; /* 1 if block bottoms resume from a kept super-block bottom */
    int32_t window_test;   /* 1 if chained blocks that cannot connect s and t were skipped */
    int32_t simd_waves;    /* wavefronts per SIMD the kernel was compiled to fit, 0 = compiler's choice */
    int32_t keep_bottom;   /* chain starts resumed from the kept block bottom: 1 in registers, 2 in LDS */
    int32_t reserved;
} bat_launch_info;

int bat_last_launch(bat_launch_info *info);

/*
 * Diagnostic: the sustained integer VALU rate of the current device, in
 * 32-bit lane operations per second (*lane_ops_per_s), measured with a
 * kernel of independent add / xor chains (64 blocks of 256 threads per
 * CU; the best of three timed launches after a warm-up).  Sweeps are
 * bound by this rate.  A CU issues up to 128 32-bit lane operations per
 * clock (two wave64 VALU instructions), so the ceiling for 256 CUs at
 * 2.4 GHz is 256 x 128 x 2.4e9 = 7.86e13; the kernel reaches about three
 * quarters of it.  Blocks the calling thread for a few
 * milliseconds.  BAT_EINVAL for a NULL pointer, BAT_EDEVICE on a HIP error.
 */
int bat_valu_peak(double *lane_ops_per_s);

/*
 * The source text of the graph-specialised kernel that the library hands
 * to hiprtc for this graph (flags: BAT_DIRECTED or 0): the forward sweep
 * (grad = 0), the gradient sweep (grad = 1), or the batched sweep of -grad
 * probability vectors (grad = -1..-32; undirected only), with
 * arc-to-counter-bit order `perm` (0..3, as "BAT_PERM"; the batched form
 * always runs order 0).
 * Diagnostics only; needs no GPU.  The text is what hiprtc compiles: it
 * declares no headers.  buf (may be NULL) receives at most *len bytes
 * including the terminating NUL; *len is set to the size needed.
 * Returns BAT_EINVAL on an invalid graph or perm, BAT_ETOOBIG if buf is
 * too small (nothing written).
 */
int bat_jit_source(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, int32_t s, int32_t t, uint32_t flags,
                   int32_t grad, int32_t perm, char *buf, uint64_t *len);

/*
 * The source text of the graph-specialised multi-state kernel that
 * bat_ms_reliability (c_lo = c_hi = 0) or bat_ms_reliability_range over
 * [c_lo, c_hi) compiles for this graph, these states and capacities
 * (capacity NULL: state k has capacity k) and demand 1 to 3 (BAT_EINVAL
 * otherwise, with no arcs, or for an empty or invalid range).  Same
 * conventions as bat_jit_source; the text does not depend on the
 * probabilities.
 */
int bat_ms_jit_source(int32_t n_nodes, int32_t n_arcs, const bat_arc *arcs, const int32_t *n_states,
                      const int32_t *capacity, int32_t s, int32_t t, int32_t demand, uint32_t flags, uint64_t c_lo,
                      uint64_t c_hi, char *buf, uint64_t *len);

#ifdef __cplusplus
}
#endif

#endif /* BAT_H */
