// bat_kernels.hip -- ahead-of-time kernels of the BAT reliability library.
//
//  k_build_tables : the probability factor tables of Eq. 1 from p (device).
//  k_fwd_dyn<N,D> : enumeration + connectivity + Pr sum, graph read at run
//                   time (N = register budget for node reach words, D =
//                   directed arcs).
//  k_grad_dyn<N,D>: the same sweep also producing T1_i / T0_i per arc.
//  k_reduce       : fixed-order double-double sum of per-work-item partials.
//  k_finalize     : results to the caller's device buffers.
//  k_batched_dyn  : many graphs x many probability vectors, persistent.
#include <hip/hip_runtime.h>

#include "bat_launch.hpp"

using bat::u32;
using bat::u64;

namespace {

// q_cb(x) for counter bit cb: arc m-1-cb; bits at or above m are padding
// (virtual arcs that never work, so only x = 0 carries weight).
__device__ __forceinline__ double qbit(const double *p, u32 m, u32 cb, u32 x)
{
    if (cb >= m) return x ? 0.0 : 1.0;
    double pi = p[m - 1 - cb];
    return x ? pi : 1.0 - pi;
}

}  // namespace

// The probability tables of one p-vector (layout: the k* offsets in
// bat_device.hpp), computed by one block.  grad = false skips the tables
// only the gradient sweep reads.
__device__ void build_tables_dev(const double *__restrict__ p, u32 m, u32 f, double *__restrict__ T, bool grad)
{
    const u32 tid = threadIdx.x;
    const u32 ubits = m > (u32)bat::kWordBits ? m - bat::kWordBits : 0u;
    // B(i) over slice bits 0..2 and its one-bit-removed variants
    for (u32 y = tid; y < 256; y += blockDim.x) {
        double s = 0.0;
        double sg[6] = {0, 0, 0, 0, 0, 0};
        for (u32 i = 0; i < 8; ++i) {
            if (!((y >> i) & 1u)) continue;
            double q0 = qbit(p, m, 0, i & 1u), q1 = qbit(p, m, 1, (i >> 1) & 1u),
                   q2 = qbit(p, m, 2, (i >> 2) & 1u);
            s += q0 * q1 * q2;
            sg[0 * 2 + (i & 1u)] += q1 * q2;
            sg[1 * 2 + ((i >> 1) & 1u)] += q0 * q2;
            sg[2 * 2 + ((i >> 2) & 1u)] += q0 * q1;
        }
        T[bat::kTB + y] = s;
        // Q_lo over iteration bits below f
        double ql = 1.0;
        for (u32 b = 0; b < f; ++b) ql *= qbit(p, m, bat::kWordBits + b, (y >> b) & 1u);
        T[bat::kQlo + y] = (y < (1u << f)) ? ql : 0.0;
        if (!grad) continue;
        for (u32 k = 0; k < 6; ++k) T[bat::kTBG + k * 256 + y] = sg[k];
        for (u32 b = 0; b < 8; ++b) {
            double qm = 1.0;
            for (u32 b2 = 0; b2 < f; ++b2)
                if (b2 != b) qm *= qbit(p, m, bat::kWordBits + b2, (y >> b2) & 1u);
            T[bat::kQLOM + b * 256 + y] = (b < f && y < (1u << f)) ? qm : 0.0;
        }
    }
    if (tid < 4) {
        T[bat::kA4 + tid] = qbit(p, m, 3, tid & 1u) * qbit(p, m, 4, tid >> 1);
        if (grad) {
            T[bat::kA4M + tid] = qbit(p, m, 4, tid >> 1);      // without slice bit 3
            T[bat::kA4M + 4 + tid] = qbit(p, m, 3, tid & 1u);  // without slice bit 4
        }
    }
    if (tid < 64) {
        double q = 1.0;
        for (u32 b = 0; b < 6; ++b) q *= qbit(p, m, bat::kSliceBits + b, (tid >> b) & 1u);
        T[bat::kQL + tid] = q;
        if (grad)
            for (u32 b = 0; b < 6; ++b) {
                double qm = 1.0;
                for (u32 b2 = 0; b2 < 6; ++b2)
                    if (b2 != b) qm *= qbit(p, m, bat::kSliceBits + b2, (tid >> b2) & 1u);
                T[bat::kQLM + b * 64 + tid] = qm;
            }
    }
    if (tid < 128) {
        u32 b = tid >> 1, x = tid & 1u;
        T[bat::kQG + tid] = (b < ubits) ? qbit(p, m, bat::kWordBits + b, x) : (x ? 0.0 : 1.0);
    }
}

// One block of 256 threads for the single-graph sweeps; also checks p.
// row[j] (nullable = identity) is the arc whose probability plays the role
// of arc j of the identity order, i.e. the arc at counter bit m-1-j.
extern "C" __global__ void __launch_bounds__(256)
k_build_tables(const double *__restrict__ p, const unsigned char *__restrict__ row, u32 m, u32 f,
               double *__restrict__ T, int *status)
{
    __shared__ double pr[64];
    const u32 tid = threadIdx.x;
    if (tid < m) pr[tid] = row ? p[row[tid]] : p[tid];
    if (tid == 0) {
        int st = 0;
        for (u32 i = 0; i < m; ++i)
            if (!(p[i] >= 0.0 && p[i] <= 1.0)) st = -1;
        *status = st;
    }
    __syncthreads();
    build_tables_dev(pr, m, f, T, true);
}

template <int NMAX, bool DIR>
__global__ void __launch_bounds__(256) k_fwd_dyn(bat::KParams P)
{
    __shared__ bat::LdsTables L;
    bat::sweep_kernel<bat::DynClosure<NMAX, DIR>, false>(P, L, nullptr);
}

template <int NMAX, bool DIR>
__global__ void __launch_bounds__(256) k_grad_dyn(bat::KParams P)
{
    __shared__ bat::LdsTables L;
    __shared__ bat::LdsGrad LG;
    bat::sweep_kernel<bat::DynClosure<NMAX, DIR>, true>(P, L, &LG);
}

template __global__ void k_fwd_dyn<16, false>(bat::KParams);
template __global__ void k_fwd_dyn<32, false>(bat::KParams);
template __global__ void k_fwd_dyn<64, false>(bat::KParams);
template __global__ void k_grad_dyn<16, false>(bat::KParams);
template __global__ void k_grad_dyn<32, false>(bat::KParams);
template __global__ void k_grad_dyn<64, false>(bat::KParams);
template __global__ void k_fwd_dyn<16, true>(bat::KParams);
template __global__ void k_fwd_dyn<32, true>(bat::KParams);
template __global__ void k_fwd_dyn<64, true>(bat::KParams);
template __global__ void k_grad_dyn<16, true>(bat::KParams);
template __global__ void k_grad_dyn<32, true>(bat::KParams);
template __global__ void k_grad_dyn<64, true>(bat::KParams);

// Column col of the partials: block col sums it over all work items in a
// fixed order (thread-strided, then a fixed tree), so the result does not
// depend on scheduling.  Block 0 also adds the counts (exact integers).
extern "C" __global__ void __launch_bounds__(256)
k_reduce(const double *__restrict__ part, const u64 *__restrict__ pcount, u64 n_chunks, u32 ncol,
         double *__restrict__ res, u64 *__restrict__ count)
{
    __shared__ double sh[256], sl[256];
    __shared__ u64 sc[256];
    const u32 tid = threadIdx.x, col = blockIdx.x;
    double hi = 0.0, lo = 0.0;
    u64 c = 0;
    for (u64 k = tid; k < n_chunks; k += 256) {
        const double *q = part + (k * ncol + col) * 2ull;
        bat::dd_add(hi, lo, q[0], q[1]);
        if (col == 0) c += pcount[k];
    }
    sh[tid] = hi;
    sl[tid] = lo;
    sc[tid] = c;
    __syncthreads();
    for (u32 st = 128; st >= 1; st >>= 1) {
        if (tid < st) {
            double h = sh[tid], l = sl[tid];
            bat::dd_add(h, l, sh[tid + st], sl[tid + st]);
            sh[tid] = h;
            sl[tid] = l;
            sc[tid] += sc[tid + st];
        }
        __syncthreads();
    }
    if (tid == 0) {
        res[2 * col] = sh[0];
        res[2 * col + 1] = sl[0];
        if (col == 0) *count = sc[0];
    }
}

// Write R, count and (if requested) T1/T0/dR/dp in arc order; arc a sits at
// counter bit cb_of_arc[a] (nullable = identity, m-1-a).  Invalid probabilities give NaN and status -1.
extern "C" __global__ void __launch_bounds__(64)
k_finalize(const double *__restrict__ res, const u64 *__restrict__ count, const int *__restrict__ status,
           const unsigned char *__restrict__ cb_of_arc, u32 m, u32 grad, double *R, u64 *cnt, double *dRdp,
           double *T1, double *T0, int *status_out)
{
    const u32 tid = threadIdx.x;
    const int st = *status;
    const double nan = __builtin_nan("");
    if (tid == 0) {
        *R = st ? nan : res[0] + res[1];
        *cnt = st ? 0ull : *count;
        if (status_out) *status_out = st;
    }
    if (grad) {
        for (u32 a = tid; a < m; a += blockDim.x) {
            u32 cb = cb_of_arc ? cb_of_arc[a] : m - 1 - a;
            const double *t0 = res + 2 * (1 + 2 * cb), *t1 = res + 2 * (1 + 2 * cb + 1);
            double g = (t1[0] - t0[0]) + (t1[1] - t0[1]);
            if (dRdp) dRdp[a] = st ? nan : g;
            if (T1) T1[a] = st ? nan : t1[0] + t1[1];
            if (T0) T0[a] = st ? nan : t0[0] + t0[1];
        }
    }
}

// ------------------------------------------------------------ batched form
// Tables of (entry, p-vector) pair k: one block per pair.
extern "C" __global__ void __launch_bounds__(256)
k_batched_tables(const batk::BatchEntry *__restrict__ entries, const u32 *__restrict__ pair_entry,
                 const u32 *__restrict__ pair_pv, const u64 *__restrict__ entry_p_off, const double *__restrict__ p,
                 double *__restrict__ tables)
{
    const u32 k = blockIdx.x;
    const u32 e = pair_entry[k], pv = pair_pv[k];
    const batk::BatchEntry E = entries[e];
    build_tables_dev(p + entry_p_off[e] + (u64)(E.pv_base + pv) * E.m, E.m, E.f,
                     tables + E.tab_off + (u64)pv * bat::kTablesFwd, false);
}

// Persistent: every block loops { take the next item from the queue; load
// its entry's tables into LDS; each wavefront sweeps 2^f iterations of the
// graph's counter and adds, for every probability vector, Q_lo * F(V) per
// word (one connectivity verdict serves all of them); fold the wavefronts
// in a fixed order into the item's own partial slot }.  Items are queued
// longest graph first.  Every wavefront leaves when the queue is empty.
template <int NMAX>
__global__ void __launch_bounds__(batk::batch_waves(NMAX) * bat::kWave) k_batched_dyn(batk::BatchParams B)
{
    using namespace batk;
    constexpr int kBatchWaves = batch_waves(NMAX);
    constexpr int kBatchThreads = kBatchWaves * bat::kWave;
    __shared__ double tb[kBatchMaxP][256];
    __shared__ double a4[kBatchMaxP][4];
    __shared__ double qlo[kBatchMaxP][1 << kBatchSegLog];
    __shared__ double full[kBatchMaxP];  // F(~0): the mass of a word whose 32 vectors all connect
    __shared__ double wsum[kBatchWaves][kBatchMaxP][2];
    __shared__ u64 wcnt[kBatchWaves];
    __shared__ u64 s_item;
    __shared__ u32 s_entry;
    const u32 tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    for (;;) {
        if (tid == 0) {
            u64 it = atomicAdd(B.ctr, 1ull);
            u32 lo = 0, hi = B.n_entries;   // entry e with item_start[e] <= it < item_start[e+1]
            while (hi - lo > 1) {
                u32 mid = (lo + hi) >> 1;
                if (B.item_start[mid] <= it) lo = mid;
                else hi = mid;
            }
            s_item = it;
            s_entry = lo;
        }
        __syncthreads();
        // uniform: the entry (and the relaxation program it points to) is
        // then read with scalar loads
        const u64 item = ((u64)__builtin_amdgcn_readfirstlane((u32)(s_item >> 32)) << 32) |
                         __builtin_amdgcn_readfirstlane((u32)s_item);
        if (item >= B.n_items) break;
        const BatchEntry E = B.entries[__builtin_amdgcn_readfirstlane(s_entry)];
        const u32 P = E.P, f = E.f;
        const double *T = B.tables + E.tab_off;
        for (u32 i = tid; i < P * 256u; i += kBatchThreads)
            tb[i >> 8][i & 255u] = T[(u64)(i >> 8) * bat::kTablesFwd + bat::kTB + (i & 255u)];
        for (u32 i = tid; i < P * 4u; i += kBatchThreads) a4[i >> 2][i & 3u] = T[(u64)(i >> 2) * bat::kTablesFwd + bat::kA4 + (i & 3u)];
        for (u32 i = tid; i < (P << kBatchSegLog); i += kBatchThreads)
            qlo[i >> kBatchSegLog][i & ((1u << kBatchSegLog) - 1u)] =
                T[(u64)(i >> kBatchSegLog) * bat::kTablesFwd + bat::kQlo + (i & ((1u << kBatchSegLog) - 1u))];
        __syncthreads();
        if (tid < P) {
            // the same operations, in the same order, as a word of all ones
            // takes through the tables below: either path gives the same bits
            double F = a4[tid][0] * tb[tid][255];
            F = __builtin_fma(a4[tid][1], tb[tid][255], F);
            F = __builtin_fma(a4[tid][2], tb[tid][255], F);
            full[tid] = __builtin_fma(a4[tid][3], tb[tid][255], F);
        }
        __syncthreads();

        const u64 iters = 1ull << E.ubits;
        const u64 seg = (item - E.item_begin) * kBatchWaves + w;
        const u64 g0 = seg << f;
        double tot[kBatchMaxP];
#pragma unroll
        for (int q = 0; q < kBatchMaxP; ++q) tot[q] = 0.0;
        u64 cnt = 0;
        if (g0 < iters) {
            u64 g1 = g0 + (1ull << f) - 1ull;
            if (g1 > iters - 1) g1 = iters - 1;
            bat::KParams K;
            K.s = E.s;
            K.t = E.t;
            K.n_relax = E.n_relax;
            K.n_groups = E.n_groups;
            K.prog = B.prog + E.prog_off;
#pragma unroll
            for (int b = 0; b < 6; ++b) K.ck_code[b] = E.ck_code[b];
            K.check_every = B.check_every;
            bat::DynClosure<NMAX> cl;
            cl.init(lane, K);
            const u64 chi = E.m >= 63 ? ~0ull : (1ull << E.m);
            // one verdict word of iteration g into all P accumulators
            auto add = [&](u64 g, u32 V) {
                if (g == iters - 1) V &= bat::edge_mask(0ull, chi, g, lane);
                cnt += __popc(V);
                if (__ballot(V != 0u) == 0ull) return;
                const u32 glo = (u32)(g & ((1ull << f) - 1ull));
                // words that are all ones or all zeros (the five in-word arcs
                // do not matter) need no byte-table reads: F is full or 0.
                // Taken only when the whole wavefront's words are (a per-lane
                // split measured no faster: the table path still issues)
                if (__ballot(V != 0u && V != ~0u) == 0ull) {
                    const double on = V ? 1.0 : 0.0;
#pragma unroll
                    for (int q = 0; q < kBatchMaxP; ++q)
                        if ((u32)q < P) tot[q] = __builtin_fma(qlo[q][glo], on * full[q], tot[q]);
                    return;
                }
                const u32 b0 = V & 255u, b1 = (V >> 8) & 255u, b2 = (V >> 16) & 255u, b3 = V >> 24;
                // re-read the per-vector byte factors every iteration (held in
                // registers they would need 256 VGPRs for 32 p-vectors): an
                // opaque zero offset keeps the compiler from hoisting them
                u32 zero;
                asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
                const double(*a4v)[4] = (const double(*)[4])(&a4[0][0] + zero);
#pragma unroll
                for (int q = 0; q < kBatchMaxP; ++q) {
                    if ((u32)q < P) {
                        double F = a4v[q][0] * tb[q][b0];
                        F = __builtin_fma(a4v[q][1], tb[q][b1], F);
                        F = __builtin_fma(a4v[q][2], tb[q][b2], F);
                        F = __builtin_fma(a4v[q][3], tb[q][b3], F);
                        tot[q] = __builtin_fma(qlo[q][glo], F, tot[q]);
                    }
                }
            };
            // chained blocks of 2^k iterations (f >= k: inside this segment)
            cl.sweep_range(g0, g1, E.chain, K, add, [](u64, u64) {});
        }
        // Q_hi of this segment and Q_L of the lane, then across the wavefront
#pragma unroll
        for (int q = 0; q < kBatchMaxP; ++q) {
            if ((u32)q < P) {
                const double *Tq = T + (u64)q * bat::kTablesFwd;
                double qhi = 1.0;
                for (u32 b = f; b < E.ubits; ++b) qhi *= Tq[bat::kQG + 2 * b + (u32)((g0 >> b) & 1ull)];
                double h = tot[q] * qhi * Tq[bat::kQL + lane], l = 0.0;
                bat::wave_sum_dd(h, l);
                if (lane == 0) {
                    wsum[w][q][0] = h;
                    wsum[w][q][1] = l;
                }
            }
        }
        u64 c = bat::wave_sum_u64(cnt);
        if (lane == 0) wcnt[w] = c;
        __syncthreads();
        if (tid < P) {
            double h = 0.0, l = 0.0;
            for (int v = 0; v < kBatchWaves; ++v) bat::dd_add(h, l, wsum[v][tid][0], wsum[v][tid][1]);
            B.part[(item * kBatchMaxP + tid) * 2] = h;
            B.part[(item * kBatchMaxP + tid) * 2 + 1] = l;
        }
        if (tid == 0) {
            u64 cs = 0;
            for (int v = 0; v < kBatchWaves; ++v) cs += wcnt[v];
            B.pcount[item] = cs;
        }
        __syncthreads();
    }
}

// The same queue with the transposed accumulation (bat_device.hpp,
// AccumBatchT): lane (q, h) holds p-vector q's share of bytes h and h + 2
// of every word (of byte h alone, four lanes per p-vector, for items of
// up to 16 p-vectors); only the wavefront's mixed words (through an LDS row)
// take byte-table reads, a word of ones adds Q_L(src) F_q(~0), and Q_L is
// applied per word, so an item ends with one exchange between the lane
// halves instead of a wavefront fold per p-vector.
template <int NMAX>
__global__ void __launch_bounds__(batk::batch_waves_t(NMAX) * bat::kWave) k_batched_dyn_t(batk::BatchParams B)
{
    using namespace batk;
    constexpr int kBatchWaves = batch_waves_t(NMAX);
    constexpr int kBatchThreads = kBatchWaves * bat::kWave;
    constexpr int kSeg = 1 << kBatchSegLog;
    __shared__ double tb[kBatchMaxP][bat::kBatchTStride];
    __shared__ double a4[kBatchMaxP][4];
    __shared__ double qlo[kBatchMaxP][kSeg + 1];
    __shared__ double ql[kBatchMaxP][bat::kWave + 1];
    __shared__ double qls[kBatchMaxP];
    __shared__ u32 row[kBatchWaves][bat::kWave];
    __shared__ double wsum[kBatchWaves][kBatchMaxP][2];
    __shared__ u64 wcnt[kBatchWaves];
    __shared__ u64 s_item;
    __shared__ u32 s_entry;
    const u32 tid = threadIdx.x, lane = tid & 63u, w = tid >> 6;
    for (;;) {
        if (tid == 0) {
            u64 it = atomicAdd(B.ctr, 1ull);
            u32 lo = 0, hi = B.n_entries;   // entry e with item_start[e] <= it < item_start[e+1]
            while (hi - lo > 1) {
                u32 mid = (lo + hi) >> 1;
                if (B.item_start[mid] <= it) lo = mid;
                else hi = mid;
            }
            s_item = it;
            s_entry = lo;
        }
        __syncthreads();
        const u64 item = ((u64)__builtin_amdgcn_readfirstlane((u32)(s_item >> 32)) << 32) |
                         __builtin_amdgcn_readfirstlane((u32)s_item);
        if (item >= B.n_items) break;
        const BatchEntry E = B.entries[__builtin_amdgcn_readfirstlane(s_entry)];
        const u32 P = E.P, f = E.f;
        const double *T = B.tables + E.tab_off;
        for (u32 i = tid; i < P * 256u; i += kBatchThreads)
            tb[i >> 8][i & 255u] = T[(u64)(i >> 8) * bat::kTablesFwd + bat::kTB + (i & 255u)];
        for (u32 i = tid; i < P * 4u; i += kBatchThreads) a4[i >> 2][i & 3u] = T[(u64)(i >> 2) * bat::kTablesFwd + bat::kA4 + (i & 3u)];
        for (u32 i = tid; i < P * (u32)kSeg; i += kBatchThreads)
            qlo[i / kSeg][i % kSeg] = T[(u64)(i / kSeg) * bat::kTablesFwd + bat::kQlo + (i % kSeg)];
        for (u32 i = tid; i < P * 64u; i += kBatchThreads)
            ql[i >> 6][i & 63u] = T[(u64)(i >> 6) * bat::kTablesFwd + bat::kQL + (i & 63u)];
        __syncthreads();
        if (tid < P) {
            double a = 0.0;
            for (u32 k = 0; k < 64u; ++k) a += ql[tid][k];
            qls[tid] = a;
        }
        __syncthreads();

        // this lane's p-vector (lanes past P add nothing) and its bytes:
        // above 16 p-vectors two lanes of two bytes each per p-vector,
        // else four lanes of one byte (uniform: P is the item's)
        const bool two = P > 16u;
        const u32 qn = two ? 32u : 16u;
        const u32 qv = lane & (qn - 1u), half = lane / qn;
        const u32 sh0 = 8u * half, sh1 = sh0 + 16u;
        const bool live = qv < P;
        const u32 q = live ? qv : 0u;
        const double a0 = live ? a4[q][half] : 0.0, a1 = (live && two) ? a4[q][(half + 2u) & 3u] : 0.0;
        const double fullp = __builtin_fma(a1, tb[q][255], a0 * tb[q][255]);
        const double qlsum = qls[q];
        const u64 iters = 1ull << E.ubits;
        const u64 seg = (item - E.item_begin) * kBatchWaves + w;
        const u64 g0 = seg << f;
        double tot = 0.0;
        u64 cnt = 0;
        if (g0 < iters) {
            u64 g1 = g0 + (1ull << f) - 1ull;
            if (g1 > iters - 1) g1 = iters - 1;
            bat::KParams K;
            K.s = E.s;
            K.t = E.t;
            K.n_relax = E.n_relax;
            K.n_groups = E.n_groups;
            K.prog = B.prog + E.prog_off;
#pragma unroll
            for (int b = 0; b < 6; ++b) K.ck_code[b] = E.ck_code[b];
            K.check_every = B.check_every;
            bat::DynClosure<NMAX> cl;
            cl.init(lane, K);
            const u64 chi = E.m >= 63 ? ~0ull : (1ull << E.m);
            u32 *myrow = row[w];
            auto add = [&](u64 g, u32 V) {
                if (g == iters - 1) V &= bat::edge_mask(0ull, chi, g, lane);
                cnt += __popc(V);
                const u64 nz = __ballot(V != 0u);
                if (nz == 0ull) return;
                const u64 om = __ballot(V == ~0u);
                const u64 mm = nz & ~om;
                double x = 0.0;
                if (om != 0ull) {
                    double os = 0.0;
                    if (om == ~0ull) {
                        os = qlsum;
                    } else {
                        for (u64 b = om; b != 0ull; b &= b - 1ull) os += ql[q][__builtin_ctzll(b)];
                    }
                    x = os * fullp;
                }
                if (mm != 0ull) {
                    // LDS operations of one wavefront complete in order
                    myrow[lane] = V;
                    asm volatile("" ::: "memory");
                    for (u64 b = mm; b != 0ull; b &= b - 1ull) {
                        const u32 sl = (u32)__builtin_ctzll(b);
                        const u32 Vs = myrow[sl];
                        double t = a0 * tb[q][(Vs >> sh0) & 255u];
                        if (two) t = __builtin_fma(a1, tb[q][(Vs >> sh1) & 255u], t);
                        x = __builtin_fma(ql[q][sl], t, x);
                    }
                    asm volatile("" ::: "memory");
                }
                const u32 glo = (u32)(g & ((1ull << f) - 1ull));
                tot = __builtin_fma(qlo[q][glo], x, tot);
            };
            cl.sweep_range(g0, g1, E.chain, K, add, [](u64, u64) {});
        }
        // Q_hi of this segment, then the two halves of each p-vector
        {
            const double *Tq = T + (u64)q * bat::kTablesFwd;
            double qhi = 1.0;
            for (u32 b = f; b < E.ubits; ++b) qhi *= Tq[bat::kQG + 2 * b + (u32)((g0 >> b) & 1ull)];
            tot *= qhi;
            double h, l;
            bat::two_sum(tot, bat::shfl_xor_d(tot, 32), h, l);
            if (!two) {
                const double oh = bat::shfl_xor_d(h, 16), ol = bat::shfl_xor_d(l, 16);
                bat::dd_add(h, l, oh, ol);
            }
            if (lane < P) {
                wsum[w][lane][0] = h;
                wsum[w][lane][1] = l;
            }
        }
        u64 c = bat::wave_sum_u64(cnt);
        if (lane == 0) wcnt[w] = c;
        __syncthreads();
        if (tid < P) {
            double h = 0.0, l = 0.0;
            for (int v = 0; v < kBatchWaves; ++v) bat::dd_add(h, l, wsum[v][tid][0], wsum[v][tid][1]);
            B.part[(item * kBatchMaxP + tid) * 2] = h;
            B.part[(item * kBatchMaxP + tid) * 2 + 1] = l;
        }
        if (tid == 0) {
            u64 cs = 0;
            for (int v = 0; v < kBatchWaves; ++v) cs += wcnt[v];
            B.pcount[item] = cs;
        }
        __syncthreads();
    }
}

template __global__ void k_batched_dyn<16>(batk::BatchParams);
template __global__ void k_batched_dyn<32>(batk::BatchParams);
template __global__ void k_batched_dyn<64>(batk::BatchParams);
template __global__ void k_batched_dyn_t<16>(batk::BatchParams);
template __global__ void k_batched_dyn_t<32>(batk::BatchParams);
template __global__ void k_batched_dyn_t<64>(batk::BatchParams);

// Entry e: its items split into kReduceGroups consecutive runs; lane q of
// group c adds p-vector q's partials of run c in item order, then thread q
// adds the runs' sums in run order (a fixed order: the result does not
// depend on timing).  The counts of the entry holding p-vector 0 likewise.
constexpr int kReduceGroups = 8;
extern "C" __global__ void __launch_bounds__(kReduceGroups * 32)
k_batched_reduce(const batk::BatchEntry *__restrict__ entries, const double *__restrict__ part,
                 const u64 *__restrict__ pcount, u32 n_pvec, double *__restrict__ R, u64 *__restrict__ counts)
{
    __shared__ double hs[kReduceGroups][32][2];
    __shared__ u64 cs[kReduceGroups];
    const batk::BatchEntry E = entries[blockIdx.x];
    const u32 q = threadIdx.x & 31u, c = threadIdx.x >> 5;
    const u64 i0 = E.item_begin + E.n_items * c / kReduceGroups;
    const u64 i1 = E.item_begin + E.n_items * (c + 1) / kReduceGroups;
    double h = 0.0, l = 0.0;
    if (q < E.P)
        for (u64 it = i0; it < i1; ++it)
            bat::dd_add(h, l, part[(it * batk::kBatchMaxP + q) * 2], part[(it * batk::kBatchMaxP + q) * 2 + 1]);
    hs[c][q][0] = h;
    hs[c][q][1] = l;
    if (q == 0) {
        u64 n = 0;
        for (u64 it = i0; it < i1; ++it) n += pcount[it];
        cs[c] = n;
    }
    __syncthreads();
    if (threadIdx.x < E.P) {
        double th = 0.0, tl = 0.0;
        for (int g = 0; g < kReduceGroups; ++g) bat::dd_add(th, tl, hs[g][threadIdx.x][0], hs[g][threadIdx.x][1]);
        R[(u64)E.graph * n_pvec + E.pv_base + threadIdx.x] = th + tl;
    }
    if (threadIdx.x == 0 && E.pv_base == 0) {
        u64 n = 0;
        for (int g = 0; g < kReduceGroups; ++g) n += cs[g];
        counts[E.graph] = n;
    }
}

// Sustained integer VALU rate (a diagnostic, no part of the sweep): per loop
// trip, 8 independent chains of one 32-bit add and one xor, i.e.
// batk::kValuPeakOpsPerTrip full-rate VALU instructions.  The chains' xor
// is stored only when it equals a value these inputs practically never
// give, which keeps every chain live.
extern "C" __global__ void __launch_bounds__(256) k_valu_peak(u32 iters, u32 *sink)
{
    u32 a[8], b[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = threadIdx.x * (2u * (u32)i + 1u);
        b[i] = blockIdx.x + 0x9E3779B9u * (u32)i;
    }
    for (u32 k = 0; k < iters; ++k) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            a[i] += b[i];
            b[i] ^= a[i];
        }
    }
    u32 x = 0u;
#pragma unroll
    for (int i = 0; i < 8; ++i) x ^= a[i] ^ b[i];
    if (x == 0x5bd1e995u) sink[threadIdx.x & 63u] = x;
}

// ------------------------------------------------------------ launchers
namespace batk {

hipError_t build_tables(hipStream_t st, const double *p, const unsigned char *row, u32 m, u32 f, double *T,
                        int *status)
{
    hipLaunchKernelGGL(k_build_tables, dim3(1), dim3(256), 0, st, p, row, m, f, T, status);
    return hipGetLastError();
}

template <bool DIR>
static void sweep_dyn_t(hipStream_t st, unsigned blocks, bool grad, int nmax, const bat::KParams &K)
{
    const dim3 g(blocks), b(bat::kBlock);
    if (nmax <= 16) {
        if (grad) hipLaunchKernelGGL((k_grad_dyn<16, DIR>), g, b, 0, st, K);
        else hipLaunchKernelGGL((k_fwd_dyn<16, DIR>), g, b, 0, st, K);
    } else if (nmax <= 32) {
        if (grad) hipLaunchKernelGGL((k_grad_dyn<32, DIR>), g, b, 0, st, K);
        else hipLaunchKernelGGL((k_fwd_dyn<32, DIR>), g, b, 0, st, K);
    } else {
        if (grad) hipLaunchKernelGGL((k_grad_dyn<64, DIR>), g, b, 0, st, K);
        else hipLaunchKernelGGL((k_fwd_dyn<64, DIR>), g, b, 0, st, K);
    }
}

hipError_t sweep_dyn(hipStream_t st, unsigned blocks, bool grad, int nmax, bool directed, const bat::KParams &K)
{
    if (directed) sweep_dyn_t<true>(st, blocks, grad, nmax, K);
    else sweep_dyn_t<false>(st, blocks, grad, nmax, K);
    return hipGetLastError();
}

hipError_t valu_peak(hipStream_t st, unsigned blocks, u32 iters, u32 *sink)
{
    hipLaunchKernelGGL(k_valu_peak, dim3(blocks), dim3(256), 0, st, iters, sink);
    return hipGetLastError();
}

hipError_t reduce(hipStream_t st, const double *part, const u64 *pcount, u64 n_chunks, u32 ncol, double *res,
                  u64 *count)
{
    hipLaunchKernelGGL(k_reduce, dim3(ncol), dim3(256), 0, st, part, pcount, n_chunks, ncol, res, count);
    return hipGetLastError();
}

hipError_t finalize(hipStream_t st, const double *res, const u64 *count, const int *status,
                    const unsigned char *cb_of_arc, u32 m, bool grad, double *R, u64 *cnt, double *dRdp, double *T1,
                    double *T0, int *status_out)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, res, count, status, cb_of_arc, m, grad ? 1u : 0u, R,
                       cnt, dRdp, T1, T0, status_out);
    return hipGetLastError();
}

hipError_t batched_tables(hipStream_t st, const BatchEntry *entries, const u32 *pair_entry, const u32 *pair_pv,
                          const u64 *entry_p_off, const double *p, unsigned n_pairs, double *tables)
{
    hipLaunchKernelGGL(k_batched_tables, dim3(n_pairs), dim3(256), 0, st, entries, pair_entry, pair_pv, entry_p_off,
                       p, tables);
    return hipGetLastError();
}

hipError_t batched_sweep(hipStream_t st, unsigned blocks, int nmax, bool transposed, const BatchParams &B)
{
    const dim3 g(blocks);
    if (transposed) {
        if (nmax <= 16) hipLaunchKernelGGL(k_batched_dyn_t<16>, g, dim3(batch_waves_t(16) * bat::kWave), 0, st, B);
        else if (nmax <= 32) hipLaunchKernelGGL(k_batched_dyn_t<32>, g, dim3(batch_waves_t(32) * bat::kWave), 0, st, B);
        else hipLaunchKernelGGL(k_batched_dyn_t<64>, g, dim3(batch_waves_t(64) * bat::kWave), 0, st, B);
    } else {
        if (nmax <= 16) hipLaunchKernelGGL(k_batched_dyn<16>, g, dim3(batch_waves(16) * bat::kWave), 0, st, B);
        else if (nmax <= 32) hipLaunchKernelGGL(k_batched_dyn<32>, g, dim3(batch_waves(32) * bat::kWave), 0, st, B);
        else hipLaunchKernelGGL(k_batched_dyn<64>, g, dim3(batch_waves(64) * bat::kWave), 0, st, B);
    }
    return hipGetLastError();
}

hipError_t batched_reduce(hipStream_t st, const BatchEntry *entries, unsigned n_entries, const double *part,
                          const u64 *pcount, u32 n_pvec, double *R, u64 *counts)
{
    hipLaunchKernelGGL(k_batched_reduce, dim3(n_entries), dim3(kReduceGroups * 32), 0, st, entries, part, pcount, n_pvec, R, counts);
    return hipGetLastError();
}

}  // namespace batk
