// bat_ms.hip -- multi-state arcs: the BAT over a mixed-radix solution space
// (Section 4.1: arcs with sigma_i states give prod_i sigma_i vectors) with a
// demand-level flow test per state vector.
//
// What is computed: arc i is in state k in 0..sigma_i-1 with probability
// w_i(k), and carries at most cap_i(k) units (either way for an undirected
// arc).  A vector X meets demand d when the maximum s-t flow is at least d;
// R_d = sum of prod_i w_i(x_i) over those X, and count = their number.  The
// paper defines reliability for binary arcs only (Eq. 1) and names the
// multi-state problem as the next one to solve; with two states of capacity
// 0 and 1 and d = 1 this is exactly Eq. 1.
//
// Mapping onto the machine.  One lane decides one state vector at a time.
// A wavefront work item is 64 consecutive runs of `run` indices, one run per
// lane; a lane decodes its first vector from the index (mixed radix, arc 0
// most significant) and steps through the rest with the generalised Rule 1
// (the last coordinate below its top state goes up by one, later ones return
// to state 0).  The flow test is augmenting paths on node bitmasks: a search
// sweeps the arcs in order, adding the far end of every arc with residual
// capacity out of the reached set, until t is reached or a sweep adds
// nothing; the path is traced back through the arcs that first reached each
// node, and the smaller of its bottleneck and the missing demand is pushed.
// Everything indexed by an arc (state, capacity, flow) is an array the
// compiler keeps in registers: every loop over arcs is unrolled to the
// kernel's arc bound MM, and only node masks are indexed at run time (by
// shifts).  Sums: per-lane compensated (two-sum) partials, a double-double
// wavefront fold, and a fixed-order reduction over work items.
#include <hip/hip_runtime.h>

#include "bat_launch.hpp"

using bat::u32;
using bat::u64;

namespace {

// Searches sweep the arcs in order; at most n - 1 sweeps add a node, so n
// sweeps always end a search.  Each reached node but s has exactly one arc
// that reached it first (tf / tb: used u -> v or v -> u), so those arcs form
// a tree rooted at s, and the augmenting path is the tree path to t: sweeps
// over the arcs in reverse order collect it, an arc joining when the node it
// reached is on the path, until s is.
template <int MM>
struct MsFlow {
    const batk::MsParams &P;  // the kernel's parameters: arc endpoints are uniform
    u32 m, n, s, t;
    int d;

    // Does the flow reach demand d?  rf / rb: residual capacity of each arc
    // u -> v and v -> u (on entry: cap and, undirected, cap again, or 0 for a
    // directed arc).  Each augmentation adds at least one unit.
    __device__ __forceinline__ bool met(int (&rf)[MM], int (&rb)[MM]) const
    {
        int total = 0;
        for (;;) {
            u32 reach = 1u << s, tf = 0u, tb = 0u;
            for (u32 sw = 0; sw < n; ++sw) {
                const u32 before = reach;
#pragma unroll
                for (int i = 0; i < MM; ++i) {
                    if ((u32)i < m) {
                        const u32 u = P.u[i], v = P.v[i];
                        const u32 ru = (reach >> u) & 1u, rv = (reach >> v) & 1u;
                        const u32 fw = ru & (rv ^ 1u) & (u32)(rf[i] > 0);
                        const u32 bw = rv & (ru ^ 1u) & (u32)(rb[i] > 0);
                        reach |= (fw << v) | (bw << u);
                        tf |= fw << i;
                        tb |= bw << i;
                    }
                }
                if (((reach >> t) & 1u) || reach == before) break;
            }
            if (!((reach >> t) & 1u)) return false;  // no augmenting path: the flow is maximal
            u32 on = 1u << t, pf = 0u, pb = 0u;
            int b = d - total;
            for (u32 sw = 0; sw < n && !((on >> s) & 1u); ++sw) {
#pragma unroll
                for (int i = MM - 1; i >= 0; --i) {
                    if ((u32)i < m) {
                        const u32 u = P.u[i], v = P.v[i];
                        const u32 jf = (tf >> i) & (on >> v) & 1u;
                        const u32 jb = (tb >> i) & (on >> u) & 1u;
                        on |= (jf << u) | (jb << v);
                        pf |= jf << i;
                        pb |= jb << i;
                        b = jf ? min(b, rf[i]) : b;
                        b = jb ? min(b, rb[i]) : b;
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < MM; ++i) {
                const int df = ((pf >> i) & 1u) ? b : 0, db = ((pb >> i) & 1u) ? b : 0;
                rf[i] += db - df;
                rb[i] += df - db;
            }
            total += b;
            if (total >= d) return true;
        }
    }
};

}  // namespace

template <int MM>
__global__ void __launch_bounds__(256) k_ms_flow(batk::MsParams P)
{
    __shared__ int capt[batk::kMsMaxTable];
    __shared__ double wt[batk::kMsMaxTable];
    const u32 tid = threadIdx.x;
    for (u32 i = tid; i < P.n_table; i += blockDim.x) {
        capt[i] = P.cap[i];
        wt[i] = P.w[i];
    }
    __syncthreads();
    const u32 lane = tid & 63u;
    const u64 item = (u64)blockIdx.x * __builtin_amdgcn_readfirstlane(blockDim.x >> 6) +
                     __builtin_amdgcn_readfirstlane(tid >> 6);
    if (item >= P.n_items) return;
    const u32 m = P.m;
    const MsFlow<MM> F{P, m, P.n, P.s, P.t, (int)P.d};

    double hi = 0.0, lo = 0.0;
    u64 cnt = 0;
    const u64 c0 = P.c_lo + (item * 64ull + lane) * P.run;
    u64 c1 = c0 + P.run;
    if (c1 > P.c_hi) c1 = P.c_hi;
    if (c0 < c1) {
        // the first vector of the run: mixed radix, arc 0 most significant
        u32 x[MM];
        u64 r = c0;
#pragma unroll
        for (int i = MM - 1; i >= 0; --i) {
            x[i] = 0u;
            if ((u32)i < m) {
                x[i] = (u32)(r % P.sig[i]);
                r /= P.sig[i];
            }
        }
        for (u64 c = c0;;) {
            int rf[MM], rb[MM];
#pragma unroll
            for (int i = 0; i < MM; ++i) {
                rf[i] = (u32)i < m ? capt[P.off[i] + x[i]] : 0;
                rb[i] = P.directed ? 0 : rf[i];
            }
            if (F.met(rf, rb)) {
                ++cnt;
                double pr = 1.0;
#pragma unroll
                for (int i = 0; i < MM; ++i)
                    if ((u32)i < m) pr *= wt[P.off[i] + x[i]];
                double s_, e_;
                bat::two_sum(hi, pr, s_, e_);
                hi = s_;
                lo += e_;
            }
            if (++c == c1) break;
            // generalised Rule 1, branch-free over the unrolled arcs
            u32 carry = 1u;
#pragma unroll
            for (int i = MM - 1; i >= 0; --i) {
                if ((u32)i < m) {
                    const u32 nx = x[i] + carry;
                    const u32 wrap = nx == P.sig[i] ? 1u : 0u;
                    x[i] = wrap ? 0u : nx;
                    carry &= wrap;
                }
            }
        }
    }
    bat::wave_sum_dd(hi, lo);
    const u64 csum = bat::wave_sum_u64(cnt);
    if (lane == 0) {
        P.part[2 * item] = hi;
        P.part[2 * item + 1] = lo;
        P.pcount[item] = csum;
    }
}

template __global__ void k_ms_flow<16>(batk::MsParams);
template __global__ void k_ms_flow<32>(batk::MsParams);

namespace batk {

hipError_t ms_sweep(hipStream_t st, unsigned blocks, const MsParams &P)
{
    const dim3 g(blocks), b(bat::kBlock);
    if (P.m <= 16) hipLaunchKernelGGL(k_ms_flow<16>, g, b, 0, st, P);
    else hipLaunchKernelGGL(k_ms_flow<32>, g, b, 0, st, P);
    return hipGetLastError();
}

}  // namespace batk
