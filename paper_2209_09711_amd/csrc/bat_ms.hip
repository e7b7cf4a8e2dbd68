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
// The kernel sees the arcs in slots (the host's sweep order); slot 0 is the
// fastest-changing coordinate of the mixed-radix index.  A wavefront work
// item is 64 consecutive runs of `run` indices, one run per lane; a lane
// decodes its first vector from the index and steps through the rest with
// the generalised Rule 1 (slot 0 up by one; a slot that passes its top state
// returns to 0 and carries).
//
// The flow test pushes augmenting paths found on node bitmasks: a search
// sweeps the slots in order, adding the far end of every arc with residual
// capacity out of the reached set, until t is reached or a sweep adds
// nothing (no augmenting path: the flow is maximal); the arcs that first
// reached each node form a tree rooted at s, whose path to t reverse sweeps
// collect; the smaller of its bottleneck and the missing demand is pushed,
// so a vector takes at most d pushes.  A lane runs one sweep per loop step
// and moves on to its next vector as soon as its own test ends, so lanes
// whose tests are short do not wait for the wavefront's longest one.
//
// Two exact shortcuts along slot 0, when its capacity never drops as its
// state goes up (the host checks): a vector that meets the demand settles
// every later state of slot 0 at once (more capacity cannot lower the
// maximum flow), and a vector that does not passes its flow on to the
// next one, which only raised slot 0's capacity, so its search goes on
// from there.
//
// The host pads the slots past the last arc up to MM with one-state self-
// loops at s (capacity 0, probability 1), which change nothing, so every
// sweep is straight-line code over MM slots with no test of the arc count.
// Every per-slot value (state, residual capacities) is a register: every
// loop over slots is unrolled to the kernel's bound MM (16, 20, 24 or 32
// slots), and node sets are
// indexed by shifts only.  Pr(X) is the product of the other slots'
// probabilities, formed when they change, times slot 0's.  Sums:
// per-lane two-sums, a double-double wavefront fold, and a fixed-order
// reduction over work items.
#include <hip/hip_runtime.h>

#include "bat_launch.hpp"

using bat::u32;
using bat::u64;

// Up to 20 slots the per-slot registers (state, two residuals) leave room
// for 4 wavefronts per SIMD (128 VGPRs); the compiler is held to that.
template <int MM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MM <= 20 ? 4 : 1, MM <= 20 ? 4 : 8)))
k_ms_flow(batk::MsParams P)
{
    __shared__ int capt[batk::kMsMaxTable + batk::kMsMaxArcs];
    __shared__ double wt[batk::kMsMaxTable + batk::kMsMaxArcs];
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
    const u32 n = P.n, s = P.s, t = P.t;
    const int d = (int)P.d;
    const bool dir = P.directed != 0;
    // slot 0's capacity never drops as its state goes up (host-checked)
    const bool warm = P.warm != 0;

    double hi = 0.0, lo = 0.0;
    u64 cnt = 0;
    const u64 c0 = P.c_lo + (item * 64ull + lane) * P.run;
    u64 c1 = c0 + P.run;
    if (c1 > P.c_hi) c1 = P.c_hi;
    if (c0 < c1) {
        // slot i holds one arc; slot 0 is the fastest-changing coordinate
        u32 x[MM];
        int rf[MM], rb[MM];  // residual capacity of each slot's arc, u -> v and v -> u
        u64 r = c0;
#pragma unroll
        for (int i = 0; i < MM; ++i) {
            x[i] = (u32)(r % P.sig[i]);
            r /= P.sig[i];
        }
        // a vector's capacities, no flow yet, and the product of the
        // probabilities of every slot but 0 (slot 0's comes per vector)
        int total = 0;
        double rest = 1.0;
        auto load = [&]() {
            double pr = 1.0;
#pragma unroll
            for (int i = 0; i < MM; ++i) {
                rf[i] = capt[P.off[i] + x[i]];
                rb[i] = dir ? 0 : rf[i];
                if (i > 0) pr *= wt[P.off[i] + x[i]];
            }
            rest = pr;
            total = 0;
        };
        load();
        // One step is one sweep over the slots, so a lane whose test ends
        // moves on to its next vector while the others go on.
        u32 phase = 0u;  // 0: search, 1: collect the path found
        u32 reach = 1u << s, tf = 0u, tb = 0u, on = 0u, pf = 0u, pb = 0u;
        int b = 0;
        u64 c = c0;
        while (c < c1) {
            int fin = -1;  // -1: the test goes on; 0: demand not met; 1: met
            if (phase == 0u) {
                // reach grows from {s} over arcs with residual capacity;
                // tf / tb mark the arc that first reached a node, used
                // u -> v or v -> u
                const u32 before = reach;
#pragma unroll
                for (int i = 0; i < MM; ++i) {
                    const u32 u = P.u[i], v = P.v[i];
                    const u32 ru = (reach >> u) & 1u, rv = (reach >> v) & 1u;
                    const u32 fw = ru & (rv ^ 1u) & (u32)(rf[i] > 0);
                    const u32 bw = rv & (ru ^ 1u) & (u32)(rb[i] > 0);
                    reach |= (fw << v) | (bw << u);
                    tf |= fw << i;
                    tb |= bw << i;
                }
                if ((reach >> t) & 1u) {
                    phase = 1u;
                    on = 1u << t;
                    pf = pb = 0u;
                    b = d - total;
                } else if (reach == before) {
                    fin = 0;  // no augmenting path: the flow is maximal
                }
            } else {
                // the marked arcs form a tree rooted at s: collect its path
                // to t in reverse slot order, an arc joining when the node
                // it reached is on the path
#pragma unroll
                for (int i = MM - 1; i >= 0; --i) {
                    const u32 u = P.u[i], v = P.v[i];
                    const u32 jf = (tf >> i) & (on >> v) & 1u;
                    const u32 jb = (tb >> i) & (on >> u) & 1u;
                    on |= (jf << u) | (jb << v);
                    pf |= jf << i;
                    pb |= jb << i;
                    b = jf ? min(b, rf[i]) : b;
                    b = jb ? min(b, rb[i]) : b;
                }
                if ((on >> s) & 1u) {
                    // push b (at least one unit) along the path
#pragma unroll
                    for (int i = 0; i < MM; ++i) {
                        const int df = ((pf >> i) & 1u) ? b : 0, db = ((pb >> i) & 1u) ? b : 0;
                        rf[i] += db - df;
                        rb[i] += df - db;
                    }
                    total += b;
                    if (total >= d) fin = 1;
                    else {
                        phase = 0u;
                        reach = 1u << s;
                        tf = tb = 0u;
                    }
                }
            }
            if (fin < 0) continue;
            // the vector is decided
            u32 q = 0u;
            if (fin) {
                // slot 0's later states (until it wraps) meet the demand
                // too when its capacity never drops: count them at once
                if (warm) {
                    const u64 left = c1 - c - 1ull;
                    q = P.sig[0] - 1u - x[0];
                    if ((u64)q > left) q = (u32)left;
                }
                double w0 = 0.0;
                for (u32 k = 0; k <= q; ++k) w0 += wt[P.off[0] + x[0] + k];
                const double pr = rest * w0;
                double s_, e_;
                bat::two_sum(hi, pr, s_, e_);
                hi = s_;
                lo += e_;
                cnt += q + 1u;
                x[0] += q;
            }
            c += q + 1u;
            if (c >= c1) break;
            if (warm && !fin && x[0] + 1u < P.sig[0]) {
                // only slot 0 moves up: the flow found so far stays feasible
                const int dc = capt[P.off[0] + x[0] + 1u] - capt[P.off[0] + x[0]];
                x[0] += 1u;
                rf[0] += dc;
                rb[0] += dir ? 0 : dc;
            } else {
                // generalised Rule 1 from slot 0, then a fresh vector
                u32 carry = 1u;
#pragma unroll
                for (int i = 0; i < MM; ++i) {
                    const u32 nx = x[i] + carry;
                    const u32 wrap = nx == P.sig[i] ? 1u : 0u;
                    x[i] = wrap ? 0u : nx;
                    carry &= wrap;
                }
                load();
            }
            phase = 0u;
            reach = 1u << s;
            tf = tb = 0u;
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
template __global__ void k_ms_flow<20>(batk::MsParams);
template __global__ void k_ms_flow<24>(batk::MsParams);
template __global__ void k_ms_flow<32>(batk::MsParams);

namespace batk {

hipError_t ms_sweep(hipStream_t st, unsigned blocks, const MsParams &P)
{
    const dim3 g(blocks), b(bat::kBlock);
    switch (ms_slots((int)P.m)) {
    case 16: hipLaunchKernelGGL(k_ms_flow<16>, g, b, 0, st, P); break;
    case 20: hipLaunchKernelGGL(k_ms_flow<20>, g, b, 0, st, P); break;
    case 24: hipLaunchKernelGGL(k_ms_flow<24>, g, b, 0, st, P); break;
    default: hipLaunchKernelGGL(k_ms_flow<32>, g, b, 0, st, P); break;
    }
    return hipGetLastError();
}

}  // namespace batk
