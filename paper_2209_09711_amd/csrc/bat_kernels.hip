// bat_kernels.hip -- ahead-of-time kernels of the BAT reliability library.
//
//  k_build_tables : the probability factor tables of Eq. 1 from p (device).
//  k_fwd_dyn<N>   : enumeration + connectivity + Pr sum, graph read at run
//                   time (N = register budget for node reach words).
//  k_grad_dyn<N>  : the same sweep also producing T1_i / T0_i per arc.
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

// One block of 256 threads.  Layout: see the k* offsets in bat_device.hpp.
extern "C" __global__ void __launch_bounds__(256)
k_build_tables(const double *__restrict__ p, u32 m, u32 f, double *__restrict__ T, int *status)
{
    const u32 tid = threadIdx.x;
    if (tid == 0) {
        int st = 0;
        for (u32 i = 0; i < m; ++i)
            if (!(p[i] >= 0.0 && p[i] <= 1.0)) st = -1;
        *status = st;
    }
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
        for (u32 k = 0; k < 6; ++k) T[bat::kTBG + k * 256 + y] = sg[k];
        // Q_lo over iteration bits below f
        double ql = 1.0;
        for (u32 b = 0; b < f; ++b) ql *= qbit(p, m, bat::kWordBits + b, (y >> b) & 1u);
        T[bat::kQlo + y] = (y < (1u << f)) ? ql : 0.0;
        for (u32 b = 0; b < 8; ++b) {
            double qm = 1.0;
            for (u32 b2 = 0; b2 < f; ++b2)
                if (b2 != b) qm *= qbit(p, m, bat::kWordBits + b2, (y >> b2) & 1u);
            T[bat::kQLOM + b * 256 + y] = (b < f && y < (1u << f)) ? qm : 0.0;
        }
    }
    if (tid < 4) {
        T[bat::kA4 + tid] = qbit(p, m, 3, tid & 1u) * qbit(p, m, 4, tid >> 1);
        T[bat::kA4M + tid] = qbit(p, m, 4, tid >> 1);      // without slice bit 3
        T[bat::kA4M + 4 + tid] = qbit(p, m, 3, tid & 1u);  // without slice bit 4
    }
    if (tid < 64) {
        double q = 1.0;
        for (u32 b = 0; b < 6; ++b) q *= qbit(p, m, bat::kSliceBits + b, (tid >> b) & 1u);
        T[bat::kQL + tid] = q;
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

template <int NMAX>
__global__ void __launch_bounds__(256) k_fwd_dyn(bat::KParams P)
{
    __shared__ bat::LdsTables L;
    bat::sweep_kernel<bat::DynClosure<NMAX>, false>(P, L, nullptr);
}

template <int NMAX>
__global__ void __launch_bounds__(256) k_grad_dyn(bat::KParams P)
{
    __shared__ bat::LdsTables L;
    __shared__ bat::LdsGrad LG;
    bat::sweep_kernel<bat::DynClosure<NMAX>, true>(P, L, &LG);
}

template __global__ void k_fwd_dyn<16>(bat::KParams);
template __global__ void k_fwd_dyn<32>(bat::KParams);
template __global__ void k_fwd_dyn<64>(bat::KParams);
template __global__ void k_grad_dyn<16>(bat::KParams);
template __global__ void k_grad_dyn<32>(bat::KParams);
template __global__ void k_grad_dyn<64>(bat::KParams);

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

// Write R, count and (if requested) T1/T0/dR/dp in arc order; counter bit
// cb belongs to arc m-1-cb.  Invalid probabilities give NaN and status -1.
extern "C" __global__ void __launch_bounds__(64)
k_finalize(const double *__restrict__ res, const u64 *__restrict__ count, const int *__restrict__ status,
           u32 m, u32 grad, double *R, u64 *cnt, double *dRdp, double *T1, double *T0, int *status_out)
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
            u32 cb = m - 1 - a;
            const double *t0 = res + 2 * (1 + 2 * cb), *t1 = res + 2 * (1 + 2 * cb + 1);
            double g = (t1[0] - t0[0]) + (t1[1] - t0[1]);
            if (dRdp) dRdp[a] = st ? nan : g;
            if (T1) T1[a] = st ? nan : t1[0] + t1[1];
            if (T0) T0[a] = st ? nan : t0[0] + t0[1];
        }
    }
}

// ------------------------------------------------------------ launchers
namespace batk {

hipError_t build_tables(hipStream_t st, const double *p, u32 m, u32 f, double *T, int *status)
{
    hipLaunchKernelGGL(k_build_tables, dim3(1), dim3(256), 0, st, p, m, f, T, status);
    return hipGetLastError();
}

hipError_t sweep_dyn(hipStream_t st, unsigned blocks, bool grad, int nmax, const bat::KParams &K)
{
    const dim3 g(blocks), b(bat::kBlock);
    if (nmax <= 16) {
        if (grad) hipLaunchKernelGGL(k_grad_dyn<16>, g, b, 0, st, K);
        else hipLaunchKernelGGL(k_fwd_dyn<16>, g, b, 0, st, K);
    } else if (nmax <= 32) {
        if (grad) hipLaunchKernelGGL(k_grad_dyn<32>, g, b, 0, st, K);
        else hipLaunchKernelGGL(k_fwd_dyn<32>, g, b, 0, st, K);
    } else {
        if (grad) hipLaunchKernelGGL(k_grad_dyn<64>, g, b, 0, st, K);
        else hipLaunchKernelGGL(k_fwd_dyn<64>, g, b, 0, st, K);
    }
    return hipGetLastError();
}

hipError_t reduce(hipStream_t st, const double *part, const u64 *pcount, u64 n_chunks, u32 ncol, double *res,
                  u64 *count)
{
    hipLaunchKernelGGL(k_reduce, dim3(ncol), dim3(256), 0, st, part, pcount, n_chunks, ncol, res, count);
    return hipGetLastError();
}

hipError_t finalize(hipStream_t st, const double *res, const u64 *count, const int *status, u32 m, bool grad,
                    double *R, u64 *cnt, double *dRdp, double *T1, double *T0, int *status_out)
{
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, st, res, count, status, m, grad ? 1u : 0u, R, cnt, dRdp,
                       T1, T0, status_out);
    return hipGetLastError();
}

}  // namespace batk
