// bat_launch.hpp -- host-side launchers for the ahead-of-time kernels in
// bat_kernels.hip (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "bat_device.hpp"

namespace batk {

hipError_t build_tables(hipStream_t st, const double *p, bat::u32 m, bat::u32 f, double *T, int *status);
hipError_t sweep_dyn(hipStream_t st, unsigned blocks, bool grad, int nmax, const bat::KParams &K);
hipError_t reduce(hipStream_t st, const double *part, const bat::u64 *pcount, bat::u64 n_chunks, bat::u32 ncol,
                  double *res, bat::u64 *count);
hipError_t finalize(hipStream_t st, const double *res, const bat::u64 *count, const int *status, bat::u32 m,
                    bool grad, double *R, bat::u64 *cnt, double *dRdp, double *T1, double *T0, int *status_out);

}  // namespace batk
