// net.h -- internal interface between the AMG solver and the learned preconditioner.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/psc.h"
#include "kernels.h"

namespace psc {

// Launch z = s net(r/s) on `st` with s = sqrt(*rr_dev / N), every kernel
// gated by g. The network's grid (psc_net_set_grid) must hold N cells.
int net_launch_apply(psc_net* net, hipStream_t st, const double* r, double* z, const double* rr_dev,
                     long long N, Gate g);
// PSC_OK when the network's grid has n cells.
int net_check_grid(const psc_net* net, long long n);
// Changes whenever buffers captured in a graph are reallocated.
uint64_t net_generation(const psc_net* net);
// The l1-Jacobi alternate of the learned schedule (copies M_0^-1).
int net_create_jacobi(const double* minv_host, long long n, void* hip_stream, psc_net** out);

}  // namespace psc
