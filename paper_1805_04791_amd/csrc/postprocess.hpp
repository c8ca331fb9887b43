// Launchers of the direct-sum kernels of postprocess.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "cx.hpp"

namespace vie {

// cell-centred grid: point (ix, iy, iz) at (ox, oy, oz) + (i + 1/2) h
struct PostGrid {
  int n;
  double h, ox, oy, oz;
};

// doubles of partial sums the launchers below need for nitems points (or
// directions), nrhs right-hand sides and nout complex outputs per item
long post_partial_doubles(long n3, int nitems, int nrhs, int nout);

// Scattered fields at points pts[npts][3] (device) from the density
// dens[nrhs][C][n^3] (device): out[nrhs][npts][k] complex128, k = 4
// (phi, grad phi) for the scalar problems, 6 (E, H) for Maxwell.
hipError_t launch_fields_at(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* pts, int npts,
                            int nrhs, double w, double* part, c128* out, hipStream_t s);

// Far-field patterns in the unit directions dirs[ndirs][3] (device):
// out[nrhs][ndirs][k], k = 1 (phi_inf) for Helmholtz, 6 (E_inf, H_inf) for Maxwell.
hipError_t launch_far_field(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* dirs, int ndirs,
                            int nrhs, double w, double* part, c128* out, hipStream_t s);

}  // namespace vie
