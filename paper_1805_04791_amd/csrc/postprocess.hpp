// Launchers of the direct-sum kernels of postprocess.hip.
#pragma once

#include <hip/hip_runtime.h>

#include "cx.hpp"

namespace vie {

// cell-centred grid: point (ix, iy, iz) at (ox, oy, oz) + (i + 1/2) h; the
// sums run over the box [x0, x0 + bx) x [y0, y0 + by) x [z0, z0 + bz) of it,
// outside which the density is zero
struct PostGrid {
  int n;
  double h, ox, oy, oz;
  int x0, y0, z0, bx, by, bz;
};

// doubles of partial sums launch_fields_at / launch_far_field need
long points_partial_doubles(const PostGrid& g, bool maxwell, int npts, int nrhs);
long far_partial_doubles(const PostGrid& g, int C, int ndirs, int nrhs);

// Scattered fields at points pts[npts][3] (device) from the density
// dens[nrhs][C][n^3] (device): out[nrhs][npts][k] complex128, k = 4
// (phi, grad phi) for the scalar problems, 6 (E, H) for Maxwell.
hipError_t launch_fields_at(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* pts, int npts,
                            int nrhs, double w, double* part, c128* out, hipStream_t s);

// Far-field patterns in the unit directions dirs[ndirs][3] (device), g.bx <= 256:
// out[nrhs][ndirs][k], k = 1 (phi_inf) for Helmholtz, 6 (E_inf, H_inf) for Maxwell.
hipError_t launch_far_field(const c128* dens, int C, bool maxwell, const PostGrid& g, const double* dirs, int ndirs,
                            int nrhs, double w, double* part, c128* out, hipStream_t s);

}  // namespace vie
