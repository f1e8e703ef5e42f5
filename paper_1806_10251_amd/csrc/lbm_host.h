// Host-side helpers shared by the single-lattice and batch C ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "../../include/lbm.h"
#include "lbm_device.h"

namespace lbmh {

using lbmk::Consts;
using lbmk::Geom;

// Records the message for lbm_last_error() on this thread; returns code.
int fail(int code, const std::string& msg);

#define HIPCHECK(expr)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::lbmh::fail(LBM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline size_t storage_bytes(int storage) {
  switch (storage) {
    case LBM_STORE_F64: return 8;
    case LBM_STORE_F32: return 4;
    default: return 2;
  }
}

// Constants of one lattice, derived from nu, gamma and the free rates
// (w4 = w5 = 1/(3 nu/gamma + 1/2), eq. 49).
template <class C>
inline Consts<C> make_consts(const lbm_params& p, double scale) {
  const double g = p.gamma;
  const double w4 = 1.0 / (3.0 * p.nu / g + 0.5);
  Consts<C> k{};
  k.rho0 = C(p.rho0);
  k.ig = C(1.0 / g);
  k.third = C(p.gi_correct ? 3.0 / g - 1.0 / (g * g) : 2.0);
  k.A = C(4.0 / (g * g) - 1.0 / g);
  k.B = C(1.0 / (g * g) - 1.0 / g);
  k.Cg = C(1.0 / g - 1.0);
  k.h3 = C(1.0 / p.omega3 - 0.5);
  k.h4 = C(1.0 / w4 - 0.5);
  k.h5 = C(1.0 / w4 - 0.5);
  k.a3 = C(2.0 / (3.0 * p.omega3));
  k.a4 = C(2.0 / (3.0 * w4));
  k.w3 = C(p.omega3);
  k.w4 = C(w4);
  k.w5 = C(w4);
  k.w6 = C(p.omega6);
  k.w7 = C(p.omega7);
  k.w8 = C(p.omega8);
  k.fx = C(p.fx);
  k.fy = C(p.fy);
  k.u_lid = C(p.u_lid);
  k.u_in_max = C(p.u_in_max);
  k.scale = C(scale);
  k.inv_scale = C(1.0 / scale);
  const double h3 = 1.0 / p.omega3 - 0.5, h4 = 1.0 / w4 - 0.5, cg = 1.0 / g - 1.0;
  k.q3 = C(p.omega3 / 12.0);
  k.q4 = C(w4 / 4.0);
  k.q5 = C(w4 / 4.0);
  k.q6 = C(p.omega6 / 4.0);
  k.q7 = C(p.omega7 / 4.0);
  k.q8 = C(p.omega8 / 4.0);
  k.cg3 = C(cg / 3.0);
  k.l3 = C(2.0 / 3.0 * h3 * cg);
  k.l4 = C(2.0 / 3.0 * h4 * cg);
  k.l5 = C(1.0 / 3.0 * h4 * cg);
  k.h5B = C(h4 * (1.0 / (g * g) - 1.0 / g));
  k.d0 = C(-2.0 * (2.0 / (3.0 * p.omega3)) * (2.0 / (3.0 * w4)));
  k.r03 = C(p.rho0 / 3.0);
  k.gi = p.gi_correct ? 1 : 0;
  k.force = (p.fx != 0.0 || p.fy != 0.0) ? 1 : 0;
  k.stencil = p.drho_stencil;
  return k;
}

// Framed, line-aligned layout: column 0 of every row starts a 128-byte line;
// one ghost column/row on each side.
inline Geom make_geom_for(int nx, int ny, const int32_t side[4], size_t esize) {
  Geom g{};
  g.nx = nx;
  g.ny = ny;
  g.sides = 0;
  for (int s = 0; s < 4; ++s) g.sides |= (side[s] & 15) << (4 * s);
  const int line = int(128 / esize);  // elements per 128-byte line
  g.padx = line;
  g.pitch = ((nx + 2 * line) + line - 1) / line * line;
  g.plane = g.pitch * (ny + 2);
  return g;
}

// One lattice (nine framed planes) is read and written through a single
// buffer resource with 32-bit byte offsets, so it must hold fewer than 2^32
// bytes at the given element size (FP32: up to about 10800^2 nodes).
inline int check_lattice_bytes(int nx, int ny, size_t esize) {
  const long long line = 128 / (long long)esize;
  const long long pitch = ((nx + 3 * line) + line - 1) / line * line;   // upper bound
  if (9LL * pitch * (ny + 2) * (long long)esize >= (1LL << 32))
    return fail(LBM_EINVAL, "lattice too large for this storage (its nine framed planes must "
                            "hold fewer than 2^32 bytes)");
  return LBM_OK;
}

// Validation shared by lbm_create and lbm_batch_create.
inline int validate(const lbm_grid* grid, const uint8_t* solid, const lbm_params* p) {
  if (!grid || !p) return fail(LBM_EINVAL, "null grid or params");
  if (grid->nx < 2 || grid->ny < 2) return fail(LBM_EINVAL, "nx and ny must be >= 2");
  if (grid->nx > (1 << 30) || grid->ny > (1 << 30)) return fail(LBM_EINVAL, "lattice too large");
  if (p->storage >= LBM_STORE_F64 && p->storage <= LBM_STORE_F16) {
    const int rc = check_lattice_bytes(grid->nx, grid->ny, storage_bytes(p->storage));
    if (rc) return rc;
  }
  for (int s = 0; s < 4; ++s)
    if (grid->side[s] < LBM_SIDE_PERIODIC || grid->side[s] > LBM_SIDE_OUTLET)
      return fail(LBM_EINVAL, "unknown side kind");
  if ((grid->side[0] == LBM_SIDE_PERIODIC) != (grid->side[1] == LBM_SIDE_PERIODIC) ||
      (grid->side[2] == LBM_SIDE_PERIODIC) != (grid->side[3] == LBM_SIDE_PERIODIC))
    return fail(LBM_EINVAL, "a periodic side must face a periodic side");
  for (int s = 0; s < 4; ++s) {
    if (grid->side[s] == LBM_SIDE_INLET && s != 0) return fail(LBM_EINVAL, "INLET only on W");
    if (grid->side[s] == LBM_SIDE_OUTLET && s != 1) return fail(LBM_EINVAL, "OUTLET only on E");
  }
  if (!(p->gamma > 0.0) || !(p->gamma <= 1.0)) return fail(LBM_EINVAL, "gamma must be in (0, 1]");
  if (!(p->nu > 0.0)) return fail(LBM_EINVAL, "nu must be > 0");
  if (p->storage < LBM_STORE_F64 || p->storage > LBM_STORE_F16)
    return fail(LBM_EINVAL, "unknown storage");
  if (p->check_every < 1) return fail(LBM_EINVAL, "check_every must be >= 1");
  if (p->strain_fd != 0 && p->strain_fd != 1) return fail(LBM_EINVAL, "strain_fd must be 0 or 1");
  if (p->mrt != 0 && p->mrt != 1) return fail(LBM_EINVAL, "mrt must be 0 or 1");
  if (!(p->omega3 >= 0 && p->omega3 < 2) || !(p->omega6 >= 0 && p->omega6 < 2) ||
      !(p->omega7 >= 0 && p->omega7 < 2) || !(p->omega8 >= 0 && p->omega8 < 2))
    return fail(LBM_EINVAL, "omega3/6/7/8 must be in (0, 2) (0 selects 1.0)");
  if (solid) {
    const size_t n = (size_t)grid->nx * grid->ny;
    size_t fluid = 0;
    for (size_t i = 0; i < n; ++i) fluid += solid[i] == 0;
    if (fluid == 0) return fail(LBM_EINVAL, "the mask leaves no fluid node");
  }
  if (grid->side[1] == LBM_SIDE_OUTLET && solid) {
    for (int j = 0; j < grid->ny; ++j)
      if (solid[(size_t)j * grid->nx + grid->nx - 1] || solid[(size_t)j * grid->nx + grid->nx - 2])
        return fail(LBM_EINVAL, "solid nodes next to an OUTLET side");
  }
  return LBM_OK;
}

}  // namespace lbmh
