// Kernels of the fused D2Q9 step (templates), shared by the per-storage
// translation units and the host API.
#pragma once

// Fused stream-collide step of the GI-corrected preconditioned cascaded
// D2Q9 LBM for gfx950, and the single-lattice C ABI declared in include/lbm.h.
//
// Kernel layout.  A block is 64 x BY threads (BY wave64 wavefronts); each
// thread owns R consecutive lattice rows of one column.  The block's region is
// 64 columns x (BY*R) rows; its outer ring (first/last lane, first/last row)
// is a halo that is pulled and summed to rho but not collided, so the output
// tile is 62 x (BY*R - 2) and neighbouring tiles overlap by two columns/rows.
// Phase 1 pulls the nine populations of every region node (coalesced loads of
// 64 consecutive x per population), writes rho - rho0 to LDS and keeps the
// populations in registers; after one barrier, phase 2 takes the isotropic
// density gradient from LDS, collides and stores the nine populations with
// coalesced stores.  Halo re-reads are served by L2: one HBM read and one HBM
// write of each population per step.  Tiles whose region and sources are
// inside the lattice with no solid node skip every boundary test.
//
// Check steps also accumulate in FP64, per block, sum |u^{n+1}-u^n|^2,
// sum |u^n|^2, sum (rho - rho0) and the guard count (wavefront shuffles, then
// LDS); a one-block kernel adds the block partials in a fixed order.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "lbm_device.h"

namespace lbmk {

constexpr int kLanes = 64;
constexpr int kOutX = kLanes - 2;

enum Flavor : int { kPlain = 0, kStore = 1, kCheck = 2 };

struct StepArgs {
  Geom g;
  int tiles_x, ntiles, out_rows;
  const uint8_t* solid;   // nullptr when the lattice has no solid node
  const uint8_t* tile_fast;
  const void* hist_in;    // outlet history [2][ny] (compute type)
  void* hist_out;
  void* ubuf;             // [2][ny][nx] previous velocity (compute type)
  double* partials;       // [ntiles][4]
};

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).
// Give each XCD one contiguous range of tiles so that tiles sharing halo
// columns and rows also share an L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = b & 7, i = b >> 3;
  return x * q + (x < rem ? x : rem) + i;
}

template <class C>
__device__ __forceinline__ C wave_sum(C v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <class S, int BY, int R, int FL>
__global__ __launch_bounds__(kLanes* BY) void step_kernel(const typename S::T* __restrict__ fa,
                                                          typename S::T* __restrict__ fb,
                                                          const StepArgs args,
                                                          const Consts<typename S::C> k) {
  using C = typename S::C;
  using T = typename S::T;
  constexpr int RR = BY * R;  // region rows
  __shared__ C s_rho[RR][kLanes];
  __shared__ double s_red[BY][4];

  const Geom& g = args.g;
  const int lane = threadIdx.x;
  const int w = threadIdx.y;
  const int tile = xcd_tile(blockIdx.x, args.ntiles);
  const int tx = tile % args.tiles_x;
  const int ty = tile / args.tiles_x;
  const int x = tx * kOutX - 1 + lane;
  const int y0 = ty * args.out_rows - 1 + w * R;
  const bool fast = args.tile_fast[tile] != 0;
  const C* hist_in = static_cast<const C*>(args.hist_in);

  C d[R][9];
  bool live[R];  // fluid node whose rho was computed
  C us_r[R], vs_r[R];
  bool outl_r[R];

#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = y0 + r;
    live[r] = false;
    outl_r[r] = false;
    C drho = C(0);
    if (fast) {
      // region and every source inside the lattice, all fluid
      const long long own = (long long)y * g.nx + x;
#pragma unroll
      for (int a = 0; a < 9; ++a)
        d[r][a] = S::dec(fa[(long long)a * g.plane + own - ex_of(a) - (long long)ey_of(a) * g.nx],
                         k.inv_scale);
      live[r] = true;
    } else if (x >= -1 && x <= g.nx && y >= -1 && y <= g.ny) {
      int gx = x, gy = y;
      bool ok = true;
      if (gx < 0 || gx >= g.nx) {
        if (g.side[gx < 0 ? kW : kE] == kPeriodic) gx = gx < 0 ? gx + g.nx : gx - g.nx;
        else ok = false;
      }
      if (gy < 0 || gy >= g.ny) {
        if (g.side[gy < 0 ? kS : kN] == kPeriodic) gy = gy < 0 ? gy + g.ny : gy - g.ny;
        else ok = false;
      }
      if (ok && args.solid && args.solid[(long long)gy * g.nx + gx]) ok = false;
      if (ok) {
        outl_r[r] = pull_node_general<S>(fa, args.solid, g, k, hist_in, gx, gy, d[r], us_r[r],
                                         vs_r[r]);
        live[r] = true;
      }
    }
    if (live[r]) {
      drho = ((d[r][0] + d[r][1]) + (d[r][2] + d[r][3])) +
             ((d[r][4] + d[r][5]) + (d[r][6] + d[r][7])) + d[r][8];
    }
    s_rho[w * R + r][lane] = live[r] ? drho : C(HUGE_VALF);
  }
  __syncthreads();

  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0, acc3 = 0.0;
  C* ubuf = static_cast<C*>(args.ubuf);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int ry = w * R + r;
    const int y = y0 + r;
    const bool out = live[r] && lane >= 1 && lane <= kOutX && ry >= 1 && ry <= RR - 2 &&
                     x < g.nx && y < g.ny;
    if (!out) continue;
    const C own = s_rho[ry][lane];
    auto nb = [&](int dy, int dx) -> C {
      const C v = s_rho[ry + dy][lane + dx];
      return v == C(HUGE_VALF) ? own : v;
    };
    C drx, dry;
    if (k.stencil == 0) {
      // isotropic: d rho = 3 sum_a w_a e_a rho(x + e_a)
      const C ne = nb(1, 1), nw = nb(1, -1), se = nb(-1, 1), sw = nb(-1, -1);
      drx = (nb(0, 1) - nb(0, -1)) * (C(1) / C(3)) + ((ne - nw) + (se - sw)) * (C(1) / C(12));
      dry = (nb(1, 0) - nb(-1, 0)) * (C(1) / C(3)) + ((ne - se) + (nw - sw)) * (C(1) / C(12));
    } else {
      drx = C(0.5) * (nb(0, 1) - nb(0, -1));
      dry = C(0.5) * (nb(1, 0) - nb(-1, 0));
    }
    C drho, ux, uy;
    const int gd = collide<C>(d[r], drx, dry, k, drho, ux, uy);
    const long long own_i = (long long)y * g.nx + x;
#pragma unroll
    for (int a = 0; a < 9; ++a) fb[(long long)a * g.plane + own_i] = S::enc(d[r][a], k.scale);
    if (outl_r[r]) {
      C* ho = static_cast<C*>(args.hist_out);
      ho[y] = us_r[r];
      ho[g.ny + y] = vs_r[r];
    }
    if (FL == kCheck) {
      const double px = ubuf[own_i], py = ubuf[g.plane + own_i];
      const double dx = double(ux) - px, dy = double(uy) - py;
      acc0 += dx * dx + dy * dy;
      acc1 += px * px + py * py;
      acc2 += double(drho);
      acc3 += double(gd);
    }
    if (FL == kStore || FL == kCheck) {
      ubuf[own_i] = ux;
      ubuf[g.plane + own_i] = uy;
    }
  }
  if (FL == kCheck) {
    acc0 = wave_sum(acc0);
    acc1 = wave_sum(acc1);
    acc2 = wave_sum(acc2);
    acc3 = wave_sum(acc3);
    if (lane == 0) {
      s_red[w][0] = acc0;
      s_red[w][1] = acc1;
      s_red[w][2] = acc2;
      s_red[w][3] = acc3;
    }
    __syncthreads();
    if (lane < 4 && w == 0) {
      double t = 0.0;
      for (int i = 0; i < BY; ++i) t += s_red[i][lane];
      args.partials[(long long)tile * 4 + lane] = t;
    }
  }
}

// Launch one fused step for a given storage type (defined in lbm_step_<type>.hip).
void launch_step_f64(int by, int rows, int flavor, const void* src, void* dst, const StepArgs& a,
                     const Consts<double>& k, int ntiles, hipStream_t st);
void launch_step_f32(int by, int rows, int flavor, const void* src, void* dst, const StepArgs& a,
                     const Consts<float>& k, int ntiles, hipStream_t st);
void launch_step_bf16(int by, int rows, int flavor, const void* src, void* dst, const StepArgs& a,
                      const Consts<float>& k, int ntiles, hipStream_t st);
void launch_step_f16(int by, int rows, int flavor, const void* src, void* dst, const StepArgs& a,
                     const Consts<float>& k, int ntiles, hipStream_t st);

}  // namespace lbmk
