// Kernels of the fused D2Q9 step (templates), shared by the per-storage
// translation units and the host API.
#pragma once

// Fused stream-collide step of the GI-corrected preconditioned cascaded
// D2Q9 LBM for gfx950.
//
// Kernel layout.  A block is 64 x BY threads (BY wave64 wavefronts) and owns
// one tile of 64 columns x (BY*R - 2) rows; each thread holds R consecutive
// rows of one column.  The block's region adds one halo row above and below
// (pulled by the first/last row of threads) and one halo column left and
// right (pulled by lanes 0 and 63), so that the density gradient at the same
// time level needs no second pass.  Phase 1 pulls the nine populations of
// every region node through the ghost frame (nine independent coalesced
// loads, no boundary logic), writes rho - rho0 to LDS (a sentinel for solid
// or outside nodes) and keeps the populations in registers; after one
// barrier, phase 2 takes the density gradient from LDS, collides, stores the
// nine populations with coalesced full-line stores and, on boundary nodes
// only, writes the bounce-back and periodic values into the ghost/solid slots
// of the destination lattice.  The outlet column is the one node set with
// extra work (non-equilibrium extrapolation from column nx-2).  Halo re-reads
// are served by L2: one HBM read and one HBM write of each population per
// step.  Tiles are mapped to blocks XCD by XCD so that neighbouring tiles
// share an L2.
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

enum Flavor : int { kPlain = 0, kStore = 1, kCheck = 2 };

struct StepArgs {
  Geom g;
  int tiles_x, ntiles, out_rows;
  const uint8_t* solid;   // [ny][nx], nullptr when the lattice has no solid node
  const void* hist_in;    // outlet history [2][ny] (compute type)
  void* hist_out;
  void* ubuf;             // [2][ny][nx] previous velocity (compute type)
  double* partials;       // [ntiles][4]
  const void* force;      // [2][ny][nx] compute type, always readable (the outlet reads
                          // it unconditionally): the per-node body force when
  int has_force;          // has_force != 0, else any buffer of that size (the uniform
                          // force of the constants applies)
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

template <class C>
__device__ __forceinline__ C sum9(const C d[9]) {
  return ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
}

// Per-node epilogue: store populations, velocity buffer and residual partials.
// li: index in the (framed) lattice; fi: index in the nx*ny field arrays.
// NTS: non-temporal population stores (the written lattice is not read again
// before the next step has streamed the whole lattice through the caches).
template <class S, int FL, bool NTS = false>
__device__ __forceinline__ void finish_node(typename S::T* __restrict__ fb, const StepArgs& args,
                                            const Consts<typename S::C>& k, const typename S::C d[9],
                                            int li, int fi, typename S::C drho,
                                            typename S::C ux, typename S::C uy, int guarded,
                                            double acc[4]) {
  using C = typename S::C;
  const Geom& g = args.g;
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    if constexpr (NTS)
      __builtin_nontemporal_store(S::enc(d[a], k.scale), &fb[a * g.plane + li]);
    else
      fb[a * g.plane + li] = S::enc(d[a], k.scale);
  }
  C* ubuf = static_cast<C*>(args.ubuf);
  const int np = g.nx * g.ny;
  if (FL == kCheck) {
    const double px = ubuf[fi], py = ubuf[np + fi];
    const double dx = double(ux) - px, dy = double(uy) - py;
    acc[0] += dx * dx + dy * dy;
    acc[1] += px * px + py * py;
    acc[2] += double(drho);
    acc[3] += double(guarded);
  }
  if (FL == kStore || FL == kCheck) {
    ubuf[fi] = ux;
    ubuf[np + fi] = uy;
  }
}

// Check-step partials of one block: wavefront shuffles, then LDS.
template <int BY>
__device__ __forceinline__ void block_partials(double acc[4], double (*s_red)[4], int lane, int w,
                                               double* __restrict__ out) {
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = wave_sum(acc[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 4; ++i) s_red[w][i] = acc[i];
  __syncthreads();
  if (lane < 4 && w == 0) {
    double t = 0.0;
    for (int i = 0; i < BY; ++i) t += s_red[i][lane];
    out[lane] = t;
  }
}

// Velocity of a pulled region node (gx, gy: its clamped lattice coordinates)
// into the LDS slots su, sv, for the finite-difference strain rates; zero
// when the node is not fluid (on = false).  The force is read without a
// branch (see outlet_links).
template <class C>
__device__ __forceinline__ void store_velocity(const C dd[9], bool on, int gx, int gy,
                                               const Consts<C>& k, bool has_force,
                                               const C* __restrict__ force, const Geom& g,
                                               C& su, C& sv) {
  const int fi = gy * g.nx + gx;
  const C ffx = force[fi], ffy = force[g.nx * g.ny + fi];
  C r_, u_, v_;
  macro<C>(dd, k, has_force ? ffx : k.fx, has_force ? ffy : k.fy, r_, u_, v_);
  su = on ? u_ : C(0);
  sv = on ? v_ : C(0);
}

// One tile of the fused step (the body of both the single-lattice kernel and
// the persistent batch kernel).  LDS: s_rho[(BY*R + 2) * 66] of type C,
// s_red[BY * 4]; with FDS (strain rates of the corrections by finite
// differences of the velocity, VAR & kVarFds) also s_u, s_v of the size of
// s_rho.  VAR & kVarMrt: the raw-moment MRT form of the collision.
template <class S, int BY, int R, int FL, bool OBST, bool OUTL, int VAR = 0, bool INT = false>
__device__ __forceinline__ void step_tile(const typename S::T* __restrict__ fa,
                                          typename S::T* __restrict__ fb, const StepArgs& args,
                                          const Consts<typename S::C>& k, int tile,
                                          typename S::C (*s_rho)[kLanes + 2],
                                          double (*s_red)[4],
                                          typename S::C (*s_u)[kLanes + 2] = nullptr,
                                          typename S::C (*s_v)[kLanes + 2] = nullptr) {
  using C = typename S::C;
  constexpr bool FDS = (VAR & kVarFds) != 0;
  constexpr int RO = BY * R;   // output rows of the tile
  constexpr int RR = RO + 2;   // region rows (one halo row above and below)
  constexpr int W = kLanes + 2;
  const C SENT = C(HUGE_VALF);
  const Geom& g = args.g;
  const int lane = threadIdx.x;
  const int w = threadIdx.y;
  const int tx = tile % args.tiles_x;
  const int ty = tile / args.tiles_x;
  const int x = tx * kLanes + lane;
  const int ytile = ty * RO;        // first output row of the tile
  const int y0 = ytile + w * R;     // this thread's first row
  const bool halo_lane = lane == 0 || lane == kLanes - 1;
  const int hx = lane == 0 ? x - 1 : x + 1;
  const int hc = lane == 0 ? 0 : W - 1;
  const C* hist_in = static_cast<const C*>(args.hist_in);
  const C* force = static_cast<const C*>(args.force);
  const bool has_force = args.has_force != 0;


  // rho - rho0 of one region row (main lane and, on lanes 0/63, the halo
  // column) into LDS row lr; used for the two halo rows
  auto halo_row = [&](int y, int lr) {
    int gx, gy, hgx, hgy;
    bool ok = region_coords(g, x, y, gx, gy) || INT;
    bool hok = halo_lane && (region_coords(g, hx, y, hgx, hgy) || INT);
    C dm[9], dh[9];
    pull9<S>(fa, g, k, gx, gy, dm);
    if (halo_lane) pull9<S>(fa, g, k, hgx, hgy, dh);
    if (OBST) {
      ok = ok && !args.solid[gy * g.nx + gx];
      if (halo_lane) hok = hok && !args.solid[hgy * g.nx + hgx];
    }
    if (OUTL) {
      C a_, b_;
      if (ok && gx == g.nx - 1) outlet_links<S>(fa, g, k, has_force, force, hist_in, gy, dm, a_, b_);
      if (hok && hgx == g.nx - 1) outlet_links<S>(fa, g, k, has_force, force, hist_in, hgy, dh, a_, b_);
    }
    s_rho[lr][lane + 1] = ok ? sum9<C>(dm) : SENT;
    if (halo_lane) s_rho[lr][hc] = hok ? sum9<C>(dh) : SENT;
    if (FDS) {
      store_velocity<C>(dm, ok, gx, gy, k, has_force, force, g, s_u[lr][lane + 1],
                        s_v[lr][lane + 1]);
      if (halo_lane)
        store_velocity<C>(dh, hok, hgx, hgy, k, has_force, force, g, s_u[lr][hc], s_v[lr][hc]);
    }
  };

  // ---- phase 1: one batch of loads per row (main node, halo column, mask),
  // then rho - rho0 to LDS (sentinel for solid / outside nodes).  The first
  // and the last wavefront also pull the halo rows.
  C d[R][9], dh[R][9];
  C us[R], vs[R];
  bool ok[R], hok[R];
  int gxr[R], gyr[R], hgx[R], hgy[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int y = y0 + r;
    ok[r] = region_coords(g, x, y, gxr[r], gyr[r]) || INT;
    hok[r] = halo_lane && (region_coords(g, hx, y, hgx[r], hgy[r]) || INT);
    pull9<S>(fa, g, k, gxr[r], gyr[r], d[r]);
    if (halo_lane) pull9<S>(fa, g, k, hgx[r], hgy[r], dh[r]);
    if (OBST) {
      ok[r] = ok[r] && !args.solid[gyr[r] * g.nx + gxr[r]];
      if (halo_lane) hok[r] = hok[r] && !args.solid[hgy[r] * g.nx + hgx[r]];
    }
  }
  if (w == 0) halo_row(ytile - 1, 0);
  if (w == BY - 1) halo_row(ytile + RO, RR - 1);
  if (OUTL) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (ok[r] && gxr[r] == g.nx - 1) outlet_links<S>(fa, g, k, has_force, force, hist_in, gyr[r], d[r], us[r], vs[r]);
      if (hok[r] && hgx[r] == g.nx - 1) {
        C a_, b_;
        outlet_links<S>(fa, g, k, has_force, force, hist_in, hgy[r], dh[r], a_, b_);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    s_rho[w * R + r + 1][lane + 1] = ok[r] ? sum9<C>(d[r]) : SENT;
    if (halo_lane) s_rho[w * R + r + 1][hc] = hok[r] ? sum9<C>(dh[r]) : SENT;
    if (FDS) {
      const int lr = w * R + r + 1;
      store_velocity<C>(d[r], ok[r], gxr[r], gyr[r], k, has_force, force, g, s_u[lr][lane + 1],
                        s_v[lr][lane + 1]);
      if (halo_lane)
        store_velocity<C>(dh[r], hok[r], hgx[r], hgy[r], k, has_force, force, g, s_u[lr][hc],
                          s_v[lr][hc]);
    }
  }
  __syncthreads();

  // ---- phase 2: gradient, collision, stores, boundary slots
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int ry = w * R + r + 1;  // LDS row
    const int y = y0 + r;
    if (x >= g.nx || y >= g.ny) continue;
    const int c = lane + 1;
    const C own = s_rho[ry][c];
    if (!INT && own == SENT) continue;  // solid node
    // the eight neighbours, sentinel = solid or outside a non-periodic side
    const C nE = s_rho[ry][c + 1], nW = s_rho[ry][c - 1];
    const C nN = s_rho[ry + 1][c], nS = s_rho[ry - 1][c];
    const C nNE = s_rho[ry + 1][c + 1], nNW = s_rho[ry + 1][c - 1];
    const C nSE = s_rho[ry - 1][c + 1], nSW = s_rho[ry - 1][c - 1];
    auto sub = [&](C v) { return (!INT && v == SENT) ? own : v; };
    C drx, dry;
    if (k.stencil == 0) {
      // isotropic: d rho = 3 sum_a w_a e_a rho(x + e_a)
      const C ne = sub(nNE), nw = sub(nNW), se = sub(nSE), sw = sub(nSW);
      drx = (sub(nE) - sub(nW)) * (C(1) / C(3)) + ((ne - nw) + (se - sw)) * (C(1) / C(12));
      dry = (sub(nN) - sub(nS)) * (C(1) / C(3)) + ((ne - se) + (nw - sw)) * (C(1) / C(12));
    } else {
      drx = C(0.5) * (sub(nE) - sub(nW));
      dry = C(0.5) * (sub(nN) - sub(nS));
    }
    C sxx = C(0), syy = C(0);
    if (FDS) {
      // d_x u_x and d_y u_y with the density-gradient stencil and neighbour rule
      auto su = [&](int rr, int cc) { return s_rho[rr][cc] == SENT ? s_u[ry][c] : s_u[rr][cc]; };
      auto sv = [&](int rr, int cc) { return s_rho[rr][cc] == SENT ? s_v[ry][c] : s_v[rr][cc]; };
      if (k.stencil == 0) {
        sxx = (su(ry, c + 1) - su(ry, c - 1)) * (C(1) / C(3)) +
              ((su(ry + 1, c + 1) - su(ry + 1, c - 1)) + (su(ry - 1, c + 1) - su(ry - 1, c - 1))) *
                  (C(1) / C(12));
        syy = (sv(ry + 1, c) - sv(ry - 1, c)) * (C(1) / C(3)) +
              ((sv(ry + 1, c + 1) - sv(ry - 1, c + 1)) + (sv(ry + 1, c - 1) - sv(ry - 1, c - 1))) *
                  (C(1) / C(12));
      } else {
        sxx = C(0.5) * (su(ry, c + 1) - su(ry, c - 1));
        syy = C(0.5) * (sv(ry + 1, c) - sv(ry - 1, c));
      }
    }
    C fx = k.fx, fy = k.fy;
    if (has_force) {
      fx = force[y * g.nx + x];
      fy = force[g.nx * g.ny + y * g.nx + x];
    }
    C drho, ux, uy;
    const int gd = collide<C, VAR>(d[r], drx, dry, k, fx, fy, drho, ux, uy, sxx, syy);
    finish_node<S, FL, (VAR & kVarNts) != 0>(fb, args, k, d[r], gidx(g, x, y), y * g.nx + x, drho, ux, uy,
                       gd, acc);
    // boundary links: source of link a is the neighbour at -e_a
    const bool any_nf = (nE == SENT) | (nW == SENT) | (nN == SENT) | (nS == SENT) |
                        (nNE == SENT) | (nNW == SENT) | (nSE == SENT) | (nSW == SENT);
    const bool edge = x == 0 || x == g.nx - 1 || y == 0 || y == g.ny - 1;
    if (!INT && (any_nf || edge)) {
      auto nonfluid = [&](int a) {
        const int sx = -ex_of(a), sy = -ey_of(a);
        const C v = sy == 0 ? (sx > 0 ? nE : nW)
                            : (sy > 0 ? (sx > 0 ? nNE : (sx < 0 ? nNW : nN))
                                      : (sx > 0 ? nSE : (sx < 0 ? nSW : nS)));
        return v == SENT;
      };
      ghost_writes<S>(fb, g, k, x, y, d[r], nonfluid);
    }
    if (OUTL && x == g.nx - 1) {
      C* ho = static_cast<C*>(args.hist_out);
      ho[y] = us[r];
      ho[g.ny + y] = vs[r];
    }
  }
  if (FL == kCheck) block_partials<BY>(acc, s_red, lane, w, args.partials + (long long)tile * 4);
}

template <class S, int BY, int R, int FL, bool OBST, bool OUTL, int VAR = 0>
__global__ __launch_bounds__(kLanes* BY) void step_kernel(const typename S::T* __restrict__ fa,
                                                          typename S::T* __restrict__ fb,
                                                          const StepArgs args,
                                                          const Consts<typename S::C> k) {
  using C = typename S::C;
  __shared__ C s_rho[BY * R + 2][kLanes + 2];
  __shared__ double s_red[BY][4];
  constexpr bool FDS = (VAR & kVarFds) != 0;
  __shared__ C s_uv[FDS ? 2 : 1][FDS ? BY * R + 2 : 1][kLanes + 2];
  const int tile = xcd_tile(blockIdx.x, args.ntiles);
  if constexpr (!OBST && (VAR & ~kVarNts) == 0) {
    // a tile whose region (with its halo ring) keeps one node away from every
    // side has no boundary link, no solid or outside neighbour and no outlet
    // node: it takes the path without those checks (default kernel only;
    // measured 1.6 % faster at 1024^2)
    const int x0 = (tile % args.tiles_x) * kLanes, y0 = (tile / args.tiles_x) * (BY * R);
    if (x0 >= 2 && x0 + kLanes + 1 <= args.g.nx - 2 && y0 >= 2 &&
        y0 + BY * R + 1 <= args.g.ny - 2) {
      step_tile<S, BY, R, FL, OBST, OUTL, VAR, true>(fa, fb, args, k, tile, s_rho, s_red,
                                                     s_uv[0], s_uv[FDS ? 1 : 0]);
      return;
    }
  }
  step_tile<S, BY, R, FL, OBST, OUTL, VAR>(fa, fb, args, k, tile, s_rho, s_red, s_uv[0],
                                           s_uv[FDS ? 1 : 0]);
}

// One fused step over all tiles (one block per tile).  var selects the
// instantiation (kVarFds: strain rates from finite differences of the
// velocity; kVarMrt: raw-moment MRT collision); it is passed here rather than
// in the constants because the kernel-argument layout of the default step is
// kept as it is (one more word in Consts re-packs its scalar loads and costs
// about 3 %).
void launch_step_f64(int by, int rows, int flavor, int var, const void* src, void* dst,
                     const StepArgs& a, const Consts<double>& k, hipStream_t st);
void launch_step_f32(int by, int rows, int flavor, int var, const void* src, void* dst,
                     const StepArgs& a, const Consts<float>& k, hipStream_t st);
void launch_step_bf16(int by, int rows, int flavor, int var, const void* src, void* dst,
                     const StepArgs& a, const Consts<float>& k, hipStream_t st);
void launch_step_f16(int by, int rows, int flavor, int var, const void* src, void* dst,
                     const StepArgs& a, const Consts<float>& k, hipStream_t st);

}  // namespace lbmk
