// Kernels of the fused D2Q9 step (templates), shared by the per-storage
// translation units and the host API.
#pragma once

// Fused stream-collide step of the GI-corrected preconditioned cascaded
// D2Q9 LBM for gfx950.
//
// Kernel layout.  A block is 64 x BY threads (BY wave64 wavefronts) and owns
// one tile of 64 columns x BY*R rows; each thread holds R consecutive rows of
// one column.  The density gradient at the same time level needs rho on the
// one-node ring around the tile too.  Phase 1 pulls the nine populations of
// every tile node through the ghost frame (nine coalesced loads per row, all
// at one per-lane byte offset: the direction's plane and streaming shift ride
// in the scalar base of a buffer resource), keeps them in registers and writes
// rho - rho0 to LDS (a sentinel for solid or outside nodes).  The ring costs
// little: the first and the last wavefront pull the halo row above and below
// the tile, and the two halo columns are loaded cooperatively, one population
// per lane (16-lane groups, one group per halo node, nine lanes used), their
// nine values summed across the group in the order of the per-node sum, so a
// halo rho equals, bit for bit, the rho its own tile computes.  After one
// barrier, phase 2 takes the density gradient from LDS, collides, stores the
// nine populations with coalesced full-line stores and, on boundary nodes
// only, writes the bounce-back and periodic values into the ghost/solid slots
// of the destination lattice.  The outlet column is the one node set with
// extra work (non-equilibrium extrapolation from column nx-2).  Halo re-reads
// are served by L2: one HBM read and one HBM write of each population per
// step.  Tiles are mapped to blocks XCD by XCD so that neighbouring tiles
// share an L2.  The finite-difference strain variant also needs the velocity
// on the ring; there lanes 0 and 63 pull the halo columns node by node.
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
  // step counter of the stochastic rounding of 16-bit storages: a kernel
  // reads rng[rng_slot] (the step index) and one thread writes that plus one
  // to rng[rng_slot ^ 1], the slot the next step reads (the source lattice
  // alternates every step); nullptr for storages rounded to nearest
  unsigned* rng;
  int rng_slot;
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
                                            double acc[4], uint32_t rng_step = 0) {
  using C = typename S::C;
  using T = typename S::T;
  const Geom& g = args.g;
  const uint32_t off = uint32_t(li) * uint32_t(sizeof(T));
  const Rsrc r = lattice_rsrc(fb);
  if constexpr (S::kSR) {
    // one hash of (node, step) per node; the nine seeds step through a Weyl
    // sequence from it
    const uint32_t h = hash32(uint32_t(li) * 0x9E3779B1u ^ hash32(rng_step));
#pragma unroll
    for (int a = 0; a < 9; ++a)
      Buf<T>::template st<NTS ? 2 : 0>(r, off, uint32_t(a * g.plane) * uint32_t(sizeof(T)),
                                       S::enc_sr(d[a], k.scale, h + uint32_t(a) * 0x9E3779B9u));
  } else {
#pragma unroll
    for (int a = 0; a < 9; ++a)
      Buf<T>::template st<NTS ? 2 : 0>(r, off, uint32_t(a * g.plane) * uint32_t(sizeof(T)),
                                       S::enc(d[a], k.scale));
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

// Lane exchange inside rows of 16 lanes (DPP; lanes outside the row read 0).
template <int CTRL>
__device__ __forceinline__ float dpp_get(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_get(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(unsigned(b)), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(unsigned(b >> 32)), CTRL, 0xF, 0xF, true);
  return __builtin_bit_cast(double, (unsigned long long)unsigned(lo) |
                                        ((unsigned long long)unsigned(hi) << 32));
}

// Sum of lanes 0..8 of every 16-lane row (lanes 9..15 hold 0) into lane 0 of
// the row, in the association of sum9: ((d0+d1)+(d2+d3)) + ((d4+d5)+(d6+d7))
// + d8.  Steps: swap neighbours (quad_perm 1,0,3,2), swap pairs (quad_perm
// 2,3,0,1), mirror the half-row (lane 0 takes lane 7, whose partial equals
// lane 4's), shift the row by 8 (lane 0 takes lane 8 = d8).
template <class C>
__device__ __forceinline__ C row16_sum9(C v) {
  v = v + dpp_get<0xB1>(v);
  v = v + dpp_get<0x4E>(v);
  v = v + dpp_get<0x141>(v);
  v = v + dpp_get<0x108>(v);
  return v;
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

// Lattice column / row of a region coordinate: wrapped across a periodic
// side, else mirrored onto the edge node across the half-way wall (the
// region extends one node beyond the lattice; coordinates further out occur
// only in ragged tiles, whose extra nodes feed no output).
template <bool CL>
__device__ __forceinline__ int col_of(const Geom& g, int x) {
  const bool px = periodic_x<CL>(g);
  if (x < 0) return px ? x + g.nx : 0;
  if (x >= g.nx) return px ? (x - g.nx < g.nx ? x - g.nx : g.nx - 1) : g.nx - 1;
  return x;
}
template <bool CL>
__device__ __forceinline__ int row_of(const Geom& g, int y) {
  const bool py = periodic_y<CL>(g);
  if (y < 0) return py ? y + g.ny : 0;
  if (y >= g.ny) return py ? (y - g.ny < g.ny ? y - g.ny : g.ny - 1) : g.ny - 1;
  return y;
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
// the batch kernel).  LDS: s_rho[(BY*R + 2) * 66] of type C, s_red[BY * 4];
// with FDS (strain rates of the corrections by finite differences of the
// velocity, VAR & kVarFds) also s_u, s_v of the size of s_rho.
// VAR & kVarMrt: the raw-moment MRT form of the collision.
//
// Region nodes beyond a non-periodic side hold the density of their mirror
// image across the half-way wall (the clamped lattice node, the density-
// gradient reading at the lattice sides), so only solid nodes carry the
// sentinel (their density is replaced by the differentiating node's own).
template <class S, int BY, int R, int FL, bool OBST, bool OUTL, int VAR = 0, bool INT = false,
          bool CL = false>
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
  const C SENT = C(HUGE_VALF);   // LDS value of a solid region node
  const Geom& g = args.g;
  const int lane = threadIdx.x;
  // blocks are 64 x BY threads: each wavefront is one threadIdx.y, so the
  // row index is wave-uniform (scalar row arithmetic and branches)
  const int w = __builtin_amdgcn_readfirstlane(int(threadIdx.y));
  const int tx = tile % args.tiles_x;
  const int ty = tile / args.tiles_x;
  const int x = tx * kLanes + lane;
  const int ytile = ty * RO;        // first output row of the tile
  const int y0 = ytile + w * R;     // this thread's first row
  const C* hist_in = static_cast<const C*>(args.hist_in);
  const C* force = static_cast<const C*>(args.force);
  const bool has_force = args.has_force != 0;
  const int x0 = tx * kLanes;       // first column of the tile

  // step index of the stochastic rounding (16-bit storages): read here, the
  // next step's written by one thread (tile 0)
  uint32_t rng_step = 0;
  if constexpr (S::kSR) {
    rng_step = __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(args.rng + args.rng_slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    if (tile == 0 && lane == 0 && w == 0)
      __hip_atomic_store(args.rng + (args.rng_slot ^ 1), rng_step + 1u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  }

  // ---- phase 1: every load of the tile is issued before any is used (one
  // memory round trip per wavefront): the own rows (nine loads per row, plus
  // the mask), the halo row of the first / last wavefront, and the
  // cooperative halo-column loads.  Then rho - rho0 to LDS.
  static_assert(BY >= 2, "the first and the last wavefront each pull one halo row");
  // lattice coordinates of the region nodes: the lane's column (per lane),
  // every row (uniform), the two halo columns (uniform)
  const int gx = INT ? x : col_of<CL>(g, x);
  C d[R][9];
  C us[R], vs[R];
  bool sol[R];
  int gyr[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    gyr[r] = INT ? y0 + r : row_of<CL>(g, y0 + r);
    pull9<S>(fa, g, k, gx, gyr[r], d[r]);
    sol[r] = OBST && args.solid[gyr[r] * g.nx + gx];
  }
  // halo row: above the tile for wavefront 0, below it for the last one
  const bool row_wave = w == 0 || w == BY - 1;
  const int hy = w == 0 ? ytile - 1 : ytile + RO;
  const int hlr = w == 0 ? 0 : RR - 1;
  const int hgy = INT ? hy : row_of<CL>(g, hy);
  C dm[9];
  bool hrsol = false;
  if (row_wave) {
    pull9<S>(fa, g, k, gx, hgy, dm);
    hrsol = OBST && args.solid[hgy * g.nx + gx];
  }

  // Region rows whose two halo-column nodes this wavefront provides: its own
  // R rows, and the halo row it pulled (corner nodes).  q-th such row: LDS row
  // and lattice row.
  const int nh = R + (row_wave ? 1 : 0);
  auto halo_rowof = [&](int q, int& lr) {
    if (q < R) {
      lr = w * R + q + 1;
      return gyr[q];
    }
    lr = hlr;
    return hgy;
  };
  const int hxl = INT ? x0 - 1 : col_of<CL>(g, x0 - 1);
  const int hxr = INT ? x0 + kLanes : col_of<CL>(g, x0 + kLanes);
  // A right halo column on (or mirrored onto) the OUTLET column needs the
  // outlet links of its nodes; lane 63 then pulls it node by node (the left
  // column stays cooperative), as the finite-difference variant does for both
  // columns.
  const bool lane_halo = FDS || (OUTL && x0 + kLanes >= g.nx - 1);
  // cooperative halo columns: 16-lane group gr takes pair p = 4 i + gr
  // (region row p / 2, left or right column p % 2), lane sub of the group
  // loads population sub of that node
  constexpr int kHC = (2 * (R + 1) + 3) / 4;
  const int sub = lane & 15, gr = lane >> 4;
  C hc[kHC];
  bool hcsol[kHC];
  int hclr[kHC];
  if (!FDS) {
    // the halo loads go through a pointer the compiler may not assume
    // unaliased, so the memory barrier below keeps them ahead of the LDS work
    using GT = const __attribute__((address_space(1))) typename S::T;
    const typename S::T* fl = uniform_ptr(fa);
    asm volatile("" : "+s"(fl));
    GT* fh = (GT*)fl;
    // e_a of a lane-dependent direction a, from 2-bit fields (e + 1) per
    // direction (no divergent selects)
    const int a = sub < 9 ? sub : 0;
    const int aex = int((0x20919u >> (2 * a)) & 3u) - 1;
    const int aey = int((0x02865u >> (2 * a)) & 3u) - 1;
#pragma unroll
    for (int i = 0; i < kHC; ++i) {
      const int p = 4 * i + gr;
      const bool act = p < 2 * nh;
      const int cy = halo_rowof(act ? (p >> 1) : 0, hclr[i]);
      const int cx = (p & 1) ? hxr : hxl;
      const long long li =
          (long long)a * g.plane + gidx(g, cx, cy) - aex - (long long)aey * g.pitch;
      hc[i] = S::dec(fh[li], k.inv_scale);
      hcsol[i] = OBST && args.solid[cy * g.nx + cx];
      if (!act || sub >= 9) hc[i] = C(0);
    }
  }

  // every load above is issued before anything below consumes one (keeps
  // the compiler from interleaving the LDS writes with the halo loads, which
  // would cost one memory round trip per group of loads)
  __builtin_amdgcn_sched_barrier(0);
  asm volatile("" ::: "memory");

  // a node on the outlet column completes its links (non-equilibrium
  // extrapolation from column nx - 2); so does a region node mirrored onto it
  if (OUTL) {
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (!sol[r] && gx == g.nx - 1)
        outlet_links<S>(fa, g, k, has_force, force, hist_in, gyr[r], d[r], us[r], vs[r]);
    if (row_wave && !hrsol && gx == g.nx - 1) {
      C a_, b_;
      outlet_links<S>(fa, g, k, has_force, force, hist_in, hgy, dm, a_, b_);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    s_rho[w * R + r + 1][lane + 1] = sol[r] ? SENT : sum9<C>(d[r]);
    if (FDS) {
      const int lr = w * R + r + 1;
      store_velocity<C>(d[r], !sol[r], gx, gyr[r], k, has_force, force, g, s_u[lr][lane + 1],
                        s_v[lr][lane + 1]);
    }
  }
  if (row_wave) {
    s_rho[hlr][lane + 1] = hrsol ? SENT : sum9<C>(dm);
    if (FDS)
      store_velocity<C>(dm, !hrsol, gx, hgy, k, has_force, force, g, s_u[hlr][lane + 1],
                        s_v[hlr][lane + 1]);
  }
  if (!FDS) {
    // both columns, or the left one when lane 63 pulls the right one
    const unsigned cols = lane_halo ? 1u : 3u;
#pragma unroll
    for (int i = 0; i < kHC; ++i) {
      if (4 * i >= 2 * nh) break;
      const int p = 4 * i + gr;
      const C v = row16_sum9<C>(hc[i]);
      if (p < 2 * nh && sub == 0 && ((cols >> (p & 1)) & 1u))
        s_rho[hclr[i]][(p & 1) ? W - 1 : 0] = hcsol[i] ? SENT : v;
    }
  }
  if (lane_halo) {
    const bool halo_lane = FDS ? (lane == 0 || lane == kLanes - 1) : lane == kLanes - 1;
    const int hcol = lane == 0 ? 0 : W - 1;
    for (int q = 0; q < nh; ++q) {
      int lr;
      const int qgy = halo_rowof(q, lr);
      if (halo_lane) {
        const int qgx = lane == 0 ? hxl : hxr;
        C dq[9];
        pull9<S>(fa, g, k, qgx, qgy, dq);
        const bool qsol = OBST && args.solid[qgy * g.nx + qgx];
        if (OUTL && !qsol && qgx == g.nx - 1) {
          C a_, b_;
          outlet_links<S>(fa, g, k, has_force, force, hist_in, qgy, dq, a_, b_);
        }
        s_rho[lr][hcol] = qsol ? SENT : sum9<C>(dq);
        if (FDS)
          store_velocity<C>(dq, !qsol, qgx, qgy, k, has_force, force, g, s_u[lr][hcol],
                            s_v[lr][hcol]);
      }
    }
  }
  __syncthreads();
  const Consts<C>& kc = k;

  // ---- phase 2: gradient, collision, stores, boundary slots
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int ry = w * R + r + 1;  // LDS row
    const int y = y0 + r;
    if (!INT && (x >= g.nx || y >= g.ny)) continue;
    const int c = lane + 1;
    // the eight neighbours (sentinel = solid node)
    const C nE = s_rho[ry][c + 1], nW = s_rho[ry][c - 1];
    const C nN = s_rho[ry + 1][c], nS = s_rho[ry - 1][c];
    const C nNE = s_rho[ry + 1][c + 1], nNW = s_rho[ry + 1][c - 1];
    const C nSE = s_rho[ry - 1][c + 1], nSW = s_rho[ry - 1][c - 1];
    const C own = s_rho[ry][c];
    if (OBST && !INT && own == SENT) continue;  // solid node
    auto sub = [&](C v) { return (OBST && !INT && v == SENT) ? own : v; };
    C drx, dry;
    if (uflag(k.stencil) == 0) {
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
      if (uflag(k.stencil) == 0) {
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
    C fx = kc.fx, fy = kc.fy;
    if (has_force) {
      fx = force[y * g.nx + x];
      fy = force[g.nx * g.ny + y * g.nx + x];
    }
    C drho, ux, uy;
    const int gd = collide<C, VAR>(d[r], drx, dry, kc, fx, fy, drho, ux, uy, sxx, syy);
    finish_node<S, FL, (VAR & kVarNts) != 0>(fb, args, kc, d[r], gidx(g, x, y), y * g.nx + x,
                                             drho, ux, uy, gd, acc, rng_step);
    // boundary slots: links whose source lies beyond a side or is a solid
    // node, populations leaving across a periodic side
    if (!INT) {
      side_slots<S, CL>(fb, g, kc, x, y, x0 == 0, x0 + kLanes >= g.nx, d[r]);
      if (OBST) {
        unsigned src = (nW == SENT ? 1u << 1 : 0u) | (nS == SENT ? 1u << 2 : 0u) |
                       (nE == SENT ? 1u << 3 : 0u) | (nN == SENT ? 1u << 4 : 0u) |
                       (nSW == SENT ? 1u << 5 : 0u) | (nSE == SENT ? 1u << 6 : 0u) |
                       (nNE == SENT ? 1u << 7 : 0u) | (nNW == SENT ? 1u << 8 : 0u);
        // a mirrored halo node that is solid is not a source: the link
        // crosses the side
        src &= ~side_links<CL>(g, x, y);
        solid_slots<S>(fb, g, kc, x, y, d[r], src);
      }
    }
    if (OUTL && x == g.nx - 1) {
      C* ho = static_cast<C*>(args.hist_out);
      ho[y] = us[r];
      ho[g.ny + y] = vs[r];
    }
  }
  if (FL == kCheck) block_partials<BY>(acc, s_red, lane, w, args.partials + (long long)tile * 4);
}

template <class S, int BY, int R, int FL, bool OBST, bool OUTL, int VAR = 0, bool CL = false>
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
      step_tile<S, BY, R, FL, OBST, OUTL, VAR, true, CL>(fa, fb, args, k, tile, s_rho, s_red,
                                                     s_uv[0], s_uv[FDS ? 1 : 0]);
      return;
    }
  }
  step_tile<S, BY, R, FL, OBST, OUTL, VAR, false, CL>(fa, fb, args, k, tile, s_rho, s_red, s_uv[0],
                                           s_uv[FDS ? 1 : 0]);
}

// One fused step over all tiles (one block per tile) for storage code ST
// (LBM_STORE_*) and flavour FL; consts points to the Consts of the storage's
// compute type.  var selects the instantiation (kVarFds: strain rates from
// finite differences of the velocity; kVarMrt: raw-moment MRT collision;
// kVarNts: non-temporal population stores); it is passed here rather than in
// the constants so that the kernel-argument layout of the default step stays
// as small as it is.  Defined in lbm_step.hip, compiled once per (ST, FL).
template <int ST, int FL>
void launch_step(int by, int rows, int var, const void* src, void* dst, const StepArgs& a,
                 const void* consts, hipStream_t st);

}  // namespace lbmk
