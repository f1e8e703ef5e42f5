// Auxiliary kernels shared by the single-lattice API and the batch API:
// fixed-order sum of block partials, equilibrium initialisation, boundary-
// slot fill and export of populations / fields.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbm_device.h"

namespace lbmk {

// cur = (cur + prev) / 2 over whole lattices (frame and solid slots too), in
// the compute precision of the storage type.  Boundary slots hold linear
// functions of the node populations plus constants, so the mean is again a
// consistent lattice.
template <class S>
__global__ __launch_bounds__(256) void average_kernel(typename S::T* __restrict__ cur,
                                                      const typename S::T* __restrict__ prev,
                                                      long long n, typename S::C scale,
                                                      typename S::C inv_scale) {
  using C = typename S::C;
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const C a = S::dec(cur[i], inv_scale), b = S::dec(prev[i], inv_scale);
    cur[i] = S::enc(C(0.5) * (a + b), scale);
  }
}

template <class C>
__global__ __launch_bounds__(256) void average_plain_kernel(C* __restrict__ cur,
                                                            const C* __restrict__ prev,
                                                            long long n) {
  for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    cur[i] = C(0.5) * (cur[i] + prev[i]);
}

// Launch average_kernel for a storage code (LBM_STORE_*); history arrays
// (outlet velocity, compute type) are averaged too when present.
inline hipError_t launch_average(int storage, void* cur, const void* prev, long long n,
                                 double scale, void* hcur, const void* hprev, long long nh,
                                 hipStream_t st) {
  const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
  switch (storage) {
    case 0:
      hipLaunchKernelGGL(average_kernel<StoreF64>, dim3(blocks), dim3(256), 0, st, (double*)cur,
                         (const double*)prev, n, 1.0, 1.0);
      break;
    case 1:
      hipLaunchKernelGGL(average_kernel<StoreF32>, dim3(blocks), dim3(256), 0, st, (float*)cur,
                         (const float*)prev, n, 1.f, 1.f);
      break;
    case 2:
      hipLaunchKernelGGL(average_kernel<StoreBF16>, dim3(blocks), dim3(256), 0, st,
                         (uint16_t*)cur, (const uint16_t*)prev, n, (float)scale,
                         (float)(1.0 / scale));
      break;
    default:
      hipLaunchKernelGGL(average_kernel<StoreF16>, dim3(blocks), dim3(256), 0, st,
                         (_Float16*)cur, (const _Float16*)prev, n, (float)scale,
                         (float)(1.0 / scale));
      break;
  }
  if (hcur && hprev && nh > 0) {
    const int hb = (int)std::min<long long>((nh + 255) / 256, 1024);
    if (storage == 0)
      hipLaunchKernelGGL(average_plain_kernel<double>, dim3(hb), dim3(256), 0, st, (double*)hcur,
                         (const double*)hprev, nh);
    else
      hipLaunchKernelGGL(average_plain_kernel<float>, dim3(hb), dim3(256), 0, st, (float*)hcur,
                         (const float*)hprev, nh);
  }
  return hipGetLastError();
}

// Fixed-order sum of the per-tile partials: out[0..3].
template <int kThreads = 256>
__global__ __launch_bounds__(kThreads) void finalize_kernel(const double* __restrict__ partials,
                                                       int n, double* __restrict__ out) {
  __shared__ double s[4][256];
  const int t = threadIdx.x;
  double a[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = t; i < n; i += 256)
    for (int c = 0; c < 4; ++c) a[c] += partials[(long long)i * 4 + c];
  for (int c = 0; c < 4; ++c) s[c][t] = a[c];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h)
      for (int c = 0; c < 4; ++c) s[c][t] += s[c][t + h];
    __syncthreads();
  }
  if (t < 4) out[t] = s[t][0];
}

// Equilibrium initialisation from optional device fields; also writes the
// velocity buffer and the outlet history.  Interior nodes of both lattices.
template <class S, class FT>
__global__ __launch_bounds__(256) void init_kernel(typename S::T* __restrict__ fa,
                                                   typename S::T* __restrict__ fb, Geom g,
                                                   Consts<typename S::C> k,
                                                   const uint8_t* __restrict__ solid,
                                                   const FT* __restrict__ rho,
                                                   const FT* __restrict__ ux,
                                                   const FT* __restrict__ uy,
                                                   typename S::C* __restrict__ ubuf,
                                                   typename S::C* __restrict__ hist0,
                                                   typename S::C* __restrict__ hist1) {
  using C = typename S::C;
  const long long np = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const bool sol = solid && solid[i];
  C drho = C(0), vx = C(0), vy = C(0);
  if (!sol) {
    if (rho) drho = C(rho[i]) - k.rho0;
    if (ux) vx = C(ux[i]);
    if (uy) vy = C(uy[i]);
  }
  C f[9];
  equilibrium_dev<C>(drho, vx, vy, k, f);
  const int x = int(i % g.nx), y = int(i / g.nx);
  const long long li = gidx(g, x, y);
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    const typename S::T v = S::enc(f[a], k.scale);
    fa[(long long)a * g.plane + li] = v;
    fb[(long long)a * g.plane + li] = v;
  }
  ubuf[i] = vx;
  ubuf[np + i] = vy;
  if (x == g.nx - 1) {
    hist0[y] = vx;
    hist0[g.ny + y] = vy;
    hist1[y] = vx;
    hist1[g.ny + y] = vy;
  }
}

// Boundary slots of a lattice from its own fluid-node values (after an
// initialisation or a checkpoint load).
template <class S>
__global__ __launch_bounds__(256) void ghost_fill_kernel(typename S::T* __restrict__ fa, Geom g,
                                                         Consts<typename S::C> k,
                                                         const uint8_t* __restrict__ solid) {
  using C = typename S::C;
  const long long np = (long long)g.nx * g.ny;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  if (solid && solid[i]) return;
  const int x = int(i % g.nx), y = int(i / g.nx);
  C d[9];
  const long long li = gidx(g, x, y);
#pragma unroll
  for (int a = 0; a < 9; ++a) d[a] = S::dec(fa[a * g.plane + li], k.inv_scale);
  unsigned bounce = side_links(g, x, y);
  if (solid)
    for (int a = 1; a < 9; ++a) {
      int gx, gy;
      if (region_coords(g, x - ex_of(a), y - ey_of(a), gx, gy) && solid[(long long)gy * g.nx + gx])
        bounce |= 1u << a;
    }
  const unsigned leave = periodic_links(g, x, y);
  ghost_writes<S>(fa, g, k, x, y, d, bounce, leave, bounce, leave);
}

// Decode populations (full f) or macroscopic fields of the current lattice,
// for the nodes first .. first + count - 1 (row-major node index); output
// element o of every array belongs to node first + o.
template <class S>
__global__ __launch_bounds__(256) void export_kernel(const typename S::T* __restrict__ fa, Geom g,
                                                     Consts<typename S::C> k,
                                                     const uint8_t* __restrict__ solid,
                                                     const typename S::C* __restrict__ force,
                                                     long long first, long long count,
                                                     double* __restrict__ pops,
                                                     float* __restrict__ rho_o,
                                                     float* __restrict__ ux_o,
                                                     float* __restrict__ uy_o,
                                                     double* __restrict__ rho_d,
                                                     double* __restrict__ ux_d,
                                                     double* __restrict__ uy_d) {
  using C = typename S::C;
  const long long np = (long long)g.nx * g.ny;
  const long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long i = first + o;
  if (o >= count || i >= np) return;
  const long long li = gidx(g, int(i % g.nx), int(i / g.nx));
  C d[9];
#pragma unroll
  for (int a = 0; a < 9; ++a) d[a] = S::dec(fa[a * g.plane + li], k.inv_scale);
  if (pops) {
#pragma unroll
    for (int a = 0; a < 9; ++a)
      pops[a * count + o] = double(d[a]) + double(w_of<C>(a)) * double(k.rho0);
  }
  const bool sol = solid && solid[i];
  // post-collision moments: rho is unchanged by collision; the momentum has
  // received F/gamma, so u = (sum e f~ - F/(2 gamma)) / rho
  C drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
  C jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
  C jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
  if (k.force) {
    // force: per-node field [2][ny][nx], or nullptr for the uniform force
    const C fx = force ? force[i] : k.fx, fy = force ? force[np + i] : k.fy;
    jx -= C(0.5) * fx * k.ig;
    jy -= C(0.5) * fy * k.ig;
  }
  const C rho = k.rho0 + drho;
  const C vx = jx / rho, vy = jy / rho;
  if (rho_o) rho_o[o] = sol ? 0.f : float(rho);
  if (ux_o) ux_o[o] = sol ? 0.f : float(vx);
  if (uy_o) uy_o[o] = sol ? 0.f : float(vy);
  if (rho_d) rho_d[o] = sol ? 0.0 : double(k.rho0) + double(drho);
  if (ux_d) ux_d[o] = sol ? 0.0 : double(vx);
  if (uy_d) uy_d[o] = sol ? 0.0 : double(vy);
}


// Storage conversion of one framed lattice (interior and ghost frame), from
// storage s1 to storage s2 (LBM_STORE_* codes), through FP64.  The two
// layouts may differ in row padding.
__device__ __forceinline__ double load_any(const void* p, int storage, long long i, double inv) {
  switch (storage) {
    case 0: return static_cast<const double*>(p)[i];
    case 1: return double(static_cast<const float*>(p)[i]);
    case 2: return double(StoreBF16::dec(static_cast<const uint16_t*>(p)[i], float(inv)));
    default: return double(StoreF16::dec(static_cast<const _Float16*>(p)[i], float(inv)));
  }
}
__device__ __forceinline__ void store_any(void* p, int storage, long long i, double v,
                                          double scale) {
  switch (storage) {
    case 0: static_cast<double*>(p)[i] = v; break;
    case 1: static_cast<float*>(p)[i] = float(v); break;
    case 2: static_cast<uint16_t*>(p)[i] = StoreBF16::enc(float(v), float(scale)); break;
    default: static_cast<_Float16*>(p)[i] = StoreF16::enc(float(v), float(scale)); break;
  }
}

__global__ __launch_bounds__(256) inline void convert_lattice_kernel(
    const void* __restrict__ src, int s1, Geom g1, double inv1, void* __restrict__ dst, int s2,
    Geom g2, double sc2) {
  const long long nfx = (long long)(g1.nx + 2), nfy = (long long)(g1.ny + 2);
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nfx * nfy) return;
  const int x = int(i % nfx) - 1, y = int(i / nfx) - 1;
  const long long i1 = gidx(g1, x, y), i2 = gidx(g2, x, y);
  for (int a = 0; a < 9; ++a)
    store_any(dst, s2, (long long)a * g2.plane + i2,
              load_any(src, s1, (long long)a * g1.plane + i1, inv1), sc2);
}

// float <-> double copy of small state arrays (velocity buffer, history)
__global__ __launch_bounds__(256) inline void convert_values_kernel(const void* __restrict__ src,
                                                                    int src_double,
                                                                    void* __restrict__ dst,
                                                                    int dst_double, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src_double ? static_cast<const double*>(src)[i]
                              : double(static_cast<const float*>(src)[i]);
  if (dst_double) static_cast<double*>(dst)[i] = v;
  else static_cast<float*>(dst)[i] = float(v);
}

}  // namespace lbmk
