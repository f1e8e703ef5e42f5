// Device-side building blocks of the fused D2Q9 step for gfx950:
// storage codecs, the equilibrium, the GI-corrected preconditioned cascaded
// collision and the pull with boundary links.  Shared by the single-lattice
// kernels (lbm_kernels.h) and the persistent batch kernel (lbm_batch.hip).
//
// Populations are held as deviations d_a = f_a - w_a rho0 throughout, so the
// large rest part never enters a rounding step; every moment below is the
// moment of the deviation plus the analytically known moment of w rho0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmk {

enum : int { kPeriodic = 0, kWall = 1, kLid = 2, kInlet = 3, kOutlet = 4 };
enum : int { kW = 0, kE = 1, kS = 2, kN = 3 };

// D2Q9 velocity set, order (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1) (-1,-1) (1,-1).
__host__ __device__ constexpr int ex_of(int a) {
  return a == 1 || a == 5 || a == 8 ? 1 : (a == 3 || a == 6 || a == 7 ? -1 : 0);
}
__host__ __device__ constexpr int ey_of(int a) {
  return a == 2 || a == 5 || a == 6 ? 1 : (a == 4 || a == 7 || a == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int a) {
  return a == 0 ? 0 : (a <= 4 ? ((a + 1) % 4) + 1 : ((a - 3) % 4) + 5);
}
template <class C>
__host__ __device__ constexpr C w_of(int a) {
  return a == 0 ? C(4) / C(9) : (a <= 4 ? C(1) / C(9) : C(1) / C(36));
}

// ---------------------------------------------------------------------------
// Storage codecs.  C is the compute type.
// ---------------------------------------------------------------------------
// enc: round to nearest even.  enc_sr: stochastic rounding (16-bit storages;
// kSR): the stored value is one of the two neighbours of v, the upper one
// with probability equal to v's distance from the lower in units of their
// spacing, drawn from the 32-bit seed; the rounding error then has zero mean,
// so a slowly changing population is not held at a fixed value by
// round-to-nearest (measured on a reduced C4 channel against the FP64
// oracle: FP16 1.0e-2 -> 1.9e-3 U, BF16 0.15 -> 1.8e-2 U).
struct StoreF64 {
  using T = double;
  using C = double;
  static constexpr bool kSR = false;
  static __device__ __forceinline__ C dec(T v, C) { return v; }
  static __device__ __forceinline__ T enc(C v, C) { return v; }
  static __device__ __forceinline__ T enc_sr(C v, C, uint32_t) { return v; }
};
struct StoreF32 {
  using T = float;
  using C = float;
  static constexpr bool kSR = false;
  static __device__ __forceinline__ C dec(T v, C) { return v; }
  static __device__ __forceinline__ T enc(C v, C) { return v; }
  static __device__ __forceinline__ T enc_sr(C v, C, uint32_t) { return v; }
};
// bfloat16 bits in a uint16_t, round-to-nearest-even; scaled by a power of two.
struct StoreBF16 {
  using T = uint16_t;
  using C = float;
  static __device__ __forceinline__ C dec(T v, C inv_scale) {
    return __uint_as_float(uint32_t(v) << 16) * inv_scale;
  }
  static __device__ __forceinline__ T enc(C v, C scale) {
    float s = v * scale;
    if (s != s) return uint16_t(0x7FC0);
    uint32_t u = __float_as_uint(s);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
  }
  static constexpr bool kSR = true;
  static __device__ __forceinline__ T enc_sr(C v, C scale, uint32_t seed) {
    using B2 = __bf16 __attribute__((ext_vector_type(2)));
    B2 r = {};
    r = __builtin_amdgcn_cvt_sr_bf16_f32(r, v * scale, seed, false);
    return uint16_t(__builtin_bit_cast(uint32_t, r) & 0xFFFFu);
  }
};
// IEEE binary16, hardware round-to-nearest-even; scaled by a power of two.
struct StoreF16 {
  using T = _Float16;
  using C = float;
  static __device__ __forceinline__ C dec(T v, C inv_scale) { return float(v) * inv_scale; }
  static __device__ __forceinline__ T enc(C v, C scale) { return _Float16(v * scale); }
  static constexpr bool kSR = true;
  static __device__ __forceinline__ T enc_sr(C v, C scale, uint32_t seed) {
    using H2 = _Float16 __attribute__((ext_vector_type(2)));
    H2 r = {};
    r = __builtin_amdgcn_cvt_sr_f16_f32(r, v * scale, seed, false);
    return r[0];
  }
};

// 32-bit integer hash (the "lowbias32" finaliser of C. Wellons' hash
// prospector): seeds of the stochastic rounding from (node, step).
__device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// ---------------------------------------------------------------------------
// Buffer-resource access to population planes.  A plane is read or written
// through a buffer resource whose 64-bit base already carries the plane
// offset (and, for the pull, the streaming shift of the direction), so the
// nine loads or stores of a node share one 32-bit byte offset and cost no
// per-population vector address arithmetic (the bases are scalar).  The
// resource size bounds the offset by the plane size; every legal offset is
// smaller because of the ghost frame.
// ---------------------------------------------------------------------------
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw 32-bit data format (gfx9 family)

// One resource per lattice; the plane offset rides in the scalar offset
// operand, so every byte offset must fit in 32 bits: the library limits one
// lattice's nine planes to fewer than 2^32 bytes.  The size field is the
// largest value (no range clamping); every access lies inside the lattice.
// The base is wave-uniform by construction; reading it from the first lane
// keeps it in scalar registers where the compiler cannot prove it uniform
// (a case descriptor read from memory inside a persistent kernel).
template <class T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane(uint32_t(a));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(uint32_t(a >> 32));
  return reinterpret_cast<T*>((uint64_t(hi) << 32) | lo);
}
template <class T>
__device__ __forceinline__ Rsrc lattice_rsrc(const T* base) {
  return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(const_cast<T*>(base)), 0,
                                           int(0xFFFFFFFFu), kRsrcWord3);
}
// Scalar byte offset (plane and streaming shift): wave-uniform by construction.
__device__ __forceinline__ int soff(uint32_t so) { return __builtin_amdgcn_readfirstlane(int(so)); }

// Raw loads/stores of one stored element; AUX 2 marks a non-temporal store.
template <class T>
struct Buf;
template <>
struct Buf<float> {
  static __device__ __forceinline__ float ld(Rsrc r, uint32_t off, uint32_t so) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, int(off), soff(so), 0));
  }
  template <int AUX>
  static __device__ __forceinline__ void st(Rsrc r, uint32_t off, uint32_t so, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, int(off), soff(so), AUX);
  }
};
template <>
struct Buf<double> {
  using V2 = __attribute__((ext_vector_type(2))) unsigned int;
  static __device__ __forceinline__ double ld(Rsrc r, uint32_t off, uint32_t so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, int(off), soff(so), 0));
  }
  template <int AUX>
  static __device__ __forceinline__ void st(Rsrc r, uint32_t off, uint32_t so, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, int(off), soff(so), AUX);
  }
};
template <>
struct Buf<uint16_t> {
  static __device__ __forceinline__ uint16_t ld(Rsrc r, uint32_t off, uint32_t so) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, int(off), soff(so), 0);
  }
  template <int AUX>
  static __device__ __forceinline__ void st(Rsrc r, uint32_t off, uint32_t so, uint16_t v) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, int(off), soff(so), AUX);
  }
};
template <>
struct Buf<_Float16> {
  static __device__ __forceinline__ _Float16 ld(Rsrc r, uint32_t off, uint32_t so) {
    return __builtin_bit_cast(_Float16,
                              __builtin_amdgcn_raw_buffer_load_b16(r, int(off), soff(so), 0));
  }
  template <int AUX>
  static __device__ __forceinline__ void st(Rsrc r, uint32_t off, uint32_t so, _Float16 v) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, v), r, int(off), soff(so),
                                          AUX);
  }
};

// ---------------------------------------------------------------------------
// Per-lattice constants (derived once on the host from nu, gamma, omegas).
// ---------------------------------------------------------------------------
template <class C>
struct Consts {
  C rho0;
  C ig;      // 1/gamma
  C third;   // 3/gamma - 1/gamma^2 (Sec. 5) or 2 (eq. 4)
  C A, B, Cg;            // A_gamma, B_gamma, C_gamma
  C h3, h4, h5;          // 1/w - 1/2
  C a3, a4;              // 2/(3 w)
  C w3, w4, w5, w6, w7, w8;
  C fx, fy;              // uniform body force
  C u_lid, u_in_max;
  C scale, inv_scale;    // storage scale (1 for F32/F64)
  // products of the above that every node needs (formed once on the host)
  C q3, q4, q5, q6, q7, q8;  // w3/12, w4/4, w5/4, w6/4, w7/4, w8/4
  C cg3;                     // C_gamma / 3
  C l3, l4, l5;              // (2/3) h3 C_gamma, (2/3) h4 C_gamma, (1/3) h5 C_gamma
  C h5B;                     // h5 B_gamma
  C d0;                      // -2 a3 a4
  C r03;                     // rho0 / 3
  int gi;                // 1: Sec. 5 kernel; 0: eq. 4
  int force;             // body force present
  int stencil;           // 0 isotropic, 1 central
};

// Integer switches of the constants, read as wave-uniform values whether the
// constants sit in scalar registers or in LDS.
__device__ __forceinline__ int uflag(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Lattice geometry and storage layout.  Each population plane holds the
// lattice inside a one-node ghost frame (x = -1 .. nx, y = -1 .. ny); rows are
// padded so that column 0 of every row starts a 128-byte line.  Ghost and
// solid slots hold the values that boundary links pull (written by the fluid
// node that owns them; see ghost_writes), so the pull itself is uniform.
struct Geom {
  int nx, ny;
  int sides;        // kind of side s (kW, kE, kS, kN) in bits 4s .. 4s + 3
  int pitch;        // stored elements per row
  int padx;         // offset of column 0 within a stored row
  int plane;        // pitch * (ny + 2); nine planes hold fewer than 2^32 bytes
};

__host__ __device__ __forceinline__ int side_of(const Geom& g, int s) {
  return (g.sides >> (4 * s)) & 15;
}
// Periodic in x / y.  CL: the lattice is known at compile time to be closed
// (every side a wall or a lid), which removes the periodic, inlet and outlet
// code from a kernel.
template <bool CL = false>
__device__ __forceinline__ bool periodic_x(const Geom& g) {
  return !CL && side_of(g, kW) == kPeriodic;
}
template <bool CL = false>
__device__ __forceinline__ bool periodic_y(const Geom& g) {
  return !CL && side_of(g, kS) == kPeriodic;
}

// Element offsets within a plane and across the nine planes fit in 32 bits
// (enforced at creation), so loads and stores use a 64-bit base plus a
// 32-bit offset.
__host__ __device__ __forceinline__ int gidx(const Geom& g, int x, int y) {
  return (y + 1) * g.pitch + g.padx + x;
}

// Reciprocal: hardware v_rcp_f32 (1 ulp) in FP32, correctly rounded in FP64.
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
__device__ __forceinline__ double rcp(double v) { return 1.0 / v; }

// ---------------------------------------------------------------------------
// Equilibrium deviation f^eq - w rho0 at (rho0 + drho, u): the Sec. 3 raw
// equilibria (orders <= 3), the central fourth-order target rho/9, mapped to
// populations with the inverse of the raw-moment basis.
// ---------------------------------------------------------------------------
template <class C>
__device__ __forceinline__ void equilibrium_dev(C drho, C ux, C uy, const Consts<C>& k, C f[9]) {
  const C rho = k.rho0 + drho;
  const C ig = k.ig;
  const C ux2 = ux * ux, uy2 = uy * uy;
  const C g1 = ig - C(1), g2 = ig - C(2);
  // central targets about u
  const C cxx = rho * (C(1) / C(3) + ux2 * g1);
  const C cyy = rho * (C(1) / C(3) + uy2 * g1);
  const C cxy = rho * ux * uy * g1;
  const C cxxy = rho * ux2 * uy * g1 * g2;
  const C cxyy = rho * ux * uy2 * g1 * g2;
  // raw moments of the deviation (rest moments removed analytically)
  const C m0 = drho;
  const C mx = rho * ux, my = rho * uy;
  const C mxx = drho * (C(1) / C(3)) + rho * ux2 * ig;
  const C myy = drho * (C(1) / C(3)) + rho * uy2 * ig;
  const C mxy = rho * ux * uy * ig;
  const C mxxy = rho * uy * (C(1) / C(3)) + rho * ux2 * uy * ig * ig;
  const C mxyy = rho * ux * (C(1) / C(3)) + rho * ux * uy2 * ig * ig;
  const C mxxyy = drho * (C(1) / C(9)) + C(2) * ux * cxyy + C(2) * uy * cxxy + ux2 * cyy +
                  uy2 * cxx + C(4) * ux * uy * cxy + rho * ux2 * uy2;
  f[0] = m0 - mxx - myy + mxxyy;
  f[1] = C(0.5) * (mx + mxx - mxyy - mxxyy);
  f[2] = C(0.5) * (my + myy - mxxy - mxxyy);
  f[3] = C(0.5) * (-mx + mxx + mxyy - mxxyy);
  f[4] = C(0.5) * (-my + myy + mxxy - mxxyy);
  f[5] = C(0.25) * (mxy + mxxy + mxyy + mxxyy);
  f[6] = C(0.25) * (-mxy + mxxy - mxyy + mxxyy);
  f[7] = C(0.25) * (mxy - mxxy - mxyy + mxxyy);
  f[8] = C(0.25) * (-mxy - mxxy + mxyy + mxxyy);
}

// density deviation and velocity of a post-stream node (forcing shifts the
// momentum by F/(2 gamma)); fx, fy: the body force at this node
template <class C>
__device__ __forceinline__ void macro(const C d[9], const Consts<C>& k, C fx, C fy, C& drho,
                                      C& ux, C& uy) {
  drho = ((d[0] + d[1]) + (d[2] + d[3])) + ((d[4] + d[5]) + (d[6] + d[7])) + d[8];
  C jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
  C jy = (d[2] - d[4]) + (d[5] + d[6]) - (d[7] + d[8]);
  if (uflag(k.force)) {
    jx += C(0.5) * fx * k.ig;
    jy += C(0.5) * fy * k.ig;
  }
  const C inv = rcp(k.rho0 + drho);
  ux = jx * inv;
  uy = jy * inv;
}

// ---------------------------------------------------------------------------
// Collision of one node (eq. 2a with the cascaded kernel of Sec. 5, or eq. 4
// when gi == 0).  d: post-stream deviations in, post-collision deviations out.
// drx, dry: density gradient; fx, fy: the body force at this node (used when
// k.force).  VAR & kVarFds: the strain rates of the corrections are
// sxx = d_x u_x and syy = d_y u_y from finite differences instead of eqs.
// 51-55.  VAR & kVarMrt: the raw-moment MRT form of the collision (eq. 7)
// instead of the cascaded kernel.  Returns whether the strain guard fired.
// VAR & kVarNts changes no arithmetic: the step stores the populations with
// non-temporal stores (lattices larger than the last-level cache).
// ---------------------------------------------------------------------------
constexpr int kVarFds = 1, kVarMrt = 2, kVarNts = 4;

template <class C, int VAR = 0>
__device__ __forceinline__ int collide(C d[9], C drx, C dry, const Consts<C>& k, C fx, C fy,
                                       C& drho_o, C& ux_o, C& uy_o, C sxx = C(0),
                                       C syy = C(0)) {
  const C s56 = d[5] + d[6], s78 = d[7] + d[8];
  const C drho = ((d[0] + d[1]) + (d[2] + d[3])) + (d[4] + (s56 + s78));
  C jx = (d[1] - d[3]) + (d[5] - d[6]) + (d[8] - d[7]);
  C jy = (d[2] - d[4]) + s56 - s78;
  // raw moments of the deviation
  C Kxx = (d[1] + d[3]) + (s56 + s78);
  C Kyy = (d[2] + d[4]) + (s56 + s78);
  C Kxy = (d[5] - d[6]) + (d[7] - d[8]);
  C Kxxy = s56 - s78;
  C Kxyy = (d[5] - d[6]) - (d[7] - d[8]);
  C Kxxyy = s56 + s78;
  if (uflag(k.force)) {
    jx += C(0.5) * fx * k.ig;
    jy += C(0.5) * fy * k.ig;
  }
  const C rho = k.rho0 + drho;
  const C inv_rho = rcp(rho);
  const C ux = jx * inv_rho, uy = jy * inv_rho;
  const C ux2 = ux * ux, uy2 = uy * uy, uxy = ux * uy;
  // source raw moments sigma' (Sec. 3); moments below are those of f = fbar + S/2
  C s[9];
  if (uflag(k.force)) {
    const C ig2 = k.ig * k.ig;
    s[0] = C(0);
    s[1] = fx * k.ig;
    s[2] = fy * k.ig;
    s[3] = C(2) * fx * ux * ig2;
    s[4] = C(2) * fy * uy * ig2;
    s[5] = (fx * uy + fy * ux) * ig2;
    s[6] = fy * ux2 + C(2) * fx * uxy;
    s[7] = fx * uy2 + C(2) * fy * uxy;
    s[8] = C(2) * (fx * ux * uy2 + fy * uy * ux2);
    Kxx += C(0.5) * s[3];
    Kyy += C(0.5) * s[4];
    Kxy += C(0.5) * s[5];
    Kxxy += C(0.5) * s[6];
    Kxyy += C(0.5) * s[7];
    Kxxyy += C(0.5) * s[8];
  }
  // second-order non-equilibrium moments (rest parts cancel: 2 rho0/3 - 2 rho0/3)
  const C m3 = (Kxx + Kyy) - C(2) / C(3) * drho - rho * (ux2 + uy2) * k.ig;
  const C m4 = (Kxx - Kyy) - rho * (ux2 - uy2) * k.ig;

  C D3 = C(0), D4 = C(0), D5 = C(0);
  int guarded = 0;
  if (uflag(k.gi)) {
    const C Aux2 = k.A * ux2, Auy2 = k.A * uy2, Bux2 = k.B * ux2, Buy2 = k.B * uy2;
    // local strain rates from the 2x2 system of eqs. 51-53 (eq. 55, sign of
    // the c~1 term as given by Cramer's rule)
    C dxux = sxx, dyuy = syy;
    const C pg = ux * drx + uy * dry, mg = ux * drx - uy * dry;
    if constexpr (!(VAR & kVarFds)) {
      const C er = k.cg3 * pg;
      const C ert = k.cg3 * mg;
      C c1 = rho * (k.a3 - C(0.5) * (Aux2 + Buy2));
      C c2 = rho * (k.a3 - C(0.5) * (Auy2 + Bux2));
      C ct1 = rho * (k.a4 - C(0.5) * (Aux2 - Buy2));
      C ct2 = rho * (k.a4 - C(0.5) * (Auy2 - Bux2));
      C D = -(c1 * ct2 + ct1 * c2);
      const C D0 = k.d0 * (rho * rho);
      if (D * D0 <= C(0) || fabs(D) < C(0.25) * fabs(D0)) {
        // singular-system guard: the gamma-free (A = B = 0) system
        c1 = c2 = rho * k.a3;
        ct1 = ct2 = rho * k.a4;
        D = D0;
        guarded = 1;
      }
      const C R3 = m3 - er, R4 = m4 - ert;
      const C invD = rcp(D);
      dxux = (ct2 * R3 + c2 * R4) * invD;
      dyuy = (ct1 * R3 - c1 * R4) * invD;
    }
    // extended-equilibrium corrections, eqs. 33 with 45-47
    D3 = -k.h3 * rho * ((Aux2 + Buy2) * dxux + (Auy2 + Bux2) * dyuy) - k.l3 * pg;
    D4 = -k.h4 * rho * ((Aux2 - Buy2) * dxux + (Bux2 - Auy2) * dyuy) - k.l4 * mg;
    D5 = -k.h5B * rho * uxy * (dxux + dyuy) - k.l5 * (uy * drx + ux * dry);
  }
  if constexpr ((VAR & kVarMrt) != 0) {
    // raw-moment MRT (eq. 7): raw moments of f = fbar + S/2 in the basis of
    // eq. 5 relax towards the raw equilibria of Sec. 3 (second order extended
    // by D3, D4, D5); the rest background of the deviations cancels against
    // that of the equilibria (2 rho0/3 in m3, rho0/9 in the fourth order)
    const C ig2 = k.ig * k.ig;
    const C c3 = -k.w3 * (m3 - D3);
    const C c4 = -k.w4 * (m4 - D4);
    const C c5 = -k.w5 * (Kxy - rho * uxy * k.ig - D5);
    const C c6 = -k.w6 * (Kxxy - rho * uy * (C(1) / C(3)) - rho * ux2 * uy * ig2);
    const C c7 = -k.w7 * (Kxyy - rho * ux * (C(1) / C(3)) - rho * ux * uy2 * ig2);
    const C c8 = -k.w8 * (Kxxyy - drho * (C(1) / C(9)) - rho * (ux2 + uy2) * (C(1) / C(3)) -
                          rho * ux2 * uy2);
    // populations from the raw-moment changes (inverse of the basis)
    const C kxx = C(0.5) * (c3 + c4), kyy = C(0.5) * (c3 - c4);
    d[0] += c8 - c3;
    d[1] += C(0.5) * (kxx - c7 - c8);
    d[3] += C(0.5) * (kxx + c7 - c8);
    d[2] += C(0.5) * (kyy - c6 - c8);
    d[4] += C(0.5) * (kyy + c6 - c8);
    d[5] += C(0.25) * (c5 + c6 + c7 + c8);
    d[6] += C(0.25) * (-c5 + c6 - c7 + c8);
    d[7] += C(0.25) * (c5 - c6 - c7 + c8);
    d[8] += C(0.25) * (-c5 - c6 + c7 + c8);
  } else {
  // cascaded moment changes (Sec. 5); K background parts written out:
  // Kxx = rho0/3 + Kxx(dev), Kyy likewise, Kxxyy = rho0/9 + Kxxyy(dev)
  const C r03 = k.r03;
  const C g3 = k.q3 * (D3 - m3);
  const C g4 = k.q4 * (D4 - m4);
  const C g5 = k.q5 * (rho * uxy * k.ig - Kxy + D5);
  const C g6 = k.q6 * (k.third * rho * ux2 * uy + Kxxy - C(2) * ux * Kxy - uy * (r03 + Kxx)) -
               C(0.5) * uy * (C(3) * g3 + g4) - C(2) * ux * g5;
  const C g7 = k.q7 * (k.third * rho * ux * uy2 + Kxyy - C(2) * uy * Kxy - ux * (r03 + Kyy)) -
               C(0.5) * ux * (C(3) * g3 - g4) - C(2) * uy * g5;
  const C g8 = k.q8 *
                   (drho * (C(1) / C(9)) + C(3) * rho * ux2 * uy2 -
                    (Kxxyy - C(2) * ux * Kxyy - C(2) * uy * Kxxy + ux2 * (r03 + Kyy) +
                     uy2 * (r03 + Kxx) + C(4) * uxy * Kxy)) -
               C(2) * g3 - C(0.5) * uy2 * (C(3) * g3 + g4) - C(0.5) * ux2 * (C(3) * g3 - g4) -
               C(4) * uxy * g5 - C(2) * uy * g6 - C(2) * ux * g7;
  // back to populations: f~ = fbar + K g + S (columns of K written per velocity)
  const C t2g3 = C(2) * g3;
  d[0] += C(4) * (g8 - g3);
  d[1] += (g4 - g3) + C(2) * (g7 - g8);
  d[2] += -(g3 + g4) + C(2) * (g6 - g8);
  d[3] += (g4 - g3) - C(2) * (g7 + g8);
  d[4] += -(g3 + g4) - C(2) * (g6 + g8);
  d[5] += t2g3 + g5 - g6 - g7 + g8;
  d[6] += t2g3 - g5 - g6 + g7 + g8;
  d[7] += t2g3 + g5 + g6 + g7 + g8;
  d[8] += t2g3 - g5 + g6 - g7 + g8;
  }
  if (uflag(k.force)) {
    // S = inverse raw-moment map of sigma'
    d[0] += s[0] - s[3] - s[4] + s[8];
    d[1] += C(0.5) * (s[1] + s[3] - s[7] - s[8]);
    d[2] += C(0.5) * (s[2] + s[4] - s[6] - s[8]);
    d[3] += C(0.5) * (-s[1] + s[3] + s[7] - s[8]);
    d[4] += C(0.5) * (-s[2] + s[4] + s[6] - s[8]);
    d[5] += C(0.25) * (s[5] + s[6] + s[7] + s[8]);
    d[6] += C(0.25) * (-s[5] + s[6] - s[7] + s[8]);
    d[7] += C(0.25) * (s[5] - s[6] - s[7] + s[8]);
    d[8] += C(0.25) * (-s[5] - s[6] + s[7] + s[8]);
  }
  drho_o = drho;
  ux_o = ux;
  uy_o = uy;
  return guarded;
}

// ---------------------------------------------------------------------------
// Streaming (eq. 2b) as a pull through the ghost frame: nine independent
// loads, f_a(x - e_a) from plane a, all at the byte offset of node x.
// ---------------------------------------------------------------------------
template <class S>
__device__ __forceinline__ void pull9(const typename S::T* __restrict__ fa, const Geom& g,
                                      const Consts<typename S::C>& k, int x, int y,
                                      typename S::C d[9]) {
  using T = typename S::T;
  const uint32_t off = uint32_t(gidx(g, x, y)) * uint32_t(sizeof(T));
  const Rsrc r = lattice_rsrc(fa);
#pragma unroll
  for (int a = 0; a < 9; ++a) {
    // plane a, shifted by -e_a; non-negative because a * plane > pitch + 1
    const uint32_t so = uint32_t(a * g.plane - ex_of(a) - ey_of(a) * g.pitch) * uint32_t(sizeof(T));
    d[a] = S::dec(Buf<T>::ld(r, off, so), k.inv_scale);
  }
}

// Links of node (nx-1, y) that cross an OUTLET side (e_x = -1, source not a
// corner), as a bit mask over the velocity index.
__device__ __forceinline__ unsigned outlet_mask(const Geom& g, int y) {
  unsigned m = 1u << 3;
  const bool py = side_of(g, kS) == kPeriodic;
  if (y - 1 >= 0 || py) m |= 1u << 6;       // e = (-1, 1): source (nx, y-1)
  if (y + 1 < g.ny || py) m |= 1u << 7;     // e = (-1,-1): source (nx, y+1)
  return m;
}

// Outlet links of node (nx-1, y): non-equilibrium extrapolation from node
// (nx-2, y) at the same time level, with the convective outlet velocity
// u* = (u*_old + U u(nx-2)) / (1 + U) and density rho0.  Returns u*.
// force: a readable [2][ny][nx] buffer of the compute type, always loaded
// (a conditional load here miscompiles for gfx950 inside the halo-row
// lambda); its values are the per-node body force when has_force, else the
// uniform k.fx, k.fy is used.
template <class S>
__device__ __forceinline__ void outlet_links(const typename S::T* __restrict__ fa, const Geom& g,
                                             const Consts<typename S::C>& k, bool has_force,
                                             const typename S::C* __restrict__ force,
                                             const typename S::C* __restrict__ hist_in, int y,
                                             typename S::C d[9], typename S::C& us,
                                             typename S::C& vs) {
  using C = typename S::C;
  C d2[9];
  pull9<S>(fa, g, k, g.nx - 2, y, d2);
  const int fi = y * g.nx + g.nx - 2;
  const C ffx = force[fi], ffy = force[g.nx * g.ny + fi];
  const C fx = has_force ? ffx : k.fx, fy = has_force ? ffy : k.fy;
  C r2, u2, v2;
  macro<C>(d2, k, fx, fy, r2, u2, v2);
  const C U = k.u_in_max;
  const C invU = C(1) / (C(1) + U);
  us = (hist_in[y] + U * u2) * invU;
  vs = (hist_in[g.ny + y] + U * v2) * invU;
  C e2[9], eo[9];
  equilibrium_dev<C>(r2, u2, v2, k, e2);
  equilibrium_dev<C>(C(0), us, vs, k, eo);
  const unsigned m = outlet_mask(g, y);
#pragma unroll
  for (int a = 0; a < 9; ++a)
    if (m & (1u << a)) d[a] = eo[a] + (d2[a] - e2[a]);
}

// Region node (x, y) of a tile (x in -1..nx, y in -1..ny): wrap periodic
// sides.  Returns false when it lies beyond the frame or outside a
// non-periodic side; gx, gy are always valid lattice coordinates (clamped
// when false), so loads can be issued unconditionally.
__device__ __forceinline__ bool region_coords(const Geom& g, int x, int y, int& gx, int& gy) {
  bool ok = x >= -1 && x <= g.nx && y >= -1 && y <= g.ny;
  gx = x;
  gy = y;
  if (gx < 0 || gx >= g.nx) {
    if (side_of(g, kW) == kPeriodic) gx = gx < 0 ? gx + g.nx : gx - g.nx;
    else ok = false;
  }
  if (gy < 0 || gy >= g.ny) {
    if (side_of(g, kS) == kPeriodic) gy = gy < 0 ? gy + g.ny : gy - g.ny;
    else ok = false;
  }
  gx = gx < 0 ? 0 : (gx >= g.nx ? g.nx - 1 : gx);
  gy = gy < 0 ? 0 : (gy >= g.ny ? g.ny - 1 : gy);
  return ok;
}

// Same, also false on a solid node (one dependent mask load).
__device__ __forceinline__ bool region_node(const Geom& g, const uint8_t* __restrict__ solid,
                                            int x, int y, int& gx, int& gy) {
  if (!region_coords(g, x, y, gx, gy)) return false;
  return !(solid && solid[(long long)gy * g.nx + gx]);
}

// Bit masks over the velocity index of the links of node (x, y) whose source
// lies beyond a non-periodic side (e_a points away from that side), and of
// the populations that leave across a periodic side.
template <bool CL = false>
__device__ __forceinline__ unsigned side_links(const Geom& g, int x, int y) {
  const bool px = periodic_x<CL>(g), py = periodic_y<CL>(g);
  unsigned m = 0;
  if (!px && x == 0) m |= (1u << 1) | (1u << 5) | (1u << 8);
  if (!px && x == g.nx - 1) m |= (1u << 3) | (1u << 6) | (1u << 7);
  if (!py && y == 0) m |= (1u << 2) | (1u << 5) | (1u << 6);
  if (!py && y == g.ny - 1) m |= (1u << 4) | (1u << 7) | (1u << 8);
  return m;
}
__device__ __forceinline__ unsigned periodic_links(const Geom& g, int x, int y) {
  const bool px = side_of(g, kW) == kPeriodic, py = side_of(g, kS) == kPeriodic;
  unsigned m = 0;
  if (px && x == 0) m |= (1u << 3) | (1u << 6) | (1u << 7);
  if (px && x == g.nx - 1) m |= (1u << 1) | (1u << 5) | (1u << 8);
  if (py && y == 0) m |= (1u << 4) | (1u << 7) | (1u << 8);
  if (py && y == g.ny - 1) m |= (1u << 2) | (1u << 5) | (1u << 6);
  return m;
}

// Boundary links owned by fluid node (x, y), written into the destination
// lattice after its collision (post-collision deviations d):
//  - half-way bounce-back (eq. 2b with a wall, lid, inlet or solid node at
//    the source), for the links in bounce: the link alpha from a non-fluid
//    source s = x - e_alpha is pulled next step from slot (s, alpha), which
//    receives d_opp(alpha) plus the moving-wall term 6 w_alpha rho0
//    (e_alpha . u_w) (lid: tangential u_lid; inlet: parabolic profile at this
//    node's y; corner and solid sources: stationary).  That slot lies at the
//    node's own offset shifted by -e_alpha in plane alpha, the offset the pull
//    itself uses, so the store needs no per-lane address arithmetic;
//  - periodic sides, for the populations in leave: the population that
//    leaves across a periodic side is copied to the frame slot its wrapped
//    target pulls from.
// Every link test is uniform across the wavefront (wave_bounce, wave_leave:
// the union over its lanes), so a wavefront only executes the links some lane
// needs.
template <class S>
__device__ __forceinline__ void ghost_writes(typename S::T* __restrict__ fb, const Geom& g,
                                             const Consts<typename S::C>& k, int x, int y,
                                             const typename S::C d[9], unsigned bounce,
                                             unsigned leave, unsigned wave_bounce,
                                             unsigned wave_leave) {
  using C = typename S::C;
  using T = typename S::T;
  const bool px = side_of(g, kW) == kPeriodic, py = side_of(g, kS) == kPeriodic;
  if (wave_bounce) {
    const Rsrc r = lattice_rsrc(fb);
    const uint32_t off = uint32_t(gidx(g, x, y)) * uint32_t(sizeof(T));
    // kind of the side crossed in x and in y by this node's links
    const int kx = x == 0 ? side_of(g, kW) : side_of(g, kE);
    const int ky = y == 0 ? side_of(g, kS) : side_of(g, kN);
    const C H = C(g.ny), yy = C(y) + C(0.5);
    const C uin = C(4) * k.u_in_max * yy * (H - yy) * rcp(H * H);
#pragma unroll
    for (int a = 1; a < 9; ++a) {
      if (!((wave_bounce >> a) & 1u)) continue;
      const int ex = ex_of(a), ey = ey_of(a);
      const bool xo = !px && ((ex > 0 && x == 0) || (ex < 0 && x == g.nx - 1));
      const bool yo = !py && ((ey > 0 && y == 0) || (ey < 0 && y == g.ny - 1));
      const int kind = xo ? kx : ky;
      const bool one = xo != yo;   // beyond exactly one side (else corner or solid)
      const C uw = kind == kLid ? (yo ? C(ex) : C(ey)) * k.u_lid
                                : (kind == kInlet ? C(ex) * uin : C(0));
      const C corr = one ? C(6) * w_of<C>(a) * k.rho0 * uw : C(0);
      const bool write = ((bounce >> a) & 1u) && !(one && kind == kOutlet);
      const uint32_t so = uint32_t(a * g.plane - ex - ey * g.pitch) * uint32_t(sizeof(T));
      if (write) Buf<T>::template st<0>(r, off, so, S::enc(d[opp_of(a)] + corr, k.scale));
    }
  }
  if (wave_leave) {
#pragma unroll
    for (int a = 1; a < 9; ++a) {
      if (!((wave_leave >> a) & 1u) || !((leave >> a) & 1u)) continue;
      const int ex = ex_of(a), ey = ey_of(a);
      int tx = x + ex, ty = y + ey;
      bool valid = true;
      if (tx < 0 || tx >= g.nx) {
        if (px) tx = tx < 0 ? tx + g.nx : tx - g.nx;
        else valid = false;
      }
      if (ty < 0 || ty >= g.ny) {
        if (py) ty = ty < 0 ? ty + g.ny : ty - g.ny;
        else valid = false;
      }
      if (valid) fb[(long long)a * g.plane + gidx(g, tx - ex, ty - ey)] = S::enc(d[a], k.scale);
    }
  }
}

// Boundary slots of the fused step, with every test that selects a link
// uniform across the wavefront.  A wavefront covers one lattice row y (so
// "y on the first / last row" is uniform) and 64 consecutive columns from
// x0 (wcol, ecol: the wavefront holds column 0, column nx - 1); the only per-lane
// choice left is which lanes store.  The moving-wall terms are uniform too.
// Each slot is written at the node's own offset plus a uniform shift.
//
// Half-way bounce-back across a side (eq. 2b with a wall, lid or inlet at
// the source, Sec. 6): slot (x - e_a, y - e_a,y) of plane a receives
// d_opp(a) + 6 w_a rho0 (e_a . u_w).  Links through a corner (source beyond
// two non-periodic sides) are stationary and written by the W/E handler; the
// S/N handler takes the links that cross its side only.  An outlet side
// takes no bounce-back (its links are completed by extrapolation), except
// at its corners.
// Periodic sides: the population d_a that leaves across a periodic side goes
// to the frame slot its wrapped target pulls from; corners that wrap on both
// axes are written by the x handler.
template <class S, bool CL = false>
__device__ __forceinline__ void side_slots(typename S::T* __restrict__ fb, const Geom& g,
                                           const Consts<typename S::C>& k, int x, int y,
                                           bool wcol, bool ecol, const typename S::C d[9]) {
  using C = typename S::C;
  using T = typename S::T;
  const bool srow = y == 0, nrow = y == g.ny - 1;
  if (!(wcol || ecol || srow || nrow)) return;
  const bool px = periodic_x<CL>(g), py = periodic_y<CL>(g);
  const Rsrc r = lattice_rsrc(fb);
  const int node = gidx(g, x, y);
  // slot (x + sx, y + sy) of plane a: the plane in the scalar offset (as in
  // every population access), the shift in the vector offset
  struct Slot {
    uint32_t vo, so;
  };
  auto shift = [&](int a, int sx, int sy) {
    return Slot{uint32_t(node + sx + sy * g.pitch) * uint32_t(sizeof(T)),
                uint32_t(a * g.plane) * uint32_t(sizeof(T))};
  };
  auto put = [&](bool on, Slot sl, C v) {
    if (on) Buf<T>::template st<0>(r, sl.vo, sl.so, S::enc(v, k.scale));
  };
  // inlet profile at this row (uniform)
  auto u_inlet = [&]() {
    const C H = C(g.ny), yy = C(y) + C(0.5);
    return C(4) * k.u_in_max * yy * (H - yy) * rcp(H * H);
  };
  // one of the three links a = A0, A1, A2 of side sd (e_a pointing into the
  // lattice across it); on: this lane's node lies on that side
  auto bounce_x = [&](int sd, bool on) {
    const int kind = side_of(g, sd);
    const C ux = !CL && kind == kInlet ? u_inlet() : C(0);
    const C uy = kind == kLid ? k.u_lid : C(0);
    const int A[3] = {sd == kW ? 1 : 3, sd == kW ? 5 : 6, sd == kW ? 8 : 7};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int a = A[i], ex = ex_of(a), ey = ey_of(a);
      const bool corner = !py && ((ey > 0 && srow) || (ey < 0 && nrow));
      if (!CL && !corner && kind == kOutlet) continue;
      const C corr = corner ? C(0) : C(6) * w_of<C>(a) * k.rho0 * (C(ex) * ux + C(ey) * uy);
      put(on, shift(a, -ex, -ey), d[opp_of(a)] + corr);
    }
  };
  auto bounce_y = [&](int sd) {
    const int kind = side_of(g, sd);
    const C ux = kind == kLid ? k.u_lid : C(0);
    const int A[3] = {sd == kS ? 2 : 4, sd == kS ? 5 : 8, sd == kS ? 6 : 7};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int a = A[i], ex = ex_of(a), ey = ey_of(a);
      // lanes whose source also lies beyond a non-periodic W/E side: corner
      const bool on = px || !((ex > 0 && x == 0) || (ex < 0 && x == g.nx - 1));
      const C corr = C(6) * w_of<C>(a) * k.rho0 * C(ex) * ux;
      put(on, shift(a, -ex, -ey), d[opp_of(a)] + corr);
    }
  };
  if (!px) {
    if (wcol) bounce_x(kW, x == 0);
    if (ecol) bounce_x(kE, x == g.nx - 1);
  } else {
    // x-periodic: d_a leaving across W (e_x < 0) or E (e_x > 0)
#pragma unroll
    for (int a = 1; a < 9; ++a) {
      const int ex = ex_of(a), ey = ey_of(a);
      if (ex == 0) continue;
      if (ex < 0 ? !wcol : !ecol) continue;
      const bool on = ex < 0 ? x == 0 : x == g.nx - 1;
      const bool cy = (ey > 0 && nrow) || (ey < 0 && srow);
      if (cy && !py) continue;   // target beyond a wall: bounce-back takes it
      put(on, shift(a, -ex * g.nx, cy ? -ey * g.ny : 0), d[a]);
    }
  }
  if (!py) {
    if (srow) bounce_y(kS);
    if (nrow) bounce_y(kN);
  } else {
    // y-periodic: d_a leaving across S (e_y < 0) or N (e_y > 0); lanes whose
    // target also crosses a W/E side are left to the x handler or to the
    // bounce-back of that side
#pragma unroll
    for (int a = 1; a < 9; ++a) {
      const int ex = ex_of(a), ey = ey_of(a);
      if (ey == 0) continue;
      if (ey < 0 ? !srow : !nrow) continue;
      const bool on = !((ex > 0 && x == g.nx - 1) || (ex < 0 && x == 0));
      put(on, shift(a, 0, -ey * g.ny), d[a]);
    }
  }
}

// Half-way bounce-back from solid nodes inside the lattice (stationary):
// link a of this node whose source is solid (bit a of solid_src; sources
// beyond a non-periodic side excluded) gets slot (x - e_a, y - e_a,y) of
// plane a (unwrapped: across a periodic side that is the frame slot the
// node pulls from) = d_opp(a).
template <class S>
__device__ __forceinline__ void solid_slots(typename S::T* __restrict__ fb, const Geom& g,
                                            const Consts<typename S::C>& k, int x, int y,
                                            const typename S::C d[9], unsigned solid_src) {
  using T = typename S::T;
  if (__builtin_amdgcn_ballot_w64(solid_src != 0) == 0) return;
  const Rsrc r = lattice_rsrc(fb);
  const int node = gidx(g, x, y);
#pragma unroll
  for (int a = 1; a < 9; ++a) {
    const bool on = (solid_src >> a) & 1u;
    if (__builtin_amdgcn_ballot_w64(on) == 0) continue;
    const uint32_t vo = uint32_t(node - ex_of(a) - ey_of(a) * g.pitch) * uint32_t(sizeof(T));
    if (on)
      Buf<T>::template st<0>(r, vo, uint32_t(a * g.plane) * uint32_t(sizeof(T)),
                             S::enc(d[opp_of(a)], k.scale));
  }
}

// Union of a link mask over the active lanes of the wavefront (one ballot per
// link; uniform result, inactive lanes contribute nothing).
__device__ __forceinline__ unsigned wave_or(unsigned m) {
  unsigned r = 0;
#pragma unroll
  for (int a = 1; a < 9; ++a)
    if (__builtin_amdgcn_ballot_w64(((m >> a) & 1u) != 0) != 0) r |= 1u << a;
  return r;
}

}  // namespace lbmk
