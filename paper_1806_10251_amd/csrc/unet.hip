// Learned warm start: U-Net layers and network on gfx950 with BF16 MFMA.
//
// Convolutions are implicit GEMMs on v_mfma_f32_16x16x32_bf16: for the
// forward pass (and the input gradient, which is the forward pass of the
// flipped, transposed filter) a wave owns 32 pixels x 32 output channels
// (2 x 2 MFMA tiles) and loops over the nine taps and the input channels in
// steps of 32.  NHWC with 8 consecutive channels per lane makes every A and
// B operand one 16-byte load (channels are the reduction dimension).  The
// weight gradient reduces over pixels, which are strided in NHWC: each wave
// stages 32 pixels x 32 channels of both operands through LDS transposed,
// so that the MFMA operands are again 16-byte reads, and the pixel range is
// split over blocks whose FP32 partial sums are added in a fixed order.
//
// MFMA 16x16x32 bf16 lane layout (verified on the device): lane l holds
// A[l % 16][8 (l / 16) + v] and B[8 (l / 16) + v][l % 16] for v < 8, and
// D[4 (l / 16) + v][l % 16] for v < 4.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "unet.h"

namespace {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

thread_local std::string g_err;

int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

#define UCHECK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess)                                                      \
      return fail(UNET_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

inline hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

__device__ __forceinline__ f32x4 mfma16(const bf16x8& a, const bf16x8& b, const f32x4& c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Convolution, forward (also the input gradient with transformed weights)
// ---------------------------------------------------------------------------
struct ConvArgs {
  const bf16* x;
  int ldx;
  const bf16* w;       // [cout][9][cin]
  const float* bias;   // [cout] or null
  void* y;
  int ldy;
  int npix, h, wd, cin, cout;
  int relu, out_f32;
};

// WC: waves along the output channels (1 or 2); 4 / WC waves along pixels.
template <int WC>
__global__ __launch_bounds__(256) void conv_fwd_kernel(ConvArgs a) {
  constexpr int WP = 4 / WC;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int px0 = blockIdx.x * (32 * WP) + 32 * (wv % WP);
  const int co0 = blockIdx.y * (32 * WC) + 32 * (wv / WP);
  const int r = lane & 15, g = lane >> 4;
  int pidx[2], py[2], pxx[2];
  bool pv[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int p = px0 + 16 * s + r;
    pv[s] = p < a.npix;
    const int q = pv[s] ? p : 0;
    pidx[s] = q;
    pxx[s] = q % a.wd;
    py[s] = (q / a.wd) % a.h;
  }
  f32x4 acc[2][2];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[s][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    const bf16* xa[2];
    bool ok[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int yy = py[s] + dy, xx = pxx[s] + dx;
      ok[s] = pv[s] && yy >= 0 && yy < a.h && xx >= 0 && xx < a.wd;
      xa[s] = a.x + (long long)(ok[s] ? pidx[s] + dy * a.wd + dx : 0) * a.ldx + 8 * g;
    }
    const bf16* wb[2];
#pragma unroll
    for (int b = 0; b < 2; ++b)
      wb[b] = a.w + ((long long)(co0 + 16 * b + r) * 9 + t) * a.cin + 8 * g;
    for (int c0 = 0; c0 < a.cin; c0 += 32) {
      bf16x8 A[2], B[2];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        A[s] = *reinterpret_cast<const bf16x8*>(xa[s] + c0);
        if (!ok[s]) A[s] = bf16x8{};
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) B[b] = *reinterpret_cast<const bf16x8*>(wb[b] + c0);
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[s][b] = mfma16(A[s], B[b], acc[s][b]);
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int co = co0 + 16 * b + r;
      const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = px0 + 16 * s + 4 * g + v;
        if (p >= a.npix) continue;
        float val = acc[s][b][v] + bias;
        if (a.relu) val = fmaxf(val, 0.f);
        if (a.out_f32)
          static_cast<float*>(a.y)[(long long)p * a.ldy + co] = val;
        else
          static_cast<bf16*>(a.y)[(long long)p * a.ldy + co] = (bf16)val;
      }
    }
}

// Larger wave tiles for large layers: v_mfma_f32_32x32x16_bf16 (lane l
// holds A[l % 32][8 (l / 32) + v], B[8 (l / 32) + v][l % 32] for v < 8 and
// D[8 (v / 4) + 4 (l / 32) + v % 4][l % 32] for v < 16; verified on the
// device).  A wave owns 64 pixels x (32 CT) output channels: per step of 16
// input channels it loads two pixel operands and CT weight operands and
// issues 2 CT MFMAs, twice the work per loaded byte of the 16x16x32 tiling.
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kConv32MinPix = 65536;  // layers with at least this many pixels
                                      // use the 64-pixel wave tiles

__device__ __forceinline__ f32x16 mfma32(const bf16x8& a, const bf16x8& b, const f32x16& c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

template <int CT>
__global__ __launch_bounds__(256) void conv_fwd32_kernel(ConvArgs a) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int px0 = blockIdx.x * 256 + 64 * wv;
  const int co0 = blockIdx.y * (32 * CT);
  const int r = lane & 31, g = lane >> 5;
  int pidx[2], py[2], pxx[2];
  bool pv[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int p = px0 + 32 * s + r;
    pv[s] = p < a.npix;
    const int q = pv[s] ? p : 0;
    pidx[s] = q;
    pxx[s] = q % a.wd;
    py[s] = (q / a.wd) % a.h;
  }
  f32x16 acc[2][CT];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int b = 0; b < CT; ++b)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[s][b][v] = 0.f;
  for (int t = 0; t < 9; ++t) {
    const int dy = t / 3 - 1, dx = t % 3 - 1;
    const bf16* xa[2];
    bool ok[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int yy = py[s] + dy, xx = pxx[s] + dx;
      ok[s] = pv[s] && yy >= 0 && yy < a.h && xx >= 0 && xx < a.wd;
      xa[s] = a.x + (long long)(ok[s] ? pidx[s] + dy * a.wd + dx : 0) * a.ldx + 8 * g;
    }
    const bf16* wb[CT];
#pragma unroll
    for (int b = 0; b < CT; ++b)
      wb[b] = a.w + ((long long)(co0 + 32 * b + r) * 9 + t) * a.cin + 8 * g;
    for (int c0 = 0; c0 < a.cin; c0 += 16) {
      bf16x8 A[2], B[CT];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        A[s] = *reinterpret_cast<const bf16x8*>(xa[s] + c0);
        if (!ok[s]) A[s] = bf16x8{};
      }
#pragma unroll
      for (int b = 0; b < CT; ++b) B[b] = *reinterpret_cast<const bf16x8*>(wb[b] + c0);
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int b = 0; b < CT; ++b) acc[s][b] = mfma32(A[s], B[b], acc[s][b]);
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int b = 0; b < CT; ++b) {
      const int co = co0 + 32 * b + r;
      const float bias = a.bias ? a.bias[co] : 0.f;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int p = px0 + 32 * s + 8 * (v / 4) + 4 * g + (v % 4);
        if (p >= a.npix) continue;
        float val = acc[s][b][v] + bias;
        if (a.relu) val = fmaxf(val, 0.f);
        if (a.out_f32)
          static_cast<float*>(a.y)[(long long)p * a.ldy + co] = val;
        else
          static_cast<bf16*>(a.y)[(long long)p * a.ldy + co] = (bf16)val;
      }
    }
}

int launch_conv(const ConvArgs& a, hipStream_t st) {
  if (a.cin <= 0 || a.cout <= 0 || a.cin % 32 || a.cout % 32)
    return fail(UNET_EINVAL, "conv: cin and cout must be positive multiples of 32");
  if (a.ldx % 8 || a.ldy % 8 || a.ldx < a.cin || a.ldy < a.cout)
    return fail(UNET_EINVAL, "conv: ld must be a multiple of 8 and cover the channels");
  if (a.npix <= 0 || a.h <= 0 || a.wd <= 0 || a.npix % (a.h * a.wd))
    return fail(UNET_EINVAL, "conv: bad image size");
  if (!a.x || !a.w || !a.y) return fail(UNET_EINVAL, "conv: null pointer");
  if (a.npix >= kConv32MinPix) {
    // large layers: 64-pixel wave tiles on the 32x32x16 MFMA
    if (a.cout % 64 == 0) {
      dim3 grid((a.npix + 255) / 256, a.cout / 64);
      hipLaunchKernelGGL(conv_fwd32_kernel<2>, grid, dim3(256), 0, st, a);
    } else {
      dim3 grid((a.npix + 255) / 256, a.cout / 32);
      hipLaunchKernelGGL(conv_fwd32_kernel<1>, grid, dim3(256), 0, st, a);
    }
  } else if (a.cout % 64 == 0) {
    dim3 grid((a.npix + 63) / 64, a.cout / 64);
    hipLaunchKernelGGL(conv_fwd_kernel<2>, grid, dim3(256), 0, st, a);
  } else {
    dim3 grid((a.npix + 127) / 128, a.cout / 32);
    hipLaunchKernelGGL(conv_fwd_kernel<1>, grid, dim3(256), 0, st, a);
  }
  UCHECK(hipGetLastError());
  return UNET_OK;
}

// wt[ci][t][co] = w[co][8 - t][ci]
__global__ void flip_transpose_kernel(const bf16* w, bf16* wt, int cin, int cout) {
  const long long total = 9LL * cin * cout;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int co = int(e % cout);
    const long long rest = e / cout;
    const int t = int(rest % 9), ci = int(rest / 9);
    wt[e] = w[((long long)co * 9 + (8 - t)) * cin + ci];
  }
}

// ---------------------------------------------------------------------------
// Convolution, weight and bias gradients
// ---------------------------------------------------------------------------
struct WgradArgs {
  const bf16* dy;
  int lddy;
  const bf16* x;
  int ldx;
  float* part;        // [splits][cout][9][cin]
  float* bpart;       // [splits][cout] or null
  int npix, h, wd, cin, cout, chunk;
};

constexpr int kPadPx = 40;   // LDS row length (32 pixels + 8) in bf16
constexpr int kWgrad2Blocks = 1024;   // blocks the channel-major path aims for

__global__ __launch_bounds__(256) void wgrad_kernel(WgradArgs a) {
  __shared__ bf16 sA[4][32][kPadPx];   // per wave: dy tile [co][pixel]
  __shared__ bf16 sB[4][32][kPadPx];   // per wave: x tile [ci][pixel]
  __shared__ float sR[4][32][33];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int bid = blockIdx.x;
  const int t = bid % 9;
  bid /= 9;
  const int nci = a.cin / 32;
  const int ci0 = (bid % nci) * 32, co0 = (bid / nci) * 32;
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  const int pbeg = blockIdx.y * a.chunk;
  const int pend = min(a.npix, pbeg + a.chunk);
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // chunk is a multiple of 128: every wave runs the same number of steps
  for (int k0 = pbeg + 32 * wv; k0 < pbeg + a.chunk; k0 += 128) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      const int q = lane + 64 * e;
      const int pl = q >> 2, cv = q & 3;
      const int p = k0 + pl;
      bf16x8 vd = bf16x8{}, vx = bf16x8{};
      if (p < pend) {
        vd = *reinterpret_cast<const bf16x8*>(a.dy + (long long)p * a.lddy + co0 + 8 * cv);
        const int xx = p % a.wd, yy = (p / a.wd) % a.h;
        const int sy = yy + dy, sx = xx + dx;
        if (sy >= 0 && sy < a.h && sx >= 0 && sx < a.wd)
          vx = *reinterpret_cast<const bf16x8*>(a.x + (long long)(p + dy * a.wd + dx) * a.ldx +
                                                ci0 + 8 * cv);
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        sA[wv][8 * cv + u][pl] = vd[u];
        sB[wv][8 * cv + u][pl] = vx[u];
      }
    }
    __syncthreads();
    bf16x8 A[2], B[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      A[b] = *reinterpret_cast<const bf16x8*>(&sA[wv][16 * b + r][8 * g]);
      B[b] = *reinterpret_cast<const bf16x8*>(&sB[wv][16 * b + r][8 * g]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(A[i], B[j], acc[i][j]);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) sR[wv][16 * i + 4 * g + v][16 * j + r] = acc[i][j][v];
  __syncthreads();
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int co = e >> 5, ci = e & 31;
    const float s = sR[0][co][ci] + sR[1][co][ci] + sR[2][co][ci] + sR[3][co][ci];
    a.part[(((long long)blockIdx.y * a.cout + co0 + co) * 9 + t) * a.cin + ci0 + ci] = s;
  }
  // bias partials: the blocks of tap 0 and the first input-channel tile
  if (a.bpart && t == 0 && ci0 == 0 && threadIdx.x < 32) {
    const int co = co0 + threadIdx.x;
    float s = 0.f;
    for (int p = pbeg; p < pend; ++p) s += (float)a.dy[(long long)p * a.lddy + co];
    a.bpart[(long long)blockIdx.y * a.cout + co] = s;
  }
}

// ---- weight gradient on channel-major copies (width a multiple of 8) ------
// The pixel sum is the MFMA reduction dimension, so both operands are first
// copied channel-major ([c][p], pixels contiguous): then every A and B
// operand is 8 consecutive pixels of one channel, one 16-byte load (two and
// a lane-local shift for the taps with dx = +-1), with no LDS transposes.

// dst[c * rowlen + p] = src[p][c] for c < ch, p < npix (bf16; rowlen a
// multiple of 8); 64 pixels x 32 channels per block through LDS.
__global__ __launch_bounds__(256) void to_channel_major_kernel(const bf16* __restrict__ src,
                                                                int lds, bf16* __restrict__ dst,
                                                                int npix, int rowlen) {
  __shared__ bf16 t[64][32 + 2];
  const int p0 = blockIdx.x * 64, c0 = blockIdx.y * 32;
  // load: 64 pixels x 4 vectors of 8 channels = 256 vectors, one per thread
  {
    const int pl = threadIdx.x >> 2, cv = threadIdx.x & 3;
    const int p = p0 + pl;
    bf16x8 v = bf16x8{};
    if (p < npix) v = *reinterpret_cast<const bf16x8*>(src + (long long)p * lds + c0 + 8 * cv);
#pragma unroll
    for (int u = 0; u < 8; ++u) t[pl][8 * cv + u] = v[u];
  }
  __syncthreads();
  // store: 32 channels x 8 vectors of 8 pixels = 256 vectors
  {
    const int c = threadIdx.x >> 3, pv = threadIdx.x & 7;
    const int p = p0 + 8 * pv;
    if (p < npix) {
      bf16x8 o;
#pragma unroll
      for (int u = 0; u < 8; ++u) o[u] = t[8 * pv + u][c];
      if (p + 8 <= npix) {
        *reinterpret_cast<bf16x8*>(dst + (long long)(c0 + c) * rowlen + p) = o;
      } else {
        for (int u = 0; u < 8 && p + u < npix; ++u) dst[(long long)(c0 + c) * rowlen + p + u] = o[u];
      }
    }
  }
}

struct Wgrad2Args {
  const bf16* dyT;    // [cout][npix]
  const bf16* xT;     // [cin][npix]
  float* part;        // [splits][cout][9][cin]
  float* bpart;       // [splits][cout] (bias partial sums) or null
  int npix, npad, h, wd, cin, cout, chunk;
};

// 8 consecutive pixels p .. p + 7 (one row: p % 8 == 0, width % 8 == 0) of
// channel row `row` (npad elements, a multiple of 8), shifted by the tap
// (dy, dx) with zero padding.
__device__ __forceinline__ bf16x8 tap_row8(const bf16* __restrict__ row, int p, int npix,
                                           int npad, int h, int wd, int dy, int dx) {
  bf16x8 z = bf16x8{};
  if (p >= npix) return z;
  const int y = (p / wd) % h;
  if (y + dy < 0 || y + dy >= h) return z;
  const int q = p + dy * wd;   // aligned source of the unshifted columns
  const bf16x8 v0 = *reinterpret_cast<const bf16x8*>(row + q);
  if (dx == 0) return v0;
  bf16x8 o;
  if (dx < 0) {
    // pixel p + u takes column u - 1: the element before the vector, zero
    // at the start of a row
    const bool first = p % wd == 0;
    const bf16x8 vp = *reinterpret_cast<const bf16x8*>(row + (q >= 8 ? q - 8 : 0));
    o[0] = first ? bf16(0.f) : vp[7];
#pragma unroll
    for (int u = 1; u < 8; ++u) o[u] = v0[u - 1];
  } else {
    const bool last = (p + 8) % wd == 0;
    const bf16x8 vn = *reinterpret_cast<const bf16x8*>(row + (q + 8 < npad ? q + 8 : q));
#pragma unroll
    for (int u = 0; u < 7; ++u) o[u] = v0[u + 1];
    o[7] = last ? bf16(0.f) : vn[0];
  }
  return o;
}

// One block: a 32 x 32 tile of one tap over one pixel chunk (split); its
// partial sum goes to `part`.  The blocks of the centre tap and the first
// input-channel tile also sum dy over their chunk for the bias gradient
// (`bpart`), so the bias needs no launch of its own.
__global__ __launch_bounds__(256) void wgrad2_kernel(Wgrad2Args a) {
  __shared__ float sR[4][32][33];
  __shared__ float sB[256];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int bid = blockIdx.x;
  const int t = bid % 9;
  bid /= 9;
  const int nci = a.cin / 32;
  const int ci0 = (bid % nci) * 32, co0 = (bid / nci) * 32;
  const int dy = t / 3 - 1, dx = t % 3 - 1;
  const int pbeg = blockIdx.y * a.chunk;
  const int r = lane & 15, g = lane >> 4;
  const bf16* arow[2];
  const bf16* brow[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    arow[b] = a.dyT + (long long)(co0 + 16 * b + r) * a.npad;
    brow[b] = a.xT + (long long)(ci0 + 16 * b + r) * a.npad;
  }
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = pbeg + 32 * wv; k0 < pbeg + a.chunk; k0 += 128) {
    const int p = k0 + 8 * g;
    bf16x8 A[2], B[2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      A[b] = p < a.npix ? *reinterpret_cast<const bf16x8*>(arow[b] + p) : bf16x8{};
      B[b] = tap_row8(brow[b], p, a.npix, a.npad, a.h, a.wd, dy, dx);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = mfma16(A[i], B[j], acc[i][j]);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) sR[wv][16 * i + 4 * g + v][16 * j + r] = acc[i][j][v];
  __syncthreads();
  const long long wcount = 9LL * a.cin * a.cout;
  for (int e = threadIdx.x; e < 1024; e += 256) {
    const int co = e >> 5, ci = e & 31;
    const float s = sR[0][co][ci] + sR[1][co][ci] + sR[2][co][ci] + sR[3][co][ci];
    a.part[blockIdx.y * wcount + ((long long)(co0 + co) * 9 + t) * a.cin + ci0 + ci] = s;
  }
  const bool bias_tile = a.bpart != nullptr && t == 4 && ci0 == 0;
  if (bias_tile) {
    // eight threads per output channel, 8 pixels per load, fixed order
    const int co = threadIdx.x >> 3, l8 = threadIdx.x & 7;
    const bf16* row = a.dyT + (long long)(co0 + co) * a.npad;
    const int pend = min(a.npix, pbeg + a.chunk);
    float s = 0.f;
    for (int p = pbeg + 8 * l8; p < pend; p += 64) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(row + p);
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (p + u < pend) s += (float)v[u];
    }
    sB[threadIdx.x] = s;
    __syncthreads();
    if (l8 == 0) {
      float b = 0.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) b += sB[threadIdx.x + u];
      a.bpart[(long long)blockIdx.y * a.cout + co0 + co] = b;
    }
  }
}

// out[i] = sum_s part[s][i] (fixed order)
__global__ void sum_splits_kernel(const float* part, long long count, int splits, float* out) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < splits; ++k) s += part[(long long)k * count + i];
    out[i] = s;
  }
}

// Both sums of the weight gradient in one launch: out[i] = sum_s part[s][i]
// for i < count and bout[j] = sum_s bpart[s][j] for j < bcount (bpart may be
// null), each in split order.
__global__ void sum_splits2_kernel(const float* part, long long count, const float* bpart,
                                   int bcount, int splits, float* out, float* bout) {
  const long long total = count + (bpart ? bcount : 0);
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total;
       i += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    if (i < count) {
      for (int k = 0; k < splits; ++k) s += part[(long long)k * count + i];
      out[i] = s;
    } else {
      const long long j = i - count;
      for (int k = 0; k < splits; ++k) s += bpart[(long long)k * bcount + j];
      bout[j] = s;
    }
  }
}

void wgrad_plan(int npix, int cin, int cout, int* splits, int* chunk, int target = 2048) {
  const int base = (cout / 32) * (cin / 32) * 9;
  const int want = std::max(1, (target + base - 1) / base);
  int c = (npix + want - 1) / want;
  c = std::max(128, (c + 127) / 128 * 128);
  *chunk = c;
  *splits = (npix + c - 1) / c;
}

// ---------------------------------------------------------------------------
// Elementwise layers (8 channels per thread)
// ---------------------------------------------------------------------------
__global__ void relu_bwd_kernel(bf16* d, int ldd, const bf16* y, int ldy, long long npix, int cv) {
  const long long total = npix * cv;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long p = e / cv;
    const int c = int(e % cv) * 8;
    bf16x8 dv = *reinterpret_cast<const bf16x8*>(d + p * ldd + c);
    const bf16x8 yv = *reinterpret_cast<const bf16x8*>(y + p * ldy + c);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (!((float)yv[u] > 0.f)) dv[u] = (bf16)0.f;
    *reinterpret_cast<bf16x8*>(d + p * ldd + c) = dv;
  }
}

// (h, wd): input size of the pooling
__global__ void pool2_fwd_kernel(const bf16* x, int ldx, bf16* y, int ldy, int n, int h, int wd,
                                 int cv) {
  const int ho = h / 2, wo = wd / 2;
  const long long total = (long long)n * ho * wo * cv;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = int(e % cv) * 8;
    const long long po = e / cv;
    const int X = int(po % wo), Y = int((po / wo) % ho);
    const long long nn = po / ((long long)wo * ho);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const long long pi = (nn * h + 2 * Y + i) * wd + 2 * X + j;
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(x + pi * ldx + c);
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += (float)v[u];
      }
    bf16x8 o;
#pragma unroll
    for (int u = 0; u < 8; ++u) o[u] = (bf16)(0.25f * s[u]);
    *reinterpret_cast<bf16x8*>(y + po * ldy + c) = o;
  }
}

__global__ void pool2_bwd_kernel(const bf16* dy, int lddy, const bf16* add, int ldadd, bf16* dx,
                                 int lddx, int n, int h, int wd, int cv) {
  const int ho = h / 2, wo = wd / 2;
  const long long total = (long long)n * h * wd * cv;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = int(e % cv) * 8;
    const long long p = e / cv;
    const int x = int(p % wd), y = int((p / wd) % h);
    const long long nn = p / ((long long)wd * h);
    const long long po = (nn * ho + y / 2) * wo + x / 2;
    const bf16x8 g = *reinterpret_cast<const bf16x8*>(dy + po * lddy + c);
    bf16x8 a = bf16x8{};
    if (add) a = *reinterpret_cast<const bf16x8*>(add + p * ldadd + c);
    bf16x8 o;
#pragma unroll
    for (int u = 0; u < 8; ++u) o[u] = (bf16)((float)a[u] + 0.25f * (float)g[u]);
    *reinterpret_cast<bf16x8*>(dx + p * lddx + c) = o;
  }
}

// (h, wd): coarse size
__global__ void up2_fwd_kernel(const bf16* x, int ldx, bf16* y, int ldy, int n, int h, int wd,
                               int cv) {
  const int hf = 2 * h, wf = 2 * wd;
  const long long total = (long long)n * hf * wf * cv;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = int(e % cv) * 8;
    const long long p = e / cv;
    const int xf = int(p % wf), yf = int((p / wf) % hf);
    const long long nn = p / ((long long)wf * hf);
    const long long pc = (nn * h + yf / 2) * wd + xf / 2;
    *reinterpret_cast<bf16x8*>(y + p * ldy + c) =
        *reinterpret_cast<const bf16x8*>(x + pc * ldx + c);
  }
}

__global__ void up2_bwd_kernel(const bf16* dy, int lddy, bf16* dx, int lddx, int n, int h, int wd,
                               int cv) {
  const int wf = 2 * wd;
  const long long total = (long long)n * h * wd * cv;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = int(e % cv) * 8;
    const long long pc = e / cv;
    const int X = int(pc % wd), Y = int((pc / wd) % h);
    const long long nn = pc / ((long long)wd * h);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const long long pf = (nn * 2 * h + 2 * Y + i) * wf + 2 * X + j;
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(dy + pf * lddy + c);
#pragma unroll
        for (int u = 0; u < 8; ++u) s[u] += (float)v[u];
      }
    bf16x8 o;
#pragma unroll
    for (int u = 0; u < 8; ++u) o[u] = (bf16)s[u];
    *reinterpret_cast<bf16x8*>(dx + pc * lddx + c) = o;
  }
}

int grid_for(long long total) {
  long long b = (total + 255) / 256;
  return (int)std::min<long long>(std::max<long long>(b, 1), 65536);
}

// ---------------------------------------------------------------------------
// Loss
// ---------------------------------------------------------------------------
constexpr int kLossBlocks = 512;

// per-block FP64 partials: work[2 b] = sum of squares, work[2 b + 1] = fluid count
__global__ __launch_bounds__(256) void loss_partial_kernel(const float* out, int ldo,
                                                           const float* t, const uint8_t* fluid,
                                                           long long npix, double* work) {
  __shared__ double s_sq[256], s_n[256];
  double sq = 0.0, cnt = 0.0;
  for (long long p = blockIdx.x * 256LL + threadIdx.x; p < npix; p += 256LL * gridDim.x) {
    if (!fluid[p]) continue;
    cnt += 1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double d = (double)out[p * ldo + c] - (double)t[p * 3 + c];
      sq += d * d;
    }
  }
  s_sq[threadIdx.x] = sq;
  s_n[threadIdx.x] = cnt;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_sq[threadIdx.x] += s_sq[threadIdx.x + w];
      s_n[threadIdx.x] += s_n[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    work[2 * blockIdx.x] = s_sq[0];
    work[2 * blockIdx.x + 1] = s_n[0];
  }
}

// fixed-order tree over the per-block partials (one block of 256 threads)
__global__ __launch_bounds__(256) void loss_final_kernel(double* work, int blocks) {
  __shared__ double ssq[256], sn[256];
  double sq = 0.0, n = 0.0;
  for (int b = threadIdx.x; b < blocks; b += 256) {
    sq += work[2 * b];
    n += work[2 * b + 1];
  }
  ssq[threadIdx.x] = sq;
  sn[threadIdx.x] = n;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      ssq[threadIdx.x] += ssq[threadIdx.x + w];
      sn[threadIdx.x] += sn[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    work[2 * blocks] = sn[0] > 0 ? ssq[0] / (3.0 * sn[0]) : 0.0;
    work[2 * blocks + 1] = sn[0];
  }
}

__global__ void loss_grad_kernel(const float* out, int ldo, const float* t, const uint8_t* fluid,
                                 long long npix, bf16* dout, const double* fin) {
  const double n = fin[1];
  const float scale = n > 0 ? float(2.0 / (3.0 * n)) : 0.f;
  const long long total = npix * ldo;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const long long p = e / ldo;
    const int c = int(e % ldo);
    float g = 0.f;
    if (c < 3 && fluid[p]) g = scale * (out[p * ldo + c] - t[p * 3 + c]);
    dout[e] = (bf16)g;
  }
}

// ---------------------------------------------------------------------------
// Adam
// ---------------------------------------------------------------------------
__global__ void adam_kernel(float* p, float* m, float* v, const float* g, bf16* pb, long long n,
                            float lr, float b1, float b2, float eps, float c1, float c2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    p[i] = pi;
    if (pb) pb[i] = (bf16)pi;
  }
}

__global__ void to_bf16_kernel(const float* p, bf16* pb, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    pb[i] = (bf16)p[i];
}

// ---------------------------------------------------------------------------
// Input and output maps
// ---------------------------------------------------------------------------
// Coarse cell I covers the fine nodes i with floor(I fine / res) <= i <
// floor((I + 1) fine / res) (at least the node floor(I fine / res)); its
// solid fraction is the mean of the mask over those nodes.
__device__ __forceinline__ void cell_range(int I, int fine, int res, int& a, int& b) {
  a = int((long long)I * fine / res);
  b = int((long long)(I + 1) * fine / res);
  if (b <= a) b = a + 1;
}

// The case kind (case_params[cps c + 3] when cps == 4, else a cavity)
// places the driven-boundary marker: the lid row (top) of a cavity, the
// inlet column (left) of a channel.
__device__ __forceinline__ int case_kind(const float* cp, int cps, long long c) {
  return cps > 3 ? int(cp[cps * c + 3]) : UNET_KIND_CAVITY;
}

__global__ void make_input_kernel(const uint8_t* solid, int nx, int ny, const float* cp, int cps,
                                  int n, int res, bf16* x0) {
  const long long total = (long long)n * res * res;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = int(e % res), j = int((e / res) % res);
    const long long c = e / ((long long)res * res);
    int i0, i1, j0, j1;
    cell_range(i, nx, res, i0, i1);
    cell_range(j, ny, res, j0, j1);
    int cnt = 0;
    for (int b = j0; b < j1; ++b)
      for (int a = i0; a < i1; ++a) cnt += solid[(c * ny + b) * nx + a] != 0;
    float v[UNET_IN_CHANNELS];
#pragma unroll
    for (int k = 0; k < UNET_IN_CHANNELS; ++k) v[k] = 0.f;
    v[0] = float(cnt) / float((i1 - i0) * (j1 - j0));
    v[1] = cp[cps * c + 0] / 500.f;
    v[2] = cp[cps * c + 1];
    v[3] = cp[cps * c + 2] / 0.1f;
    v[4] = (i + 0.5f) / res;
    v[5] = (j + 0.5f) / res;
    v[6] = (case_kind(cp, cps, c) == UNET_KIND_CHANNEL ? i == 0 : j == res - 1) ? 1.f : 0.f;
    v[7] = 1.f;
#pragma unroll
    for (int q = 0; q < UNET_IN_CHANNELS / 8; ++q) {
      bf16x8 o;
#pragma unroll
      for (int u = 0; u < 8; ++u) o[u] = (bf16)v[8 * q + u];
      *reinterpret_cast<bf16x8*>(x0 + e * UNET_IN_CHANNELS + 8 * q) = o;
    }
  }
}

__device__ float bilinear(const float* out, int ldo, long long c, int res, int ch, float u,
                          float v) {
  // (u, v): position in coarse pixel-centre coordinates
  u = fminf(fmaxf(u, 0.f), float(res - 1));
  v = fminf(fmaxf(v, 0.f), float(res - 1));
  const int i0 = min(int(u), res - 2 < 0 ? 0 : res - 2), j0 = min(int(v), res - 2 < 0 ? 0 : res - 2);
  const int i1 = min(i0 + 1, res - 1), j1 = min(j0 + 1, res - 1);
  const float fu = u - i0, fv = v - j0;
  auto at = [&](int i, int j) { return out[((c * res + j) * res + i) * ldo + ch]; };
  return (1 - fv) * ((1 - fu) * at(i0, j0) + fu * at(i1, j0)) +
         fv * ((1 - fu) * at(i0, j1) + fu * at(i1, j1));
}

__global__ void fields_kernel(const float* out, int ldo, int n, int res, const float* cp,
                              int cps, const uint8_t* solid, int nx, int ny, float* rho,
                              float* ux, float* uy) {
  const long long total = (long long)n * nx * ny;
  const float scx = float(res) / float(nx), scy = float(res) / float(ny);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int i = int(e % nx), j = int((e / nx) % ny);
    const long long c = e / ((long long)nx * ny);
    if (solid[e]) {
      rho[e] = 1.f;
      ux[e] = 0.f;
      uy[e] = 0.f;
      continue;
    }
    const float U = cp[cps * c + 2];
    const float u = (i + 0.5f) * scx - 0.5f, v = (j + 0.5f) * scy - 0.5f;
    rho[e] = 1.f + 3.f * U * U * bilinear(out, ldo, c, res, 0, u, v);
    ux[e] = U * bilinear(out, ldo, c, res, 1, u, v);
    uy[e] = U * bilinear(out, ldo, c, res, 2, u, v);
  }
}

// One block per case (fixed-order FP64 sums).  (1) Remove the fluid mean of
// rho - 1.  (2) Remove the staggered momentum components: with bounce-back
// walls and no force, every step flips the sign of
// Ix = sum_fluid (-1)^i j_x and of Iy = sum_fluid (-1)^j j_y (collision
// conserves j at each node; streaming and bounce-back move each population
// with e_x != 0 to a column of the other parity, or reverse it in place), so
// a start with Ix or Iy != 0 never settles: the state keeps an undamped
// period-2 oscillation.  u_x -= (-1)^i Ix / sum rho (likewise u_y) makes
// both zero, as they are for the state at rest.  Closed lattices (cavities)
// only: a channel's inlet and outlet change its mass and do not keep these
// sums, so its prediction is left as it is.
__global__ __launch_bounds__(256) void mass_fix_kernel(float* rho, float* ux, float* uy,
                                                       const uint8_t* solid, int nx, int ny,
                                                       const float* cp, int cps) {
  __shared__ double s[4][256];
  if (case_kind(cp, cps, blockIdx.x) != UNET_KIND_CAVITY) return;
  const long long base = (long long)blockIdx.x * nx * ny;
  const long long cnt = (long long)nx * ny;
  auto block_sum = [&](int q) {
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) s[q][threadIdx.x] += s[q][threadIdx.x + w];
      __syncthreads();
    }
    return s[q][0];
  };
  double acc = 0.0, nf = 0.0;
  for (long long k = threadIdx.x; k < cnt; k += 256)
    if (!solid[base + k]) {
      acc += (double)rho[base + k] - 1.0;
      nf += 1.0;
    }
  s[0][threadIdx.x] = acc;
  s[1][threadIdx.x] = nf;
  const double sum_dr = block_sum(0), n_fluid = block_sum(1);
  const float mean = n_fluid > 0 ? float(sum_dr / n_fluid) : 0.f;
  double sx = 0.0, sy = 0.0, sr = 0.0;
  for (long long k = threadIdx.x; k < cnt; k += 256)
    if (!solid[base + k]) {
      const float r = rho[base + k] - mean;
      rho[base + k] = r;
      const int i = int(k % nx), j = int(k / nx);
      sx += (i & 1 ? -1.0 : 1.0) * (double)r * (double)ux[base + k];
      sy += (j & 1 ? -1.0 : 1.0) * (double)r * (double)uy[base + k];
      sr += (double)r;
    }
  __syncthreads();
  s[0][threadIdx.x] = sx;
  s[1][threadIdx.x] = sy;
  s[2][threadIdx.x] = sr;
  const double Ix = block_sum(0), Iy = block_sum(1), R = block_sum(2);
  const float mx = R > 0 ? float(Ix / R) : 0.f, my = R > 0 ? float(Iy / R) : 0.f;
  for (long long k = threadIdx.x; k < cnt; k += 256)
    if (!solid[base + k]) {
      const int i = int(k % nx), j = int(k / nx);
      ux[base + k] -= (i & 1) ? -mx : mx;
      uy[base + k] -= (j & 1) ? -my : my;
    }
}

}  // namespace

// ===========================================================================
// Input and output maps of either shape (cps: floats per case in case_params)
// ===========================================================================
static int launch_make_input(const uint8_t* solid, int nx, int ny, const float* cp, int cps, int n,
                      int res, void* x0, void* stream) {
  if (!solid || !cp || !x0 || n <= 0 || res <= 0 || nx <= 0 || ny <= 0)
    return fail(UNET_EINVAL, "make_input: bad arguments");
  hipLaunchKernelGGL(make_input_kernel, dim3(grid_for((long long)n * res * res)), dim3(256), 0,
                     as_stream(stream), solid, nx, ny, cp, cps, n, res, static_cast<bf16*>(x0));
  UCHECK(hipGetLastError());
  return UNET_OK;
}

static int launch_fields(const float* out, int ldo, int n, int res, const float* cp, int cps,
                  const uint8_t* solid, int nx, int ny, float* rho, float* ux, float* uy,
                  void* stream) {
  if (!out || !cp || !solid || !rho || !ux || !uy || n <= 0 || res < 2 || nx <= 0 || ny <= 0 ||
      ldo < 3)
    return fail(UNET_EINVAL, "fields_from_output: bad arguments");
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(fields_kernel, dim3(grid_for((long long)n * nx * ny)), dim3(256), 0, st,
                     out, ldo, n, res, cp, cps, solid, nx, ny, rho, ux, uy);
  hipLaunchKernelGGL(mass_fix_kernel, dim3(n), dim3(256), 0, st, rho, ux, uy, solid, nx, ny, cp,
                     cps);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

// ===========================================================================
// C ABI: layers
// ===========================================================================
extern "C" {

const char* unet_last_error(void) { return g_err.c_str(); }

int unet_conv3x3_fwd(const void* x, int32_t ldx, const void* w, const float* bias, void* y,
                     int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout,
                     int32_t relu, int32_t out_f32, void* stream) {
  if (n <= 0 || h <= 0 || wd <= 0) return fail(UNET_EINVAL, "conv: bad size");
  ConvArgs a{static_cast<const bf16*>(x), ldx, static_cast<const bf16*>(w), bias, y, ldy,
             n * h * wd, h, wd, cin, cout, relu, out_f32};
  return launch_conv(a, as_stream(stream));
}

int unet_conv3x3_bwd_data(const void* dy, int32_t lddy, const void* w, void* dx, int32_t lddx,
                          int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, void* work,
                          void* stream) {
  if (!work || !w) return fail(UNET_EINVAL, "bwd_data: null pointer");
  if (n <= 0 || h <= 0 || wd <= 0) return fail(UNET_EINVAL, "bwd_data: bad size");
  hipStream_t st = as_stream(stream);
  const long long cnt = 9LL * cin * cout;
  hipLaunchKernelGGL(flip_transpose_kernel, dim3(grid_for(cnt)), dim3(256), 0, st,
                     static_cast<const bf16*>(w), static_cast<bf16*>(work), cin, cout);
  ConvArgs a{static_cast<const bf16*>(dy), lddy, static_cast<const bf16*>(work), nullptr, dx,
             lddx, n * h * wd, h, wd, cout, cin, 0, 0};
  return launch_conv(a, st);
}

int64_t unet_wgrad_work_floats(int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout) {
  if (n <= 0 || h <= 0 || wd <= 0 || cin <= 0 || cout <= 0) return 0;
  int splits, chunk;
  wgrad_plan(n * h * wd, cin, cout, &splits, &chunk);
  int64_t words = (int64_t)splits * (9LL * cin * cout + cout);
  if (wd % 8 == 0) {
    // channel-major path: fewer splits, plus the two bf16 copies
    wgrad_plan(n * h * wd, cin, cout, &splits, &chunk, kWgrad2Blocks);
    const int64_t npad = ((int64_t)n * h * wd + 7) / 8 * 8 + 8;
    words = std::max<int64_t>(words, (int64_t)splits * (9LL * cin * cout + cout) +
                                         (npad * (cin + cout) + 1) / 2 + 64);
  }
  return words;
}

int unet_conv3x3_bwd_weight(const void* dy, int32_t lddy, const void* x, int32_t ldx, float* dw,
                            float* dbias, int32_t n, int32_t h, int32_t wd, int32_t cin,
                            int32_t cout, float* work, void* stream) {
  if (!dy || !x || !dw || !work) return fail(UNET_EINVAL, "bwd_weight: null pointer");
  if (n <= 0 || h <= 0 || wd <= 0) return fail(UNET_EINVAL, "bwd_weight: bad size");
  if (cin % 32 || cout % 32 || cin <= 0 || cout <= 0)
    return fail(UNET_EINVAL, "bwd_weight: cin and cout must be positive multiples of 32");
  if (lddy % 8 || ldx % 8 || lddy < cout || ldx < cin)
    return fail(UNET_EINVAL, "bwd_weight: bad ld");
  hipStream_t st = as_stream(stream);
  const int npix = n * h * wd;
  int splits, chunk;
  const long long wcount = 9LL * cin * cout;
  if (wd % 8 == 0) {
    wgrad_plan(npix, cin, cout, &splits, &chunk, kWgrad2Blocks);
    const int npad = (npix + 7) / 8 * 8 + 8;
    float* part = work;
    float* bpart = work + (long long)splits * wcount;
    // bf16 copies after the partial sums (256-byte aligned)
    const long long used = ((long long)splits * (wcount + cout) + 63) / 64 * 64;
    bf16* dyT = reinterpret_cast<bf16*>(work + used);
    bf16* xT = dyT + (long long)cout * npad;
    const int tiles = (cout / 32) * (cin / 32) * 9;
    hipLaunchKernelGGL(to_channel_major_kernel, dim3((npix + 63) / 64, cout / 32), dim3(256), 0,
                       st, static_cast<const bf16*>(dy), lddy, dyT, npix, npad);
    hipLaunchKernelGGL(to_channel_major_kernel, dim3((npix + 63) / 64, cin / 32), dim3(256), 0,
                       st, static_cast<const bf16*>(x), ldx, xT, npix, npad);
    UCHECK(hipGetLastError());
    Wgrad2Args a2{dyT, xT, part, dbias ? bpart : nullptr, npix, npad, h, wd, cin, cout, chunk};
    hipLaunchKernelGGL(wgrad2_kernel, dim3(tiles, splits), dim3(256), 0, st, a2);
    UCHECK(hipGetLastError());
    hipLaunchKernelGGL(sum_splits2_kernel, dim3(grid_for(wcount + cout)), dim3(256), 0, st, part,
                       wcount, dbias ? bpart : nullptr, cout, splits, dw, dbias);
    UCHECK(hipGetLastError());
    return UNET_OK;
  }
  wgrad_plan(npix, cin, cout, &splits, &chunk);
  WgradArgs a{static_cast<const bf16*>(dy), lddy, static_cast<const bf16*>(x), ldx, work,
              work + (long long)splits * wcount, npix, h, wd, cin, cout, chunk};
  dim3 grid((cout / 32) * (cin / 32) * 9, splits);
  hipLaunchKernelGGL(wgrad_kernel, grid, dim3(256), 0, st, a);
  UCHECK(hipGetLastError());
  hipLaunchKernelGGL(sum_splits_kernel, dim3(grid_for(wcount)), dim3(256), 0, st, work, wcount,
                     splits, dw);
  if (dbias)
    hipLaunchKernelGGL(sum_splits_kernel, dim3(grid_for(cout)), dim3(256), 0, st,
                       work + (long long)splits * wcount, (long long)cout, splits, dbias);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int unet_relu_bwd(void* d, int32_t ldd, const void* y, int32_t ldy, int64_t npix, int32_t ch,
                  void* stream) {
  if (!d || !y || ch % 8 || ldd % 8 || ldy % 8 || npix < 0)
    return fail(UNET_EINVAL, "relu_bwd: bad arguments");
  hipLaunchKernelGGL(relu_bwd_kernel, dim3(grid_for(npix * (ch / 8))), dim3(256), 0,
                     as_stream(stream), static_cast<bf16*>(d), ldd, static_cast<const bf16*>(y),
                     ldy, (long long)npix, ch / 8);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int unet_pool2_fwd(const void* x, int32_t ldx, void* y, int32_t ldy, int32_t n, int32_t h,
                   int32_t wd, int32_t ch, void* stream) {
  if (!x || !y || h % 2 || wd % 2 || ch % 8 || ldx % 8 || ldy % 8 || n <= 0)
    return fail(UNET_EINVAL, "pool2_fwd: bad arguments");
  const long long total = (long long)n * (h / 2) * (wd / 2) * (ch / 8);
  hipLaunchKernelGGL(pool2_fwd_kernel, dim3(grid_for(total)), dim3(256), 0, as_stream(stream),
                     static_cast<const bf16*>(x), ldx, static_cast<bf16*>(y), ldy, n, h, wd,
                     ch / 8);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int unet_pool2_bwd(const void* dy, int32_t lddy, const void* add, int32_t ldadd, void* dx,
                   int32_t lddx, int32_t n, int32_t h, int32_t wd, int32_t ch, void* stream) {
  if (!dy || !dx || h % 2 || wd % 2 || ch % 8 || lddy % 8 || lddx % 8 || n <= 0 ||
      (add && ldadd % 8))
    return fail(UNET_EINVAL, "pool2_bwd: bad arguments");
  const long long total = (long long)n * h * wd * (ch / 8);
  hipLaunchKernelGGL(pool2_bwd_kernel, dim3(grid_for(total)), dim3(256), 0, as_stream(stream),
                     static_cast<const bf16*>(dy), lddy, static_cast<const bf16*>(add), ldadd,
                     static_cast<bf16*>(dx), lddx, n, h, wd, ch / 8);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int unet_up2_fwd(const void* x, int32_t ldx, void* y, int32_t ldy, int32_t n, int32_t h,
                 int32_t wd, int32_t ch, void* stream) {
  if (!x || !y || ch % 8 || ldx % 8 || ldy % 8 || n <= 0 || h <= 0 || wd <= 0)
    return fail(UNET_EINVAL, "up2_fwd: bad arguments");
  const long long total = (long long)n * 4 * h * wd * (ch / 8);
  hipLaunchKernelGGL(up2_fwd_kernel, dim3(grid_for(total)), dim3(256), 0, as_stream(stream),
                     static_cast<const bf16*>(x), ldx, static_cast<bf16*>(y), ldy, n, h, wd,
                     ch / 8);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int unet_up2_bwd(const void* dy, int32_t lddy, void* dx, int32_t lddx, int32_t n, int32_t h,
                 int32_t wd, int32_t ch, void* stream) {
  if (!dy || !dx || ch % 8 || lddy % 8 || lddx % 8 || n <= 0 || h <= 0 || wd <= 0)
    return fail(UNET_EINVAL, "up2_bwd: bad arguments");
  const long long total = (long long)n * h * wd * (ch / 8);
  hipLaunchKernelGGL(up2_bwd_kernel, dim3(grid_for(total)), dim3(256), 0, as_stream(stream),
                     static_cast<const bf16*>(dy), lddy, static_cast<bf16*>(dx), lddx, n, h, wd,
                     ch / 8);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int64_t unet_loss_work_doubles(int64_t npix) {
  (void)npix;
  return 2 * kLossBlocks + 2;
}

int unet_mse_loss(const float* out, int32_t ldo, const float* target, const uint8_t* fluid,
                  int64_t npix, void* dout, double* loss, double* work, void* stream) {
  if (!out || !target || !fluid || !dout || !work || ldo < 3 || ldo % 8 || npix <= 0)
    return fail(UNET_EINVAL, "mse_loss: bad arguments");
  hipStream_t st = as_stream(stream);
  hipLaunchKernelGGL(loss_partial_kernel, dim3(kLossBlocks), dim3(256), 0, st, out, ldo, target,
                     fluid, (long long)npix, work);
  hipLaunchKernelGGL(loss_final_kernel, dim3(1), dim3(256), 0, st, work, kLossBlocks);
  hipLaunchKernelGGL(loss_grad_kernel, dim3(grid_for(npix * ldo)), dim3(256), 0, st, out, ldo,
                     target, fluid, (long long)npix, static_cast<bf16*>(dout),
                     (const double*)(work + 2 * kLossBlocks));
  UCHECK(hipGetLastError());
  if (loss) {
    UCHECK(hipMemcpyAsync(loss, work + 2 * kLossBlocks, sizeof(double), hipMemcpyDeviceToHost,
                          st));
    UCHECK(hipStreamSynchronize(st));
  }
  return UNET_OK;
}

int unet_adam(float* p, float* m, float* v, const float* g, void* pb, int64_t count, double lr,
              double beta1, double beta2, double eps, int64_t t, void* stream) {
  if (!p || !m || !v || !g || count < 0 || t < 1) return fail(UNET_EINVAL, "adam: bad arguments");
  const double c1 = 1.0 / (1.0 - std::pow(beta1, (double)t));
  const double c2 = 1.0 / (1.0 - std::pow(beta2, (double)t));
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(count)), dim3(256), 0, as_stream(stream), p, m,
                     v, g, static_cast<bf16*>(pb), (long long)count, (float)lr, (float)beta1,
                     (float)beta2, (float)eps, (float)c1, (float)c2);
  UCHECK(hipGetLastError());
  return UNET_OK;
}

int unet_make_input(const uint8_t* solid, int32_t fine, const float* case_params, int32_t n,
                    int32_t res, void* x0, void* stream) {
  return launch_make_input(solid, fine, fine, case_params, 3, n, res, x0, stream);
}

int unet_fields_from_output(const float* out, int32_t ldo, int32_t n, int32_t res,
                            const float* case_params, const uint8_t* solid, int32_t fine,
                            float* rho, float* ux, float* uy, void* stream) {
  return launch_fields(out, ldo, n, res, case_params, 3, solid, fine, fine, rho, ux, uy, stream);
}

int unet_make_input_rect(const uint8_t* solid, int32_t nx, int32_t ny, const float* case_params,
                         int32_t n, int32_t res, void* x0, void* stream) {
  return launch_make_input(solid, nx, ny, case_params, 4, n, res, x0, stream);
}

int unet_fields_from_output_rect(const float* out, int32_t ldo, int32_t n, int32_t res,
                                 const float* case_params, const uint8_t* solid, int32_t nx,
                                 int32_t ny, float* rho, float* ux, float* uy, void* stream) {
  return launch_fields(out, ldo, n, res, case_params, 4, solid, nx, ny, rho, ux, uy, stream);
}

}  // extern "C"

// ===========================================================================
// The network
// ===========================================================================
namespace {

// Activation buffers (bf16 NHWC) and their channel counts.
enum Buf {
  B_X0, B_E0A, B_CAT0, B_P1, B_E1A, B_CAT1, B_P2, B_E2A, B_CAT2, B_P3, B_B3A, B_B3,
  B_D2A, B_D2, B_D1A, B_D1, B_D0A, B_D0, B_COUNT
};

struct BufInfo {
  int level, ch;
};
constexpr BufInfo kBuf[B_COUNT] = {
    {0, UNET_IN_CHANNELS}, {0, 32}, {0, 96}, {1, 32}, {1, 64}, {1, 192}, {2, 64}, {2, 128},
    {2, 384}, {3, 128}, {3, 256}, {3, 256}, {2, 128}, {2, 128}, {1, 64}, {1, 64}, {0, 32},
    {0, 32}};

struct Conv {
  int in, in_off, cin, out, out_off, cout, level, relu;   // out = -1: network output (FP32)
  long long w_off, b_off;
};

// Layer table: input buffer/channel offset, output buffer/channel offset.
const Conv kConvs[] = {
    {B_X0, 0, 32, B_E0A, 0, 32, 0, 1, 0, 0},   {B_E0A, 0, 32, B_CAT0, 64, 32, 0, 1, 0, 0},
    {B_P1, 0, 32, B_E1A, 0, 64, 1, 1, 0, 0},   {B_E1A, 0, 64, B_CAT1, 128, 64, 1, 1, 0, 0},
    {B_P2, 0, 64, B_E2A, 0, 128, 2, 1, 0, 0},  {B_E2A, 0, 128, B_CAT2, 256, 128, 2, 1, 0, 0},
    {B_P3, 0, 128, B_B3A, 0, 256, 3, 1, 0, 0}, {B_B3A, 0, 256, B_B3, 0, 256, 3, 1, 0, 0},
    {B_CAT2, 0, 384, B_D2A, 0, 128, 2, 1, 0, 0}, {B_D2A, 0, 128, B_D2, 0, 128, 2, 1, 0, 0},
    {B_CAT1, 0, 192, B_D1A, 0, 64, 1, 1, 0, 0},  {B_D1A, 0, 64, B_D1, 0, 64, 1, 1, 0, 0},
    {B_CAT0, 0, 96, B_D0A, 0, 32, 0, 1, 0, 0},   {B_D0A, 0, 32, B_D0, 0, 32, 0, 1, 0, 0},
    {B_D0, 0, 32, -1, 0, UNET_OUT_CHANNELS, 0, 0, 0, 0}};
constexpr int kNumConvs = sizeof(kConvs) / sizeof(kConvs[0]);

}  // namespace

struct unet {
  int max_batch = 0, res = 0;
  hipStream_t stream = nullptr;
  std::vector<Conv> convs;
  long long nparams = 0;
  float* p = nullptr;    // FP32 master parameters
  bf16* pb = nullptr;    // bf16 copy (weights used by the kernels)
  float* grad = nullptr;
  float* m = nullptr;
  float* v = nullptr;
  long long t = 0;       // Adam steps taken
  bf16* act[B_COUNT] = {};
  bf16* gact[B_COUNT] = {};
  float* out = nullptr;  // FP32 network output (training)
  bf16* gout = nullptr;  // bf16 gradient of the output
  void* wt = nullptr;    // flipped weights scratch
  float* wwork = nullptr;
  double* lwork = nullptr;
};

namespace {

int side(const unet* net, int level) { return net->res >> level; }

long long npix(const unet* net, int level, int n) {
  const long long s = side(net, level);
  return (long long)n * s * s;
}

int forward_impl(unet* net, const bf16* x0, int n, float* out) {
  hipStream_t st = net->stream;
  net->act[B_X0] = const_cast<bf16*>(x0);
  auto conv = [&](int k) -> int {
    const Conv& c = net->convs[k];
    const int s = side(net, c.level);
    ConvArgs a{};
    a.x = net->act[c.in] + c.in_off;
    a.ldx = kBuf[c.in].ch;
    a.w = net->pb + c.w_off;
    a.bias = net->p + c.b_off;
    if (c.out < 0) {
      a.y = out;
      a.ldy = UNET_OUT_CHANNELS;
      a.out_f32 = 1;
    } else {
      a.y = net->act[c.out] + c.out_off;
      a.ldy = kBuf[c.out].ch;
      a.out_f32 = 0;
    }
    a.npix = n * s * s;
    a.h = s;
    a.wd = s;
    a.cin = c.cin;
    a.cout = c.cout;
    a.relu = c.relu;
    return launch_conv(a, st);
  };
  auto pool = [&](int src, int off, int dst, int level, int ch) -> int {
    const int s = side(net, level);
    return unet_pool2_fwd(net->act[src] + off, kBuf[src].ch, net->act[dst], kBuf[dst].ch, n, s, s,
                          ch, st);
  };
  auto up = [&](int src, int dst, int coarse_level, int ch) -> int {
    const int s = side(net, coarse_level);
    return unet_up2_fwd(net->act[src], kBuf[src].ch, net->act[dst], kBuf[dst].ch, n, s, s, ch,
                        st);
  };
  int rc;
  if ((rc = conv(0)) || (rc = conv(1)) || (rc = pool(B_CAT0, 64, B_P1, 0, 32)) ||
      (rc = conv(2)) || (rc = conv(3)) || (rc = pool(B_CAT1, 128, B_P2, 1, 64)) ||
      (rc = conv(4)) || (rc = conv(5)) || (rc = pool(B_CAT2, 256, B_P3, 2, 128)) ||
      (rc = conv(6)) || (rc = conv(7)) || (rc = up(B_B3, B_CAT2, 3, 256)) || (rc = conv(8)) ||
      (rc = conv(9)) || (rc = up(B_D2, B_CAT1, 2, 128)) || (rc = conv(10)) || (rc = conv(11)) ||
      (rc = up(B_D1, B_CAT0, 1, 64)) || (rc = conv(12)) || (rc = conv(13)) || (rc = conv(14)))
    return rc;
  return UNET_OK;
}

// Gradients of conv k given the gradient of its (pre-activation) output.
int conv_backward(unet* net, int k, int n, const bf16* dy, int lddy, bool need_dx) {
  const Conv& c = net->convs[k];
  const int s = side(net, c.level);
  hipStream_t st = net->stream;
  int rc = unet_conv3x3_bwd_weight(dy, lddy, net->act[c.in] + c.in_off, kBuf[c.in].ch,
                                   net->grad + c.w_off, net->grad + c.b_off, n, s, s, c.cin,
                                   c.cout, net->wwork, st);
  if (rc || !need_dx) return rc;
  return unet_conv3x3_bwd_data(dy, lddy, net->pb + c.w_off, net->gact[c.in] + c.in_off,
                               kBuf[c.in].ch, n, s, s, c.cin, c.cout, net->wt, st);
}

// In place: gradient of buffer b (channels [off, off + ch)) times relu'.
int relu_back(unet* net, int b, int off, int ch, int n) {
  return unet_relu_bwd(net->gact[b] + off, kBuf[b].ch, net->act[b] + off, kBuf[b].ch,
                       npix(net, kBuf[b].level, n), ch, net->stream);
}

int backward_impl(unet* net, int n) {
  hipStream_t st = net->stream;
  int rc;
  auto upb = [&](int fine_buf, int coarse_buf, int coarse_level, int ch) -> int {
    const int s = side(net, coarse_level);
    return unet_up2_bwd(net->gact[fine_buf], kBuf[fine_buf].ch, net->gact[coarse_buf],
                        kBuf[coarse_buf].ch, n, s, s, ch, st);
  };
  auto poolb = [&](int coarse_buf, int fine_buf, int off, int fine_level, int ch) -> int {
    const int s = side(net, fine_level);
    bf16* g = net->gact[fine_buf] + off;
    return unet_pool2_bwd(net->gact[coarse_buf], kBuf[coarse_buf].ch, g, kBuf[fine_buf].ch, g,
                          kBuf[fine_buf].ch, n, s, s, ch, st);
  };
  // output layer (linear)
  if ((rc = conv_backward(net, 14, n, net->gout, UNET_OUT_CHANNELS, true))) return rc;
  // level 0 decoder
  if ((rc = relu_back(net, B_D0, 0, 32, n)) || (rc = conv_backward(net, 13, n, net->gact[B_D0], 32, true)))
    return rc;
  if ((rc = relu_back(net, B_D0A, 0, 32, n)) ||
      (rc = conv_backward(net, 12, n, net->gact[B_D0A], 32, true)))
    return rc;
  if ((rc = upb(B_CAT0, B_D1, 1, 64))) return rc;
  // level 1 decoder
  if ((rc = relu_back(net, B_D1, 0, 64, n)) || (rc = conv_backward(net, 11, n, net->gact[B_D1], 64, true)))
    return rc;
  if ((rc = relu_back(net, B_D1A, 0, 64, n)) ||
      (rc = conv_backward(net, 10, n, net->gact[B_D1A], 64, true)))
    return rc;
  if ((rc = upb(B_CAT1, B_D2, 2, 128))) return rc;
  // level 2 decoder
  if ((rc = relu_back(net, B_D2, 0, 128, n)) ||
      (rc = conv_backward(net, 9, n, net->gact[B_D2], 128, true)))
    return rc;
  if ((rc = relu_back(net, B_D2A, 0, 128, n)) ||
      (rc = conv_backward(net, 8, n, net->gact[B_D2A], 128, true)))
    return rc;
  if ((rc = upb(B_CAT2, B_B3, 3, 256))) return rc;
  // bottom
  if ((rc = relu_back(net, B_B3, 0, 256, n)) ||
      (rc = conv_backward(net, 7, n, net->gact[B_B3], 256, true)))
    return rc;
  if ((rc = relu_back(net, B_B3A, 0, 256, n)) ||
      (rc = conv_backward(net, 6, n, net->gact[B_B3A], 256, true)))
    return rc;
  // level 2 encoder: skip gradient (cat2[256:]) plus the pooled path
  if ((rc = poolb(B_P3, B_CAT2, 256, 2, 128))) return rc;
  if ((rc = relu_back(net, B_CAT2, 256, 128, n)) ||
      (rc = conv_backward(net, 5, n, net->gact[B_CAT2] + 256, 384, true)))
    return rc;
  if ((rc = relu_back(net, B_E2A, 0, 128, n)) ||
      (rc = conv_backward(net, 4, n, net->gact[B_E2A], 128, true)))
    return rc;
  // level 1 encoder
  if ((rc = poolb(B_P2, B_CAT1, 128, 1, 64))) return rc;
  if ((rc = relu_back(net, B_CAT1, 128, 64, n)) ||
      (rc = conv_backward(net, 3, n, net->gact[B_CAT1] + 128, 192, true)))
    return rc;
  if ((rc = relu_back(net, B_E1A, 0, 64, n)) ||
      (rc = conv_backward(net, 2, n, net->gact[B_E1A], 64, true)))
    return rc;
  // level 0 encoder
  if ((rc = poolb(B_P1, B_CAT0, 64, 0, 32))) return rc;
  if ((rc = relu_back(net, B_CAT0, 64, 32, n)) ||
      (rc = conv_backward(net, 1, n, net->gact[B_CAT0] + 64, 96, true)))
    return rc;
  if ((rc = relu_back(net, B_E0A, 0, 32, n)) ||
      (rc = conv_backward(net, 0, n, net->gact[B_E0A], 32, false)))
    return rc;
  return UNET_OK;
}

uint64_t splitmix_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ULL;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

double splitmix_uniform(uint64_t& s) { return (splitmix_next(s) >> 11) * (1.0 / 9007199254740992.0); }

void free_net(unet* net) {
  void* ptrs[] = {net->p, net->pb, net->grad, net->m, net->v, net->out, net->gout, net->wt,
                  net->wwork, net->lwork};
  for (void* q : ptrs) (void)hipFree(q);
  for (int b = 1; b < B_COUNT; ++b) (void)hipFree(net->act[b]);
  for (int b = 0; b < B_COUNT; ++b) (void)hipFree(net->gact[b]);
  delete net;
}

}  // namespace

extern "C" {

int unet_create(int32_t max_batch, int32_t res, uint64_t seed, unet** out) {
  if (!out) return fail(UNET_EINVAL, "null output pointer");
  *out = nullptr;
  if (max_batch <= 0 || res < 8 || res % 8) return fail(UNET_EINVAL, "res must be a multiple of 8");
  unet* net = new (std::nothrow) unet();
  if (!net) return fail(UNET_ENOMEM, "host allocation failed");
  net->max_batch = max_batch;
  net->res = res;
  long long off = 0;
  size_t wt_max = 0;
  long long wwork_max = 0;
  for (int k = 0; k < kNumConvs; ++k) {
    Conv c = kConvs[k];
    c.w_off = off;
    off += 9LL * c.cin * c.cout;
    c.b_off = off;
    off += c.cout;
    net->convs.push_back(c);
    wt_max = std::max(wt_max, (size_t)9 * c.cin * c.cout);
    const int s = res >> c.level;
    for (int nb = 1; nb <= max_batch; ++nb)
      wwork_max = std::max<long long>(wwork_max, unet_wgrad_work_floats(nb, s, s, c.cin, c.cout));
  }
  net->nparams = off;
  auto alloc = [&](void** p, size_t bytes) {
    return hipMalloc(p, bytes) == hipSuccess;
  };
  bool ok = alloc((void**)&net->p, sizeof(float) * off) && alloc((void**)&net->pb, 2 * off) &&
            alloc((void**)&net->grad, sizeof(float) * off) &&
            alloc((void**)&net->m, sizeof(float) * off) &&
            alloc((void**)&net->v, sizeof(float) * off) &&
            alloc((void**)&net->out, sizeof(float) * (size_t)max_batch * res * res * UNET_OUT_CHANNELS) &&
            alloc((void**)&net->gout, 2ULL * max_batch * res * res * UNET_OUT_CHANNELS) &&
            alloc(&net->wt, 2 * wt_max) && alloc((void**)&net->wwork, sizeof(float) * wwork_max) &&
            alloc((void**)&net->lwork, sizeof(double) * unet_loss_work_doubles(0));
  for (int b = 0; ok && b < B_COUNT; ++b) {
    const long long s = res >> kBuf[b].level;
    const size_t bytes = 2ULL * max_batch * s * s * kBuf[b].ch;
    if (b != B_X0) ok = alloc((void**)&net->act[b], bytes);
    if (ok) ok = alloc((void**)&net->gact[b], bytes);
  }
  if (!ok) {
    free_net(net);
    return fail(UNET_ENOMEM, "device allocation failed");
  }
  // He-normal weights (Box-Muller on a SplitMix64 stream), zero biases
  std::vector<float> h(off, 0.f);
  uint64_t st = seed;
  for (const Conv& c : net->convs) {
    const double sd = std::sqrt((c.relu ? 2.0 : 1.0) / (9.0 * c.cin));
    for (long long i = 0; i < 9LL * c.cin * c.cout; ++i) {
      const double u1 = std::max(splitmix_uniform(st), 1e-300), u2 = splitmix_uniform(st);
      h[c.w_off + i] = float(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2));
    }
  }
  *out = net;
  int rc = unet_set_params(net, h.data());
  if (rc) {
    free_net(net);
    *out = nullptr;
    return rc;
  }
  return UNET_OK;
}

void unet_destroy(unet* net) {
  if (!net) return;
  (void)hipStreamSynchronize(net->stream);
  free_net(net);
}

int unet_set_stream(unet* net, void* s) {
  if (!net) return fail(UNET_EINVAL, "null network");
  net->stream = as_stream(s);
  return UNET_OK;
}

int unet_num_params(unet* net, int64_t* count) {
  if (!net || !count) return fail(UNET_EINVAL, "null argument");
  *count = net->nparams;
  return UNET_OK;
}

int unet_get_params(unet* net, float* host) {
  if (!net || !host) return fail(UNET_EINVAL, "null argument");
  UCHECK(hipStreamSynchronize(net->stream));
  UCHECK(hipMemcpy(host, net->p, sizeof(float) * net->nparams, hipMemcpyDeviceToHost));
  return UNET_OK;
}

int unet_set_params(unet* net, const float* host) {
  if (!net || !host) return fail(UNET_EINVAL, "null argument");
  UCHECK(hipStreamSynchronize(net->stream));
  UCHECK(hipMemcpy(net->p, host, sizeof(float) * net->nparams, hipMemcpyHostToDevice));
  UCHECK(hipMemset(net->m, 0, sizeof(float) * net->nparams));
  UCHECK(hipMemset(net->v, 0, sizeof(float) * net->nparams));
  net->t = 0;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(net->nparams)), dim3(256), 0, net->stream,
                     net->p, net->pb, net->nparams);
  UCHECK(hipGetLastError());
  UCHECK(hipStreamSynchronize(net->stream));
  return UNET_OK;
}

int unet_get_grads(unet* net, float* host) {
  if (!net || !host) return fail(UNET_EINVAL, "null argument");
  UCHECK(hipStreamSynchronize(net->stream));
  UCHECK(hipMemcpy(host, net->grad, sizeof(float) * net->nparams, hipMemcpyDeviceToHost));
  return UNET_OK;
}

int unet_forward(unet* net, const void* x0, int32_t n, float* out) {
  if (!net || !x0 || !out) return fail(UNET_EINVAL, "null argument");
  if (n <= 0 || n > net->max_batch) return fail(UNET_EINVAL, "batch size outside [1, max_batch]");
  return forward_impl(net, static_cast<const bf16*>(x0), n, out);
}

int unet_backward(unet* net, const void* x0, const float* target, const uint8_t* fluid,
                  int32_t n, double* loss) {
  if (!net || !x0 || !target || !fluid) return fail(UNET_EINVAL, "null argument");
  if (n <= 0 || n > net->max_batch) return fail(UNET_EINVAL, "batch size outside [1, max_batch]");
  int rc = forward_impl(net, static_cast<const bf16*>(x0), n, net->out);
  if (rc) return rc;
  rc = unet_mse_loss(net->out, UNET_OUT_CHANNELS, target, fluid, (int64_t)n * net->res * net->res,
                     net->gout, loss, net->lwork, net->stream);
  if (rc) return rc;
  return backward_impl(net, n);
}

int unet_train_step(unet* net, const void* x0, const float* target, const uint8_t* fluid,
                    int32_t n, double lr, double* loss) {
  int rc = unet_backward(net, x0, target, fluid, n, loss);
  if (rc) return rc;
  net->t += 1;
  return unet_adam(net->p, net->m, net->v, net->grad, net->pb, net->nparams, lr, 0.9, 0.999, 1e-8,
                   net->t, net->stream);
}

}  // extern "C"
