/*
 * Learned warm start for steady lattice Boltzmann runs: a small 2-D U-Net
 * that maps a geometry and its flow parameters to an initial density and
 * velocity field, run and trained with hand-written BF16 MFMA kernels for
 * gfx950 (FP32 accumulation).  The lattice Boltzmann method itself (see
 * lbm.h) then starts from the equilibrium at the predicted fields; the
 * network only changes where the iteration starts, never its fixed point.
 *
 * Tensors are NHWC: element (n, y, x, c) of a tensor with pixel stride ld
 * (in elements) is at ((n*H + y)*W + x)*ld + c.  Activations and weights are
 * bfloat16 (stored as raw 16-bit words); accumulation, the output layer,
 * targets, gradients of the parameters and the optimizer state are FP32.
 * Channel counts of convolutions are multiples of 32; ld and channel
 * offsets are multiples of 8 elements; device pointers come from
 * hipMalloc (256-byte aligned).
 *
 * Every function returns 0 (UNET_OK) or a negative error code and leaves a
 * thread-local message for unet_last_error().  Device pointers are owned by
 * the caller unless stated otherwise; calls are asynchronous on the given
 * stream (NULL = the null stream) unless they return host values.
 */
#ifndef UNET_H
#define UNET_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { UNET_OK = 0, UNET_EINVAL = -1, UNET_ENOMEM = -2, UNET_EDEVICE = -3 };

/* Number of input channels of the network (geometry and flow parameters,
 * zero padded) and of its output layer (the first three are used: the
 * normalised density deviation (rho - 1)/(3 U^2), u_x/U and u_y/U). */
#define UNET_IN_CHANNELS 32
#define UNET_OUT_CHANNELS 32

/* Case kinds of the rectangular input/output maps (case_params[i][3]). */
enum { UNET_KIND_CAVITY = 0, UNET_KIND_CHANNEL = 1 };

/* ---------------------------------------------------------------------- */
/* Layer kernels (stateless)                                               */
/* ---------------------------------------------------------------------- */

/* 3x3 convolution with zero padding, stride 1 (cross-correlation, as in
 * every CNN library): y[p][co] = bias[co] + sum_{tap, ci} x[p + tap][ci] *
 * w[co][tap][ci], taps in row-major order (dy, dx) in {-1,0,1}^2.  x: bf16
 * [n*h*w][ldx] (channels [0, cin) read); w: bf16 [cout][9][cin]; bias: FP32
 * [cout] or NULL; y: [n*h*w][ldy], bf16 or, with out_f32, FP32.  relu != 0
 * applies max(0, .) before the store.  cin, cout multiples of 32. */
int unet_conv3x3_fwd(const void* x, int32_t ldx, const void* w, const float* bias, void* y,
                     int32_t ldy, int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout,
                     int32_t relu, int32_t out_f32, void* stream);

/* Gradient with respect to the input of the convolution above:
 * dx[p][ci] = sum_{tap, co} dy[p - tap][co] * w[co][tap][ci] (bf16 out).
 * work: device scratch of at least 18 * cin * cout bytes (the flipped,
 * transposed weights). */
int unet_conv3x3_bwd_data(const void* dy, int32_t lddy, const void* w, void* dx, int32_t lddx,
                          int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout, void* work,
                          void* stream);

/* Gradients with respect to the weights and bias: dw[co][tap][ci] =
 * sum_p dy[p][co] * x[p + tap][ci] and dbias[co] = sum_p dy[p][co] (FP32,
 * overwritten; dbias may be NULL).  work: FP32 device scratch of
 * unet_wgrad_work_floats(n, h, wd, cin, cout) entries.  The pixel sum is
 * split over blocks and the partial sums are added in a fixed order. */
int64_t unet_wgrad_work_floats(int32_t n, int32_t h, int32_t wd, int32_t cin, int32_t cout);
int unet_conv3x3_bwd_weight(const void* dy, int32_t lddy, const void* x, int32_t ldx, float* dw,
                            float* dbias, int32_t n, int32_t h, int32_t wd, int32_t cin,
                            int32_t cout, float* work, void* stream);

/* d[p][c] = 0 where y[p][c] <= 0 (backward of the ReLU applied in the
 * forward convolution; y is its output), in place, c < ch. */
int unet_relu_bwd(void* d, int32_t ldd, const void* y, int32_t ldy, int64_t npix, int32_t ch,
                  void* stream);

/* 2x2 average pooling (h, wd even: the input size) and its backward:
 * dx = add + dy/4 on each of the four inputs (add may be NULL). */
int unet_pool2_fwd(const void* x, int32_t ldx, void* y, int32_t ldy, int32_t n, int32_t h,
                   int32_t wd, int32_t ch, void* stream);
int unet_pool2_bwd(const void* dy, int32_t lddy, const void* add, int32_t ldadd, void* dx,
                   int32_t lddx, int32_t n, int32_t h, int32_t wd, int32_t ch, void* stream);

/* Nearest-neighbour 2x upsampling (h, wd: the coarse size) and its
 * backward (sum of the four fine gradients). */
int unet_up2_fwd(const void* x, int32_t ldx, void* y, int32_t ldy, int32_t n, int32_t h,
                 int32_t wd, int32_t ch, void* stream);
int unet_up2_bwd(const void* dy, int32_t lddy, void* dx, int32_t lddx, int32_t n, int32_t h,
                 int32_t wd, int32_t ch, void* stream);

/* Masked mean-squared error over the first three output channels:
 * L = sum_{fluid p, c<3} (out[p][c] - t[p][c])^2 / (3 * #fluid), with
 * out FP32 [npix][ldo], t FP32 [npix][3], fluid u8 [npix] (nonzero = use).
 * Writes dout (bf16 [npix][ldo], zero outside the fluid and for c >= 3),
 * and the loss to *loss (host; synchronises the stream).  work: FP64 device
 * scratch of unet_loss_work_doubles(npix) entries. */
int64_t unet_loss_work_doubles(int64_t npix);
int unet_mse_loss(const float* out, int32_t ldo, const float* target, const uint8_t* fluid,
                  int64_t npix, void* dout, double* loss, double* work, void* stream);

/* Adam step (Kingma & Ba, 2015) on FP32 parameters p with moments m, v:
 * t is the 1-based step count; also writes the bf16 copy pb (may be NULL). */
int unet_adam(float* p, float* m, float* v, const float* g, void* pb, int64_t count, double lr,
              double beta1, double beta2, double eps, int64_t t, void* stream);

/* Network input from geometry and flow parameters: for case i the solid
 * mask (u8, [n][fine][fine], any fine >= 1) becomes a solid fraction at
 * res x res (coarse cell I covers the fine nodes floor(I fine/res) ..
 * floor((I+1) fine/res) - 1, at least one node); case_params[i] =
 * {Re, gamma, U} (FP32, device).  x0: bf16 [n][res][res][UNET_IN_CHANNELS]:
 * channel 0 solid fraction, 1 Re/500, 2 gamma, 3 U/0.1, 4 x, 5 y (node
 * centres scaled to (0, 1)), 6 one on the top row (lid), 7 one; rest 0. */
int unet_make_input(const uint8_t* solid, int32_t fine, const float* case_params, int32_t n,
                    int32_t res, void* x0, void* stream);

/* Lattice fields from the network output (FP32 [n][res][res][ldo]):
 * bilinear interpolation to the fine grid, rho = 1 + 3 U^2 o0,
 * u = U (o1, o2); solid nodes get rho = 1, u = 0.  Per case, the fluid mean
 * of rho - 1 is removed (the warm start holds the cold start's mass), and
 * so are the staggered momenta sum (-1)^i rho u_x and sum (-1)^j rho u_y
 * (u_x -= (-1)^i c_x, c_x = sum (-1)^i rho u_x / sum rho; likewise u_y):
 * with bounce-back walls every step flips their sign, so a start that
 * carries them keeps an undamped period-2 oscillation and never reaches a
 * steady state, while the state at rest carries none.
 * rho, ux, uy: FP32 device [n][fine][fine]. */
int unet_fields_from_output(const float* out, int32_t ldo, int32_t n, int32_t res,
                            const float* case_params, const uint8_t* solid, int32_t fine,
                            float* rho, float* ux, float* uy, void* stream);

/* The same two maps for lattices of nx x ny nodes (cavities and channels
 * alike): solid is u8 [n][ny][nx]; case_params[i] = {Re, gamma, U, kind}
 * (FP32, device; kind UNET_KIND_CAVITY or UNET_KIND_CHANNEL, as a float).
 * Coarse cells cover floor(I nx/res) .. floor((I+1) nx/res) - 1 along x and
 * likewise along y with ny.  Channel 6 of the input marks the driven
 * boundary: the top row of a cavity (lid), the left column of a channel
 * (inlet).  The fields of a cavity are corrected as above; those of a
 * channel (its inlet and outlet change the mass, and it keeps no staggered
 * sums) are the interpolated prediction as it is.  rho, ux, uy: FP32 device
 * [n][ny][nx].  With square lattices and kind 0 the results equal those of
 * unet_make_input and unet_fields_from_output. */
int unet_make_input_rect(const uint8_t* solid, int32_t nx, int32_t ny, const float* case_params,
                         int32_t n, int32_t res, void* x0, void* stream);
int unet_fields_from_output_rect(const float* out, int32_t ldo, int32_t n, int32_t res,
                                 const float* case_params, const uint8_t* solid, int32_t nx,
                                 int32_t ny, float* rho, float* ux, float* uy, void* stream);

/* ---------------------------------------------------------------------- */
/* The network: 4 levels, 32/64/128/256 channels, two 3x3 convolutions      */
/* (ReLU) per level, 2x2 average pooling down, nearest upsampling and       */
/* channel concatenation of the skip connection up, a linear 3x3 output     */
/* convolution.  It owns its parameters, Adam state and activations for up  */
/* to max_batch samples at res x res (res a multiple of 8).                 */
/* ---------------------------------------------------------------------- */
typedef struct unet unet;

/* Parameters are initialised (He normal, biases zero) from a SplitMix64
 * stream seeded with `seed`. */
int unet_create(int32_t max_batch, int32_t res, uint64_t seed, unet** out);
void unet_destroy(unet* net);
int unet_set_stream(unet* net, void* hip_stream);

/* Parameter vector (FP32): layers in network order, each weights
 * [cout][9][cin] then bias [cout]. */
int unet_num_params(unet* net, int64_t* count);
int unet_get_params(unet* net, float* host);
int unet_set_params(unet* net, const float* host);
/* Gradient of the last unet_train_step (or unet_backward), same layout. */
int unet_get_grads(unet* net, float* host);

/* Forward pass: x0 bf16 [n][res][res][UNET_IN_CHANNELS] (device) ->
 * out FP32 [n][res][res][UNET_OUT_CHANNELS] (device).  n <= max_batch. */
int unet_forward(unet* net, const void* x0, int32_t n, float* out);

/* Forward, masked MSE loss against target (FP32 device [n][res][res][3],
 * fluid u8 device [n][res][res]) and backward; the gradients stay in the
 * network (unet_get_grads).  *loss on the host. */
int unet_backward(unet* net, const void* x0, const float* target, const uint8_t* fluid,
                  int32_t n, double* loss);

/* unet_backward followed by one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8) with learning rate lr. */
int unet_train_step(unet* net, const void* x0, const float* target, const uint8_t* fluid,
                    int32_t n, double lr, double* loss);

const char* unet_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* UNET_H */
