/*
 * cg_net.h -- learned warm start of libcg: a convolutional encoder-decoder
 * (U-Net) that predicts the displacement field of a converged cartogram
 * from the log-density texture of the original map, trained and run by the
 * library's own HIP kernels (bfloat16 weights and activations, float32
 * accumulation on the matrix cores).
 *
 * The paper has no learned component; it notes that a good starting
 * deformation (the previous step of a series, Method: time-varying
 * cartograms) shortens the iteration.  The warm start is such a starting
 * deformation.  The plain iteration always follows it and judges it: see
 * cg_series_desc.init_field and CG_FLAG_FALLBACK in cg.h.
 *
 * Architecture (fixed by the config): `levels` resolutions; level l has
 * base_channels * 2^l channels and two 3x3 convolutions (zero padding,
 * bias, ReLU); 2x2 average pooling between encoder levels; the decoder
 * upsamples x2 (nearest), concatenates [upsampled, encoder skip] and
 * applies two 3x3 convolutions; a 1x1 head maps base_channels to 2 and
 * multiplies by out_scale; with a residual gain g the output adds g times
 * input channels 1 and 2 (a first estimate of the field given as input).
 * Output = displacement (dx, dy) in units of the unit square at the pixel
 * centres of the input.
 *
 * Parameter vector (float32, this order): for each 3x3 layer (enc0a,
 * enc0b, enc1a, ..., enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b)
 * W[o][ky][kx][c] then bias[o]; then the head W[2][base] and bias[2].
 *
 * Every array argument is device memory unless its comment says host.
 * Calls are asynchronous on `stream` (NULL = HIP null stream) and return
 * CG_OK or a negative CG_E* code (text via cg_last_error of the context).
 */
#ifndef CG_NET_H_
#define CG_NET_H_

#include <stddef.h>
#include <stdint.h>

#include "cg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cg_net cg_net;

typedef struct {
  int32_t base_channels; /* channels of level 0; a multiple of 32 */
  int32_t levels;        /* 2..5 */
  int32_t height, width; /* input size; multiples of 2^(levels-1) */
  int32_t max_batch;     /* largest batch passed to forward / backward; max_batch x height x width < 2^24 */
  float out_scale;       /* head output multiplier */
  uint64_t seed;         /* weight initialisation (He normal, zero biases) */
  int32_t in_channels;   /* input channels, 1..8 */
  float residual_gain;   /* output += residual_gain * input channels 1, 2 (needs in_channels >= 3; 0 = off) */
} cg_net_config;

/* Create a net on the context's device; allocates weights, Adam moments,
 * gradients and the activations of `max_batch` inputs.  CG_EINVAL on a
 * config outside the limits above. */
int cg_net_create(cg_ctx* ctx, const cg_net_config* cfg, cg_net** out);
int cg_net_destroy(cg_net* net);
int64_t cg_net_n_params(const cg_net* net);

/* Copy the float32 parameter vector out of / into the net (device
 * [n_params]); set_params also refreshes the bfloat16 working copies. */
int cg_net_get_params(cg_net* net, float* dst, void* stream);
int cg_net_set_params(cg_net* net, const float* src, void* stream);
/* Accumulated gradients (device [n_params]) and their reset. */
int cg_net_get_grads(cg_net* net, float* dst, void* stream);
int cg_net_zero_grads(cg_net* net, void* stream);

/* Forward pass: input float [B][H][W][in_channels] (channel 0: log of
 * density over its mean; further channels as the caller's features),
 * output float [B][H][W][2] (dx, dy).  Keeps the activations for the next
 * cg_net_backward.  1 <= B <= max_batch. */
int cg_net_forward(cg_net* net, const float* input, int32_t batch, float* out, void* stream);

/* Backward pass of the mean squared error between the last forward's
 * output and `target` (float [B][H][W][2], same B): adds the parameter
 * gradients into the net's gradient buffer; `loss` (device double [1], or
 * NULL) receives the loss, mean over B*H*W*2 values, added to its content. */
int cg_net_backward(cg_net* net, const float* target, int32_t batch, double* loss, void* stream);

/* One Adam step (Kingma and Ba, with bias correction) on the accumulated
 * gradients; the gradients are left as they are. */
int cg_net_adam_step(cg_net* net, float lr, float beta1, float beta2, float eps, void* stream);

/* Save / load the config and parameters to / from a host file path.
 * load fails with CG_EINVAL if the file's architecture differs. */
int cg_net_save(cg_net* net, const char* path);
int cg_net_load(cg_net* net, const char* path);

/* Input of the net for a map: the log-density texture of Step 3 (value
 * over pixel count per region, background = shape x mean density),
 * out[q][p] = log(d(p, q) / mean d), from a label map and the pixel counts
 * of cg_rasterize.  labels [N][N], counts int64 [R+1], values float [R],
 * out float [N][N]. */
int cg_log_density(cg_ctx* ctx, int N, const uint16_t* labels, const int64_t* counts, const float* values,
                   int32_t n_regions, float shape, float* out, void* stream);

/* Log-density textures of n maps in one call (one rasterisation plan for
 * all): for map k, the texture of cg_log_density from the labels and counts
 * cg_rasterize gives for maps[k] at positions xy[k].  maps, xy and values
 * are HOST arrays of n pointers; xy[k] device float [n_vertices_k][2],
 * values[k] device float [R_k] (1 <= R_k <= 65535), out device float
 * [n][N][N].  The learned warm start's first input channel for a batch. */
int cg_log_density_maps(cg_ctx* ctx, int32_t n, const cg_map* const* maps, const float* const* xy, int N,
                        const float* const* values, float shape, float* out, void* stream);

/* Tracer grid of G x G pixel centres: with final == NULL, out[j][i] =
 * ((i + 1/2)/G, (j + 1/2)/G); otherwise out[j][i] = final[j][i] - that
 * centre (the displacement of tracers moved along by cg_step_series).
 * final and out float [G][G][2]. */
int cg_tracer_field(cg_ctx* ctx, int32_t G, const float* final_xy, float* out, void* stream);

/* Box average of a field over factor x factor cells: in float [G][G][2],
 * out float [G/factor][G/factor][2] (factor divides G).  A coarser
 * warm-start field moves neighbouring vertices more alike, which keeps
 * small regions from folding. */
int cg_field_pool(cg_ctx* ctx, int32_t G, const float* in, int32_t factor, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CG_NET_H_ */
