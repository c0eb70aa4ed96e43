// Host side of the learned warm start (cg_net.h): layer table, parameter
// and activation buffers, and the order of kernel launches of the forward
// and backward passes of the encoder-decoder.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <random>
#include <string>
#include <vector>

#include "cg.h"
#include "cg_net.h"
#include "host.h"

namespace cgn {
bool conv3_supported(int Cin, int Cout);
void launch_conv3(const uint16_t* in, int Cin, const uint16_t* wA, const float* bias, uint16_t* out, int Cout, int Bn,
                  int H, int W, int relu, hipStream_t s);
int64_t wgrad_splits(int64_t P, int Cin, int Cout, int64_t* px_per_block);
int64_t bias_blocks(int64_t P, int64_t* px_per_block);
void launch_conv3_wgrad(const uint16_t* in, int Cin, const uint16_t* g, int Cout, float* dW, float* part, int Bn, int H, int W,
                        hipStream_t s);
void launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s);
void launch_conv3_f32(const uint16_t* in, int Cin, const uint16_t* wA, float* out, int Cout, int Bn, int H, int W,
                      hipStream_t s);
void launch_relu_mask(const float* g, const uint16_t* act, uint16_t* gm, int64_t n, hipStream_t s);
void launch_pool(const uint16_t* x, uint16_t* y, int Bn, int H, int W, int C, hipStream_t s);
void launch_upcat(const uint16_t* deep, int Cd, const uint16_t* skip, int Cs, uint16_t* cat, int Bn, int H, int W,
                  hipStream_t s);
bool launch_conv3_upcat(const uint16_t* deep, int Cd, const uint16_t* skip, int Cs, const uint16_t* wA,
                        const float* bias, uint16_t* out, int Cout, int Bn, int H, int W, int relu, hipStream_t s);
void launch_up_grad(const float* gcat, int Ccat, int Cd, float* gdeep, int Bn, int Ho, int Wo, hipStream_t s);
void launch_skip_grad(const float* gcat, int Ccat, int Cd, const float* gpool, float* gskip, int Cs, int Bn,
                      int H, int W, hipStream_t s);
void launch_bias_grad(const float* g, const uint16_t* act, int C, int64_t P, float* db, float* part, hipStream_t s);
void launch_head_fwd(const uint16_t* x, int C, const float* w, const float* b, float scale, const float* resid,
                     int rc, float gain, float* out, int64_t P, hipStream_t s);
void launch_head_bwd(const uint16_t* x, int C, const float* w, float scale, const float* out, const float* target,
                     int64_t P, float* gx, float* dw, double* loss, float* part, double* lpart, hipStream_t s);
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s);
void launch_pack_w(const float* w, int Cin, int Cout, uint16_t* wA, uint16_t* wT, hipStream_t s);
void launch_fill_f32(float* x, int64_t n, float v, hipStream_t s);
}  // namespace cgn

using namespace cgh;

namespace {

struct Conv {
  int cin, cout, level;
  int64_t w_off, b_off;      // into the float32 parameter vector
  uint16_t* wA = nullptr;    // bfloat16 [cout][9 cin]
  uint16_t* wT = nullptr;    // bfloat16 [cin][9 cout], taps reversed (input gradient)
};

constexpr char kMagic[8] = {'C', 'G', 'N', 'E', 'T', '0', '0', '2'};

}  // namespace

struct cg_net {
  cg_ctx* ctx = nullptr;
  cg_net_config cfg{};
  int L = 0, c = 0, H = 0, W = 0, maxB = 0;
  std::vector<Conv> conv;    // enc0a, enc0b, ..., enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b
  int64_t head_w = 0, head_b = 0, n_params = 0;
  int64_t step = 0;
  std::vector<void*> allocs;
  float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
  // activations (bfloat16, NHWC) for max_batch inputs
  uint16_t* x_in = nullptr;
  std::vector<uint16_t*> in_l, a_l, e_l;   // encoder: pooled input (l > 0), first and second conv outputs
  std::vector<uint16_t*> cat_l, da_l, d_l; // decoder (levels 0..L-2)
  std::vector<char> cat_ok;                // cat_l[l] holds the last forward's concatenation
  std::vector<const uint16_t*> deep_l;     // the deeper decoder input of level l in that forward
  float* out = nullptr;                    // head output [B][H][W][2] of the last forward
  int lastB = 0;
  // gradient scratch: float32 gradients between layers, one bfloat16
  // buffer for the masked gradient that the matrix-core products consume
  float *GA = nullptr, *GB = nullptr, *GC = nullptr;
  uint16_t* GM = nullptr;
  std::vector<float*> gskip;
  // per-block shares of the parameter gradients and the loss, summed in a
  // fixed order (the backward pass is deterministic)
  float* part = nullptr;
  double* lpart = nullptr;
};

namespace {

int ch(const cg_net* n, int l) { return n->c << l; }
int hl(const cg_net* n, int l) { return n->H >> l; }
int wl(const cg_net* n, int l) { return n->W >> l; }

int net_alloc(cg_net* n, size_t bytes, void** p) {
  HIP_OK(n->ctx, hipMalloc(p, bytes ? bytes : 16));
  n->allocs.push_back(*p);
  return CG_OK;
}

void net_free(cg_net* n) {
  for (void* p : n->allocs) (void)hipFree(p);
  n->allocs.clear();
}

// bfloat16 copies of every conv layer's weights from the float32 vector
void pack_all(cg_net* n, hipStream_t s) {
  for (auto& L : n->conv) cgn::launch_pack_w(n->params + L.w_off, L.cin, L.cout, L.wA, L.wT, s);
}

int check(cg_net* n) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(n->ctx, CG_EDEVICE, std::string("net kernel launch: ") + hipGetErrorString(e));
  return CG_OK;
}

}  // namespace

extern "C" {

int cg_net_create(cg_ctx* ctx, const cg_net_config* cfg, cg_net** out) {
  if (!ctx) return CG_EINVAL;
  if (!cfg || !out) return fail(ctx, CG_EINVAL, "cg_net_create: null argument");
  *out = nullptr;
  const int L = cfg->levels, c = cfg->base_channels;
  if (L < 2 || L > 5) return fail(ctx, CG_EINVAL, "cg_net_create: levels must be 2..5");
  if (c < 32 || c % 32 != 0 || (c << (L - 1)) > 1024)
    return fail(ctx, CG_EINVAL, "cg_net_create: base_channels must be a multiple of 32 (deepest level <= 1024)");
  const int q = 1 << (L - 1);
  if (cfg->height < q || cfg->width < q || cfg->height % q || cfg->width % q || cfg->height > 8192 ||
      cfg->width > 8192)
    return fail(ctx, CG_EINVAL, "cg_net_create: height and width must be multiples of 2^(levels-1), <= 8192");
  if (cfg->max_batch < 1) return fail(ctx, CG_EINVAL, "cg_net_create: max_batch must be >= 1");
  if ((int64_t)cfg->max_batch * cfg->height * cfg->width >= (int64_t)1 << 24)
    return fail(ctx, CG_EINVAL, "cg_net_create: max_batch x height x width must stay below 2^24 pixels");
  if (!std::isfinite(cfg->out_scale)) return fail(ctx, CG_EINVAL, "cg_net_create: bad out_scale");
  if (cfg->in_channels < 1 || cfg->in_channels > 8) return fail(ctx, CG_EINVAL, "cg_net_create: in_channels must be 1..8");
  if (!std::isfinite(cfg->residual_gain) || (cfg->residual_gain != 0.f && cfg->in_channels < 3))
    return fail(ctx, CG_EINVAL, "cg_net_create: a residual gain needs in_channels >= 3");
  HIP_OK(ctx, hipSetDevice(ctx->device));
  cg_net* n = new cg_net();
  n->ctx = ctx;
  n->cfg = *cfg;
  n->L = L;
  n->c = c;
  n->H = cfg->height;
  n->W = cfg->width;
  n->maxB = cfg->max_batch;
  // layer table
  int64_t off = 0;
  auto add = [&](int cin, int cout, int level) {
    Conv cv;
    cv.cin = cin;
    cv.cout = cout;
    cv.level = level;
    cv.w_off = off;
    off += (int64_t)cout * 9 * cin;
    cv.b_off = off;
    off += cout;
    n->conv.push_back(cv);
  };
  for (int l = 0; l < L; ++l) {
    add(l == 0 ? cfg->in_channels : ch(n, l - 1), ch(n, l), l);
    add(ch(n, l), ch(n, l), l);
  }
  for (int l = L - 2; l >= 0; --l) {
    add(ch(n, l + 1) + ch(n, l), ch(n, l), l);
    add(ch(n, l), ch(n, l), l);
  }
  n->head_w = off;
  off += 2 * c;
  n->head_b = off;
  off += 2;
  n->n_params = off;
  int rc = CG_OK;
  auto A = [&](size_t bytes, void** p) {
    if (rc == CG_OK) rc = net_alloc(n, bytes, p);
  };
  const size_t pb = sizeof(float) * (size_t)off;
  A(pb, (void**)&n->params);
  A(pb, (void**)&n->grads);
  A(pb, (void**)&n->m);
  A(pb, (void**)&n->v);
  for (auto& cv : n->conv) {
    const size_t wb = sizeof(uint16_t) * (size_t)cv.cout * 9 * cv.cin;
    A(wb, (void**)&cv.wA);
    A(wb, (void**)&cv.wT);
  }
  const int64_t B = n->maxB;
  auto act = [&](int l, int C) { return sizeof(uint16_t) * (size_t)B * hl(n, l) * wl(n, l) * C; };
  A(act(0, cfg->in_channels), (void**)&n->x_in);
  n->in_l.assign(L, nullptr);
  n->a_l.assign(L, nullptr);
  n->e_l.assign(L, nullptr);
  n->cat_l.assign(L, nullptr);
  n->da_l.assign(L, nullptr);
  n->d_l.assign(L, nullptr);
  n->gskip.assign(L, nullptr);
  size_t gmax = act(0, 2 * c);
  for (int l = 0; l < L; ++l) {
    if (l > 0) A(act(l, ch(n, l - 1)), (void**)&n->in_l[l]);
    A(act(l, ch(n, l)), (void**)&n->a_l[l]);
    A(act(l, ch(n, l)), (void**)&n->e_l[l]);
    gmax = std::max(gmax, act(l, ch(n, l)));
    if (l < L - 1) {
      const int cc = ch(n, l + 1) + ch(n, l);
      A(act(l, cc), (void**)&n->cat_l[l]);
      A(act(l, ch(n, l)), (void**)&n->da_l[l]);
      A(act(l, ch(n, l)), (void**)&n->d_l[l]);
      A(2 * act(l, ch(n, l)), (void**)&n->gskip[l]);
      gmax = std::max(gmax, act(l, cc));
    }
  }
  A(sizeof(float) * (size_t)B * n->H * n->W * 2, (void**)&n->out);
  {
    // largest share table of any layer at any batch up to max_batch
    size_t parts = 0;
    const int64_t hblocks = (B * n->H * n->W + 255) / 256;
    parts = std::max(parts, (size_t)hblocks * (2 * c + 2));
    for (const Conv& cv : n->conv)
      for (int64_t b = 1; b <= B; ++b) {
        const int64_t P = b * hl(n, cv.level) * wl(n, cv.level);
        parts = std::max(parts, (size_t)cgn::wgrad_splits(P, cv.cin, cv.cout, nullptr) * cv.cout * 9 * cv.cin);
        parts = std::max(parts, (size_t)cgn::bias_blocks(P, nullptr) * cv.cout);
      }
    A(sizeof(float) * parts, (void**)&n->part);
    A(sizeof(double) * (size_t)hblocks, (void**)&n->lpart);
  }
  A(2 * gmax, (void**)&n->GA);
  A(2 * gmax, (void**)&n->GB);
  A(2 * gmax, (void**)&n->GC);
  A(gmax, (void**)&n->GM);
  if (rc != CG_OK) {
    net_free(n);
    delete n;
    return rc;
  }
  // He-normal weights, zero biases (host generator, seeded)
  std::vector<float> h((size_t)off, 0.f);
  std::mt19937_64 gen(cfg->seed);
  for (auto& cv : n->conv) {
    std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / (9.0 * cv.cin)));
    for (int64_t i = 0; i < (int64_t)cv.cout * 9 * cv.cin; ++i) h[cv.w_off + i] = (float)nd(gen);
  }
  {
    std::normal_distribution<double> nd(0.0, std::sqrt(1.0 / c));
    for (int64_t i = 0; i < 2 * c; ++i) h[n->head_w + i] = (float)nd(gen);
  }
  hipStream_t st = ctx->stream;
  if (hipMemcpyAsync(n->params, h.data(), pb, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    net_free(n);
    delete n;
    return fail(ctx, CG_EDEVICE, "cg_net_create: weight upload failed");
  }
  cgn::launch_fill_f32(n->grads, off, 0.f, st);
  cgn::launch_fill_f32(n->m, off, 0.f, st);
  cgn::launch_fill_f32(n->v, off, 0.f, st);
  pack_all(n, st);
  if ((rc = check(n)) || hipStreamSynchronize(st) != hipSuccess) {
    net_free(n);
    delete n;
    return rc ? rc : fail(ctx, CG_EDEVICE, "cg_net_create: initialisation failed");
  }
  *out = n;
  return CG_OK;
}

int cg_net_destroy(cg_net* n) {
  if (!n) return CG_EINVAL;
  (void)hipSetDevice(n->ctx->device);
  (void)hipDeviceSynchronize();
  net_free(n);
  delete n;
  return CG_OK;
}

int64_t cg_net_n_params(const cg_net* n) { return n ? n->n_params : -1; }

int cg_net_get_params(cg_net* n, float* dst, void* stream) {
  if (!n) return CG_EINVAL;
  if (!dst) return fail(n->ctx, CG_EINVAL, "cg_net_get_params: null destination");
  hipStream_t st = pick_stream(n->ctx, stream);
  HIP_OK(n->ctx, hipMemcpyAsync(dst, n->params, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st));
  return CG_OK;
}

int cg_net_set_params(cg_net* n, const float* src, void* stream) {
  if (!n) return CG_EINVAL;
  if (!src) return fail(n->ctx, CG_EINVAL, "cg_net_set_params: null source");
  hipStream_t st = pick_stream(n->ctx, stream);
  HIP_OK(n->ctx, hipMemcpyAsync(n->params, src, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st));
  pack_all(n, st);
  return check(n);
}

int cg_net_get_grads(cg_net* n, float* dst, void* stream) {
  if (!n) return CG_EINVAL;
  if (!dst) return fail(n->ctx, CG_EINVAL, "cg_net_get_grads: null destination");
  hipStream_t st = pick_stream(n->ctx, stream);
  HIP_OK(n->ctx, hipMemcpyAsync(dst, n->grads, sizeof(float) * n->n_params, hipMemcpyDeviceToDevice, st));
  return CG_OK;
}

int cg_net_zero_grads(cg_net* n, void* stream) {
  if (!n) return CG_EINVAL;
  hipStream_t st = pick_stream(n->ctx, stream);
  cgn::launch_fill_f32(n->grads, n->n_params, 0.f, st);
  return check(n);
}

int cg_net_forward(cg_net* n, const float* input, int32_t B, float* out, void* stream) {
  if (!n) return CG_EINVAL;
  if (!input || !out) return fail(n->ctx, CG_EINVAL, "cg_net_forward: null argument");
  if (B < 1 || B > n->maxB) return fail(n->ctx, CG_EINVAL, "cg_net_forward: batch outside 1..max_batch");
  (void)hipSetDevice(n->ctx->device);
  hipStream_t st = pick_stream(n->ctx, stream);
  const int L = n->L;
  cgn::launch_to_bf16(input, n->x_in, (int64_t)B * n->H * n->W * n->cfg.in_channels, st);
  size_t li = 0;
  for (int l = 0; l < L; ++l) {
    const int h = hl(n, l), w = wl(n, l);
    const uint16_t* src = n->x_in;
    if (l > 0) {
      cgn::launch_pool(n->e_l[l - 1], n->in_l[l], B, hl(n, l - 1), wl(n, l - 1), ch(n, l - 1), st);
      src = n->in_l[l];
    }
    const Conv& ca = n->conv[li++];
    const Conv& cb = n->conv[li++];
    cgn::launch_conv3(src, ca.cin, ca.wA, n->params + ca.b_off, n->a_l[l], ca.cout, B, h, w, 1, st);
    cgn::launch_conv3(n->a_l[l], cb.cin, cb.wA, n->params + cb.b_off, n->e_l[l], cb.cout, B, h, w, 1, st);
  }
  const uint16_t* deep = n->e_l[L - 1];
  n->cat_ok.assign(L, 0);
  n->deep_l.assign(L, nullptr);
  for (int l = L - 2; l >= 0; --l) {
    const int h = hl(n, l), w = wl(n, l);
    const Conv& ca = n->conv[li++];
    const Conv& cb = n->conv[li++];
    // the concatenation [up(deep), e_l] is read in place where the row-staged
    // convolution applies (the backward pass builds it when it needs it)
    n->deep_l[l] = deep;
    if (!cgn::launch_conv3_upcat(deep, ch(n, l + 1), n->e_l[l], ch(n, l), ca.wA, n->params + ca.b_off, n->da_l[l],
                                 ca.cout, B, h, w, 1, st)) {
      cgn::launch_upcat(deep, ch(n, l + 1), n->e_l[l], ch(n, l), n->cat_l[l], B, h, w, st);
      n->cat_ok[l] = 1;
      cgn::launch_conv3(n->cat_l[l], ca.cin, ca.wA, n->params + ca.b_off, n->da_l[l], ca.cout, B, h, w, 1, st);
    }
    cgn::launch_conv3(n->da_l[l], cb.cin, cb.wA, n->params + cb.b_off, n->d_l[l], cb.cout, B, h, w, 1, st);
    deep = n->d_l[l];
  }
  const int64_t P = (int64_t)B * n->H * n->W;
  cgn::launch_head_fwd(deep, n->c, n->params + n->head_w, n->params + n->head_b, n->cfg.out_scale,
                       n->cfg.residual_gain != 0.f ? input : nullptr, n->cfg.in_channels, n->cfg.residual_gain, n->out,
                       P, st);
  HIP_OK(n->ctx, hipMemcpyAsync(out, n->out, sizeof(float) * P * 2, hipMemcpyDeviceToDevice, st));
  n->lastB = B;
  return check(n);
}

int cg_net_backward(cg_net* n, const float* target, int32_t B, double* loss, void* stream) {
  if (!n) return CG_EINVAL;
  if (!target) return fail(n->ctx, CG_EINVAL, "cg_net_backward: null target");
  if (B != n->lastB || B < 1) return fail(n->ctx, CG_EINVAL, "cg_net_backward: batch differs from the last forward");
  (void)hipSetDevice(n->ctx->device);
  hipStream_t st = pick_stream(n->ctx, stream);
  const int L = n->L;
  const int64_t P0 = (int64_t)B * n->H * n->W;
  float* G = n->grads;
  // head: gradient of d_0 into GA
  const uint16_t* d0 = L >= 2 ? n->d_l[0] : n->e_l[0];
  cgn::launch_head_bwd(d0, n->c, n->params + n->head_w, n->cfg.out_scale, n->out, target, P0, n->GA,
                       G + n->head_w, loss, n->part, n->lpart, st);   // head_b follows head_w
  // decoder, from level 0 upwards; conv index of dec level l: 2L + 2 (L-2-l)
  for (int l = 0; l <= L - 2; ++l) {
    const int h = hl(n, l), w = wl(n, l);
    const int64_t P = (int64_t)B * h * w;
    const Conv& ca = n->conv[2 * L + 2 * (L - 2 - l)];
    const Conv& cb = n->conv[2 * L + 2 * (L - 2 - l) + 1];
    // d = relu(conv_b(da)); GA holds the gradient of d
    cgn::launch_relu_mask(n->GA, n->d_l[l], n->GM, P * cb.cout, st);
    cgn::launch_conv3_wgrad(n->da_l[l], cb.cin, n->GM, cb.cout, G + cb.w_off, n->part, B, h, w, st);
    cgn::launch_bias_grad(n->GA, n->d_l[l], cb.cout, P, G + cb.b_off, n->part, st);
    cgn::launch_conv3_f32(n->GM, cb.cout, cb.wT, n->GB, cb.cin, B, h, w, st);
    // da = relu(conv_a(cat))
    cgn::launch_relu_mask(n->GB, n->da_l[l], n->GM, P * ca.cout, st);
    if (!n->cat_ok[l]) {   // the forward read it in place
      cgn::launch_upcat(n->deep_l[l], ch(n, l + 1), n->e_l[l], ch(n, l), n->cat_l[l], B, h, w, st);
      n->cat_ok[l] = 1;
    }
    cgn::launch_conv3_wgrad(n->cat_l[l], ca.cin, n->GM, ca.cout, G + ca.w_off, n->part, B, h, w, st);
    cgn::launch_bias_grad(n->GB, n->da_l[l], ca.cout, P, G + ca.b_off, n->part, st);
    cgn::launch_conv3_f32(n->GM, ca.cout, ca.wT, n->GC, ca.cin, B, h, w, st);
    // cat = [up(deep), e_l]
    const int Cd = ch(n, l + 1), Cs = ch(n, l);
    cgn::launch_skip_grad(n->GC, Cd + Cs, Cd, nullptr, n->gskip[l], Cs, B, h, w, st);
    cgn::launch_up_grad(n->GC, Cd + Cs, Cd, n->GA, B, hl(n, l + 1), wl(n, l + 1), st);
  }
  // encoder, from the deepest level down; GA holds the gradient of e_{L-1}
  for (int l = L - 1; l >= 0; --l) {
    const int h = hl(n, l), w = wl(n, l);
    const int64_t P = (int64_t)B * h * w;
    const Conv& ca = n->conv[2 * l];
    const Conv& cb = n->conv[2 * l + 1];
    if (l < L - 1)  // e_l feeds the decoder skip and the pooled input of level l+1 (gradient in GC)
      cgn::launch_skip_grad(n->gskip[l], ch(n, l), 0, n->GC, n->GA, ch(n, l), B, h, w, st);
    cgn::launch_relu_mask(n->GA, n->e_l[l], n->GM, P * cb.cout, st);
    cgn::launch_conv3_wgrad(n->a_l[l], cb.cin, n->GM, cb.cout, G + cb.w_off, n->part, B, h, w, st);
    cgn::launch_bias_grad(n->GA, n->e_l[l], cb.cout, P, G + cb.b_off, n->part, st);
    cgn::launch_conv3_f32(n->GM, cb.cout, cb.wT, n->GB, cb.cin, B, h, w, st);
    cgn::launch_relu_mask(n->GB, n->a_l[l], n->GM, P * ca.cout, st);
    const uint16_t* src = l == 0 ? n->x_in : n->in_l[l];
    cgn::launch_conv3_wgrad(src, ca.cin, n->GM, ca.cout, G + ca.w_off, n->part, B, h, w, st);
    cgn::launch_bias_grad(n->GB, n->a_l[l], ca.cout, P, G + ca.b_off, n->part, st);
    if (l > 0) cgn::launch_conv3_f32(n->GM, ca.cout, ca.wT, n->GC, ca.cin, B, h, w, st);
  }
  return check(n);
}

int cg_net_adam_step(cg_net* n, float lr, float b1, float b2, float eps, void* stream) {
  if (!n) return CG_EINVAL;
  if (!(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps > 0))
    return fail(n->ctx, CG_EINVAL, "cg_net_adam_step: bad hyper-parameters");
  hipStream_t st = pick_stream(n->ctx, stream);
  n->step += 1;
  const float c1 = (float)(1.0 - std::pow((double)b1, (double)n->step));
  const float c2 = (float)(1.0 - std::pow((double)b2, (double)n->step));
  cgn::launch_adam(n->params, n->grads, n->m, n->v, n->n_params, lr, b1, b2, eps, c1, c2, st);
  pack_all(n, st);
  return check(n);
}

int cg_net_save(cg_net* n, const char* path) {
  if (!n) return CG_EINVAL;
  if (!path) return fail(n->ctx, CG_EINVAL, "cg_net_save: null path");
  std::vector<float> h((size_t)n->n_params);
  HIP_OK(n->ctx, hipDeviceSynchronize());
  HIP_OK(n->ctx, hipMemcpy(h.data(), n->params, sizeof(float) * n->n_params, hipMemcpyDeviceToHost));
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return fail(n->ctx, CG_EINVAL, std::string("cg_net_save: cannot write ") + tmp);
    const int32_t hdr[5] = {n->cfg.base_channels, n->cfg.levels, n->cfg.height, n->cfg.width, n->cfg.in_channels};
    f.write(kMagic, 8);
    f.write((const char*)hdr, sizeof(hdr));
    f.write((const char*)&n->cfg.out_scale, sizeof(float));
    f.write((const char*)&n->cfg.residual_gain, sizeof(float));
    const int64_t np = n->n_params;
    f.write((const char*)&np, sizeof(np));
    f.write((const char*)h.data(), sizeof(float) * h.size());
    if (!f) return fail(n->ctx, CG_EINVAL, "cg_net_save: write failed");
  }
  if (std::rename(tmp.c_str(), path) != 0) return fail(n->ctx, CG_EINVAL, "cg_net_save: rename failed");
  return CG_OK;
}

int cg_net_load(cg_net* n, const char* path) {
  if (!n) return CG_EINVAL;
  if (!path) return fail(n->ctx, CG_EINVAL, "cg_net_load: null path");
  std::ifstream f(path, std::ios::binary);
  if (!f) return fail(n->ctx, CG_EINVAL, std::string("cg_net_load: cannot read ") + path);
  char mg[8];
  int32_t hdr[5];
  float sc = 0.f, gain = 0.f;
  int64_t np = 0;
  f.read(mg, 8);
  f.read((char*)hdr, sizeof(hdr));
  f.read((char*)&sc, sizeof(sc));
  f.read((char*)&gain, sizeof(gain));
  f.read((char*)&np, sizeof(np));
  if (!f || memcmp(mg, kMagic, 8) != 0) return fail(n->ctx, CG_EINVAL, "cg_net_load: not a net file");
  if (hdr[0] != n->cfg.base_channels || hdr[1] != n->cfg.levels || hdr[4] != n->cfg.in_channels ||
      np != n->n_params)
    return fail(n->ctx, CG_EINVAL, "cg_net_load: architecture differs from the net's");
  std::vector<float> h((size_t)np);
  f.read((char*)h.data(), sizeof(float) * h.size());
  if (!f) return fail(n->ctx, CG_EINVAL, "cg_net_load: truncated file");
  n->cfg.out_scale = sc;
  n->cfg.residual_gain = gain;
  HIP_OK(n->ctx, hipDeviceSynchronize());
  HIP_OK(n->ctx, hipMemcpy(n->params, h.data(), sizeof(float) * np, hipMemcpyHostToDevice));
  hipStream_t st = n->ctx->stream;
  pack_all(n, st);
  HIP_OK(n->ctx, hipStreamSynchronize(st));
  return check(n);
}

}  // extern "C"
