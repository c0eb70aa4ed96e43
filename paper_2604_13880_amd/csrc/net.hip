// Kernels of the learned warm start: a convolutional encoder-decoder
// (U-Net) that maps a log-density texture to the displacement field of the
// converged cartogram.  The net is not part of the paper; it follows the
// paper's remark that a good starting deformation (the previous step of a
// series) shortens the iteration, and is always checked by the plain
// iteration that follows it.
//
// Activations are bfloat16 in NHWC order ([batch][row][column][channel]);
// every convolution accumulates in float32 on the matrix cores
// (v_mfma_f32_16x16x32_bf16).  A 3x3 convolution with C_in input channels
// is an implicit GEMM with K = 9 C_in, k = tap * C_in + c (tap = 3 ky + kx):
//   forward      out[p][o]  = sum_k W[o][k] * patch(in)[p][k]
//   input grad   gin[p][c]  = sum_k W'[c][k'] * patch(g)[p][k']
//                (W'[c][tap' C_out + o] = W[o][(8 - tap') C_in + c])
//   weight grad  dW[o][k]   = sum_p g[p][o] * patch(in)[p][k]
// The first two share one kernel (weights as the A operand, 16 output
// channels per fragment row, 16 pixels per fragment column); the third
// stages pixel-major tiles in LDS transposed so that the pixel index
// becomes the MFMA reduction axis.
#include "cg_net_dev.h"

namespace cgn {

__device__ __forceinline__ bf16x8 load8(const uint16_t* p) {
  return __builtin_bit_cast(bf16x8, *(const u32x4*)p);
}
__device__ __forceinline__ bf16x8 zero8() { return __builtin_bit_cast(bf16x8, u32x4{0u, 0u, 0u, 0u}); }

// ---------------------------------------------------------------------------
// 3x3 convolution (stride 1, zero padding 1) as an implicit GEMM.
// Block: 4 wavefronts x 64 pixels = 256 pixels, 16*MF output channels.
// GEN = element-wise operand gathers (any C_in; used for C_in % 32 != 0).
// F32OUT: float32 output (input gradients), else bfloat16.
template <int MF, bool GEN, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv3(const uint16_t* __restrict__ in, int Cin,
                                               const uint16_t* __restrict__ wA, const float* __restrict__ bias,
                                               void* __restrict__ out, int Cout, int64_t P, int H, int W,
                                               int relu) {
  constexpr int NF = 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int kq = lane >> 4, lr = lane & 15;
  const int64_t px0 = (int64_t)blockIdx.x * 256 + wv * 64;
  const int co0 = blockIdx.y * (16 * MF);
  const int K = 9 * Cin;
  const int64_t HW = (int64_t)H * W;
  int64_t pimg[NF];
  int py[NF], pxx[NF];
  bool pv[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int64_t p = px0 + 16 * f + lr;
    pv[f] = p < P;
    const int64_t b = pv[f] ? p / HW : 0;
    const int64_t rem = pv[f] ? p - b * HW : 0;
    py[f] = (int)(rem / W);
    pxx[f] = (int)(rem - (int64_t)py[f] * W);
    pimg[f] = b * HW;
  }
  f32x4 acc[MF][NF];
#pragma unroll
  for (int m = 0; m < MF; ++m)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[m][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this lane's biases (output channels co0 + 16 m + 4 kq + r), read once
  f32x4 bv[MF];
#pragma unroll
  for (int m = 0; m < MF; ++m)
    bv[m] = bias ? *(const f32x4*)(bias + co0 + 16 * m + 4 * kq) : f32x4{0.f, 0.f, 0.f, 0.f};

  if (!GEN) {
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      const uint16_t* src[NF];
      bool ok[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int yy = py[f] + dy, xx = pxx[f] + dx;
        ok[f] = pv[f] && yy >= 0 && yy < H && xx >= 0 && xx < W;
        src[f] = in + (ok[f] ? ((pimg[f] + (int64_t)yy * W + xx) * Cin + 8 * kq) : 0);
      }
      const uint16_t* wrow = wA + (int64_t)(co0 + lr) * K + tap * Cin + 8 * kq;
      for (int c0 = 0; c0 < Cin; c0 += 32) {
        bf16x8 a[MF], bb[NF];
#pragma unroll
        for (int m = 0; m < MF; ++m) a[m] = load8(wrow + (int64_t)16 * m * K + c0);
#pragma unroll
        for (int f = 0; f < NF; ++f) bb[f] = ok[f] ? load8(src[f] + c0) : zero8();
#pragma unroll
        for (int m = 0; m < MF; ++m)
#pragma unroll
          for (int f = 0; f < NF; ++f)
            acc[m][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[f], acc[m][f], 0, 0, 0);
      }
    }
  } else {
    for (int k0 = 0; k0 < K; k0 += 32) {
      // element gathers from clamped addresses (all in flight together),
      // zeroed afterwards where k or the tap's pixel is outside
      bf16x8 a[MF], bb[NF];
#pragma unroll
      for (int m = 0; m < MF; ++m) {
        const uint16_t* wr = wA + (int64_t)(co0 + 16 * m + lr) * K;
        u16x8 tv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + 8 * kq + e;
          const uint16_t v = wr[k < K ? k : 0];
          tv[e] = k < K ? v : (uint16_t)0;
        }
        a[m] = __builtin_bit_cast(bf16x8, tv);
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        u16x8 tv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int k = k0 + 8 * kq + e;
          const int tap = k / Cin, c = k - tap * Cin;
          const int yy = py[f] + tap / 3 - 1, xx = pxx[f] + tap % 3 - 1;
          const bool ok = k < K && pv[f] && yy >= 0 && yy < H && xx >= 0 && xx < W;
          const uint16_t v = in[ok ? (pimg[f] + (int64_t)yy * W + xx) * Cin + c : 0];
          tv[e] = ok ? v : (uint16_t)0;
        }
        bb[f] = __builtin_bit_cast(bf16x8, tv);
      }
#pragma unroll
      for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f = 0; f < NF; ++f)
          acc[m][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[f], acc[m][f], 0, 0, 0);
    }
  }
  // lane holds D[o = 4 kq + r][pixel = lr] of every fragment
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int64_t p = px0 + 16 * f + lr;
    if (p >= P) continue;
#pragma unroll
    for (int m = 0; m < MF; ++m) {
      const int o = co0 + 16 * m + 4 * kq;
      f32x4 v4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[m][f][r] + bv[m][r];
        if (relu) v = fmaxf(v, 0.f);
        v4[r] = v;
      }
      if (F32OUT) {
        *(f32x4*)((float*)out + p * Cout + o) = v4;
      } else {
        u16x4 tv;
#pragma unroll
        for (int r = 0; r < 4; ++r) tv[r] = f2bf(v4[r]);
        *(u16x4*)((uint16_t*)out + p * Cout + o) = tv;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same convolution for C_in % 32 == 0 when a block's 256 pixels are
// whole rows of one image (W a power of two, 16 <= W <= 128, H W a
// multiple of 256).  For every 32 input channels the block stages in LDS
// its rows plus a one-pixel border ((256/W + 2) x (W + 2) pixels, zeros
// outside the image, 64 bytes per pixel) and the weights of its output
// channels for all nine taps; the taps then read their A and B fragments
// from LDS (B at shifted offsets), so each input pixel is fetched once per
// block and channel chunk instead of once per tap, and the matrix cores
// wait on one round of global loads per chunk (all issued together)
// instead of one per tap and fragment.
constexpr int conv_rows_pix(int W) { return (256 / W + 2) * (W + 2); }
constexpr int kConvRowsMaxPix = conv_rows_pix(128) > conv_rows_pix(16) ? conv_rows_pix(128) : conv_rows_pix(16);
static_assert(conv_rows_pix(32) <= kConvRowsMaxPix && conv_rows_pix(64) <= kConvRowsMaxPix, "LDS tile bound");

bool conv3_rows_ok(int Cin, int64_t P, int H, int W) {
  (void)P;
  return Cin % 32 == 0 && W >= 16 && W <= 128 && (W & (W - 1)) == 0 && ((int64_t)H * W) % 256 == 0;
}

// With `deep` set, the input is the concatenation [nearest x2 upsampling
// of deep (Cd channels at half resolution), in (Cin - Cd channels)] read in
// place: a chunk of 32 channels comes from one of the two (Cd % 32 == 0).
template <int MF, bool F32OUT>
__global__ __launch_bounds__(256) void k_conv3_rows(const uint16_t* __restrict__ in, int Cin,
                                                    const uint16_t* __restrict__ deep, int Cd,
                                                    const uint16_t* __restrict__ wA, const float* __restrict__ bias,
                                                    void* __restrict__ out, int Cout, int64_t P, int H, int W,
                                                    int relu) {
  constexpr int NF = 4;
  constexpr int NA = 9 * 16 * MF * 4;                          // 16-byte pieces of the chunk's weights
  constexpr int HALO_IT = (kConvRowsMaxPix * 4 + 255) / 256;    // pieces per thread
  constexpr int A_IT = (NA + 255) / 256;
  __shared__ __align__(16) uint16_t tile[kConvRowsMaxPix * 32];   // [pixel][32 channels]
  __shared__ __align__(16) uint16_t wl[9 * 16 * MF * 32];        // [tap][output channel][32 channels]
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int kq = lane >> 4, lr = lane & 15;
  const int64_t p0 = (int64_t)blockIdx.x * 256;   // first pixel of the block (whole rows, P % 256 == 0)
  const int co0 = blockIdx.y * (16 * MF);
  const int K = 9 * Cin;
  const int64_t HW = (int64_t)H * W;
  const int64_t img = p0 / HW;
  const int y0 = (int)((p0 - img * HW) / W);
  const int RB = 256 / W, Wp = W + 2;                   // rows of the block, padded row length
  const int npix = (RB + 2) * Wp;
  const int Cs = deep ? Cin - Cd : Cin, Coff = deep ? Cd : 0;   // channels of `in` and where they start
  const uint16_t* src0 = in + img * HW * Cs;
  const uint16_t* deep0 = deep ? deep + img * (HW / 4) * Cd : nullptr;
  // this lane's four pixels (local index wv*64 + 16f + lr): LDS pixel of tap (0, 0)
  int base[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int li = wv * 64 + 16 * f + lr;
    const int r = li / W, c = li - r * W;   // W is a power of two
    base[f] = (r + 1) * Wp + (c + 1);
  }
  f32x4 acc[MF][NF];
#pragma unroll
  for (int m = 0; m < MF; ++m)
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[m][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  // this lane's biases (output channels co0 + 16 m + 4 kq + r), read once
  f32x4 bv[MF];
#pragma unroll
  for (int m = 0; m < MF; ++m)
    bv[m] = bias ? *(const f32x4*)(bias + co0 + 16 * m + 4 * kq) : f32x4{0.f, 0.f, 0.f, 0.f};

  // every load of a chunk in flight together, the next chunk's during
  // this one's products: unconditional loads from clamped addresses,
  // zeroed where outside the image
  u32x4 hv[HALO_IT], av[A_IT];
  bool hok[HALO_IT];
  auto issue = [&](int c0) {
#pragma unroll
    for (int i = 0; i < HALO_IT; ++i) {
      const int e = t + 256 * i;
      const int pix = e >> 2, j = e & 3;
      const int ty = pix / Wp, tx = pix - ty * Wp;
      const int yy = y0 - 1 + ty, xx = tx - 1;
      hok[i] = e < npix * 4 && yy >= 0 && yy < H && xx >= 0 && xx < W;
      if (deep0 && c0 < Cd) {   // uniform per chunk
        const int64_t off = hok[i] ? ((int64_t)(yy >> 1) * (W >> 1) + (xx >> 1)) * Cd + c0 + 8 * j : 0;
        hv[i] = *(const u32x4*)(deep0 + off);
      } else {
        const int64_t off = hok[i] ? ((int64_t)yy * W + xx) * Cs + (c0 - Coff) + 8 * j : 0;
        hv[i] = *(const u32x4*)(src0 + off);
      }
    }
#pragma unroll
    for (int i = 0; i < A_IT; ++i) {
      const int e = min(t + 256 * i, NA - 1);
      const int tap = e / (64 * MF), row = (e >> 2) & (16 * MF - 1), j = e & 3;
      av[i] = *(const u32x4*)(wA + (int64_t)(co0 + row) * K + tap * Cin + c0 + 8 * j);
    }
  };
  issue(0);
  for (int c0 = 0; c0 < Cin; c0 += 32) {
    __syncthreads();   // the previous chunk's LDS reads are done
#pragma unroll
    for (int i = 0; i < HALO_IT; ++i) {
      const int e = t + 256 * i;
      if (e < npix * 4) *(u32x4*)(tile + (e >> 2) * 32 + 8 * (e & 3)) = hok[i] ? hv[i] : u32x4{0u, 0u, 0u, 0u};
    }
#pragma unroll
    for (int i = 0; i < A_IT; ++i) {
      const int e = t + 256 * i;
      if (e < NA) *(u32x4*)(wl + e * 8) = av[i];   // piece e: tap, row, j in that order
    }
    __syncthreads();
    if (c0 + 32 < Cin) issue(c0 + 32);
#pragma unroll 3
    for (int tap = 0; tap < 9; ++tap) {
      const int off = (tap / 3 - 1) * Wp + (tap % 3 - 1);
      bf16x8 a[MF], bb[NF];
#pragma unroll
      for (int m = 0; m < MF; ++m) a[m] = load8(wl + ((tap * 16 * MF + 16 * m + lr) * 32 + 8 * kq));
#pragma unroll
      for (int f = 0; f < NF; ++f) bb[f] = load8(tile + (base[f] + off) * 32 + 8 * kq);
#pragma unroll
      for (int m = 0; m < MF; ++m)
#pragma unroll
        for (int f = 0; f < NF; ++f)
          acc[m][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[f], acc[m][f], 0, 0, 0);
    }
  }
  // lane holds D[o = 4 kq + r][pixel = lr] of every fragment
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int64_t p = p0 + wv * 64 + 16 * f + lr;
#pragma unroll
    for (int m = 0; m < MF; ++m) {
      const int o = co0 + 16 * m + 4 * kq;
      f32x4 v4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float v = acc[m][f][r] + bv[m][r];
        if (relu) v = fmaxf(v, 0.f);
        v4[r] = v;
      }
      if (F32OUT) {
        *(f32x4*)((float*)out + p * Cout + o) = v4;
      } else {
        u16x4 tv;
#pragma unroll
        for (int r = 0; r < 4; ++r) tv[r] = f2bf(v4[r]);
        *(u16x4*)((uint16_t*)out + p * Cout + o) = tv;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Weight gradient dW[o][k] += sum_p g[p][o] * patch(in)[p][k].
// Block: 32 output channels x 128 columns of K, 4 wavefronts each owning 32
// columns; pixels in steps of kWgPix staged in LDS transposed ([channel][pixel]);
// every block stores its partial sums for its share of the pixels
// (blockIdx.z) in part[z][o][k]; k_sum_parts adds the shares to the
// gradient in a fixed order, so the result does not depend on scheduling.
// n = q d + r for 0 <= n < 2^24 and d >= 1, from a float reciprocal
// corrected by one step (the float quotient is off by at most one there).
__device__ __forceinline__ void divmod24(int n, int d, float inv, int& q, int& r) {
  q = (int)((float)n * inv);
  r = n - q * d;
  q = r < 0 ? q - 1 : (r >= d ? q + 1 : q);
  r = n - q * d;
}

constexpr int kWgPix = 64;
constexpr int kWgPad = kWgPix + 8;   // row pitch in LDS (elements)

template <bool GEN>
__global__ __launch_bounds__(256) void k_conv3_wgrad(const uint16_t* __restrict__ in, int Cin,
                                                     const uint16_t* __restrict__ g, int Cout,
                                                     float* __restrict__ part, int64_t P, int H, int W,
                                                     int64_t px_per_block) {
  __shared__ __align__(16) uint16_t As[32][kWgPad];    // g tile [o][pixel]
  __shared__ __align__(16) uint16_t Bs[128][kWgPad];   // patch tile [k][pixel]
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int kq = lane >> 4, lr = lane & 15;
  const int K = 9 * Cin;
  const int k0 = blockIdx.x * 128;
  const int o0 = blockIdx.y * 32;
  const int64_t pbeg = (int64_t)blockIdx.z * px_per_block;
  const int64_t pend = pbeg + px_per_block < P ? pbeg + px_per_block : P;
  const int64_t HW = (int64_t)H * W;
  f32x4 acc[2][2];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int f = 0; f < 2; ++f) acc[m][f] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Per step of kWgPix pixels: the g tile (pixels x 32 channels, one chunk
  // of 8 channels per thread) and the patch tile (pixels x 128 columns of
  // K, 8 columns of four consecutive pixels per thread, C_in % 8 == 0) are
  // loaded from clamped addresses, the next step's while this one's
  // products run, and written to LDS transposed so that pixels are the
  // reduction axis.
  constexpr int NB = kWgPix * 16 / 256;
  u16x8 gv, bv[NB];
  bool gok, bok[NB];
  // pixel -> (row, column) by float reciprocals (P < 2^24, checked on the
  // host); this thread's columns of K, hence its tap, are fixed
  const int HWi = H * W;
  const float inv_hw = 1.f / (float)HWi, inv_w = 1.f / (float)W;
  const int kk_t = (t & 15) * 8, k_t = k0 + kk_t;
  const int tap_t = k_t / Cin, ci_t = k_t - tap_t * Cin;
  const int dy_t = tap_t / 3 - 1, dx_t = tap_t % 3 - 1;
  const bool kok_t = k_t < K;
  auto issue = [&](int64_t p0) {
    {
      const int pi = t >> 2, cc = (t & 3) * 8;
      const int64_t p = p0 + pi;
      gok = p < pend;
      gv = *(const u16x8*)(g + (gok ? p * Cout + o0 + cc : 0));
    }
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      const int p = (int)p0 + NB * (t >> 4) + i;   // NB consecutive pixels per thread
      int b, rem, y, x;
      divmod24(p, HWi, inv_hw, b, rem);
      divmod24(rem, W, inv_w, y, x);
      const int yy = y + dy_t, xx = x + dx_t;
      bok[i] = p < pend && kok_t && yy >= 0 && yy < H && xx >= 0 && xx < W;
      bv[i] = *(const u16x8*)(in + (bok[i] ? ((int64_t)p + dy_t * W + dx_t) * Cin + ci_t : 0));
    }
  };
  if (!GEN) issue(pbeg);
  for (int64_t p0 = pbeg; p0 < pend; p0 += kWgPix) {
    __syncthreads();
    if (!GEN) {
      {
        const int pi = t >> 2, cc = (t & 3) * 8;
#pragma unroll
        for (int e = 0; e < 8; ++e) As[cc + e][pi] = gok ? gv[e] : (uint16_t)0;
      }
      // this thread's NB pixels are consecutive: one 8-byte store per column
      static_assert(NB == 4, "four pixels per 8-byte store");
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        u16x4 w;
#pragma unroll
        for (int i = 0; i < NB; ++i) w[i] = bok[i] ? bv[i][e] : (uint16_t)0;
        *(u16x4*)&Bs[kk_t + e][NB * (t >> 4)] = w;
      }
    } else {
      // g tile as above; patch element by element (any C_in)
      {
        const int pi = t >> 2, cc = (t & 3) * 8;
        const int64_t p = p0 + pi;
        u16x8 v = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
        if (p < pend) v = *(const u16x8*)(g + p * Cout + o0 + cc);
#pragma unroll
        for (int e = 0; e < 8; ++e) As[cc + e][pi] = v[e];
      }
      // this thread's column of K (c & 127 = t & 127) and tap are fixed
      const int kk = t & 127, k = k0 + kk;
      const int tap = k / Cin, ci = k - tap * Cin;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      constexpr int NE = kWgPix * 128 / 256;
      uint16_t ev[NE];
#pragma unroll
      for (int j = 0; j < NE; ++j) {
        const int p = (int)p0 + (t >> 7) + 2 * j;
        int b, rem, y, x;
        divmod24(p, HWi, inv_hw, b, rem);
        divmod24(rem, W, inv_w, y, x);
        const int yy = y + dy, xx = x + dx;
        const bool ok = p < pend && k < K && yy >= 0 && yy < H && xx >= 0 && xx < W;
        const uint16_t v = in[ok ? ((int64_t)p + dy * W + dx) * Cin + ci : 0];
        ev[j] = ok ? v : (uint16_t)0;
      }
#pragma unroll
      for (int j = 0; j < NE; ++j) Bs[kk][(t >> 7) + 2 * j] = ev[j];
    }
    __syncthreads();
    if (!GEN && p0 + kWgPix < pend) issue(p0 + kWgPix);
#pragma unroll
    for (int kk = 0; kk < kWgPix; kk += 32) {
      bf16x8 a[2], bb[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) a[m] = load8(&As[16 * m + lr][kk + 8 * kq]);
#pragma unroll
      for (int f = 0; f < 2; ++f) bb[f] = load8(&Bs[32 * wv + 16 * f + lr][kk + 8 * kq]);
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int f = 0; f < 2; ++f)
          acc[m][f] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[m], bb[f], acc[m][f], 0, 0, 0);
    }
  }
  // lane holds D[o = 4 kq + r][k = lr] of every fragment
  float* dst = part + (int64_t)blockIdx.z * Cout * K;
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int k = k0 + 32 * wv + 16 * f + lr;
      if (k >= K) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int o = o0 + 16 * m + 4 * kq + r;
        dst[(int64_t)o * K + k] = acc[m][f][r];
      }
    }
}

// dst[i] += sum over z = 0..parts-1 of part[z][i] in a fixed order: a
// block takes 64 consecutive elements (one per lane, so every load is 256
// contiguous bytes); wavefront g sums the shares z = g, g+4, g+8, ... in
// increasing z, and the four partial sums are added in g order.
__global__ __launch_bounds__(256) void k_sum_parts(const float* __restrict__ part, int64_t n, int parts,
                                                   float* __restrict__ dst) {
  __shared__ float red[4][64];
  const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  float s = 0.f;
  if (i < n)
    for (int z = g; z < parts; z += 4) s += part[(int64_t)z * n + i];
  red[g][lane] = s;
  __syncthreads();
  if (g == 0 && i < n) dst[i] += ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// dst[0] += sum over z of part[z] (FP64), fixed order: strided sums per
// thread, then a fixed tree (one block).
__global__ __launch_bounds__(256) void k_sum_parts_f64(const double* __restrict__ part, int parts,
                                                       double* __restrict__ dst) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int z = t; z < parts; z += 256) s += part[z];
  red[t] = s;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if (t < d) red[t] += red[t + d];
    __syncthreads();
  }
  if (t == 0) dst[0] += red[0];
}

// ---------------------------------------------------------------------------
// element-wise and reshaping kernels (8 channels per thread)

__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) y[i] = f2bf(x[i]);
}

// gm = g where act > 0, else 0 (ReLU backward; act is the stored output),
// rounded once to bfloat16 for the matrix-core products that consume it
__global__ __launch_bounds__(256) void k_relu_mask(const float* __restrict__ g, const uint16_t* __restrict__ act,
                                                   uint16_t* __restrict__ gm, int64_t n8) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n8) return;
  const f32x4 g0 = *(const f32x4*)(g + 8 * i), g1 = *(const f32x4*)(g + 8 * i + 4);
  const u16x8 av = *(const u16x8*)(act + 8 * i);
  u16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const float v = e < 4 ? g0[e] : g1[e - 4];
    o[e] = bf2f(av[e]) > 0.f ? f2bf(v) : (uint16_t)0;
  }
  *(u16x8*)(gm + 8 * i) = o;
}

// 2x2 average pooling, [B][H][W][C] -> [B][H/2][W/2][C]
__global__ __launch_bounds__(256) void k_pool(const uint16_t* __restrict__ x, uint16_t* __restrict__ y, int Bn, int H,
                                              int W, int C) {
  const int C8 = C / 8, Ho = H / 2, Wo = W / 2;
  const int64_t n = (int64_t)Bn * Ho * Wo * C8;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c8 = (int)(i % C8);
  int64_t r = i / C8;
  const int xo = (int)(r % Wo);
  r /= Wo;
  const int yo = (int)(r % Ho);
  const int64_t b = r / Ho;
  const uint16_t* s = x + (((b * H + 2 * yo) * W + 2 * xo) * C + 8 * c8);
  const u16x8 a0 = *(const u16x8*)s, a1 = *(const u16x8*)(s + C), a2 = *(const u16x8*)(s + (int64_t)W * C),
              a3 = *(const u16x8*)(s + (int64_t)W * C + C);
  u16x8 o;
#pragma unroll
  for (int e = 0; e < 8; ++e) o[e] = f2bf(0.25f * (bf2f(a0[e]) + bf2f(a1[e]) + bf2f(a2[e]) + bf2f(a3[e])));
  *(u16x8*)(y + i * 8) = o;
}

// cat[b][y][x] = (deep[b][y/2][x/2][0:Cd], skip[b][y][x][0:Cs])
__global__ __launch_bounds__(256) void k_upcat(const uint16_t* __restrict__ deep, int Cd, const uint16_t* __restrict__ skip,
                                               int Cs, uint16_t* __restrict__ cat, int Bn, int H, int W) {
  const int C8 = (Cd + Cs) / 8;
  const int64_t n = (int64_t)Bn * H * W * C8;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C8) * 8;
  const int64_t p = i / C8;
  const int x = (int)(p % W);
  const int64_t r = p / W;
  const int y = (int)(r % H);
  const int64_t b = r / H;
  u16x8 v;
  if (c < Cd) v = *(const u16x8*)(deep + ((b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cd + c);
  else v = *(const u16x8*)(skip + p * Cs + (c - Cd));
  *(u16x8*)(cat + p * (Cd + Cs) + c) = v;
}

// gdeep[b][y][x][c] = sum over the 2x2 children of gcat[..][c], c < Cd (float32)
__global__ __launch_bounds__(256) void k_up_grad(const float* __restrict__ gcat, int Ccat, int Cd,
                                                 float* __restrict__ gdeep, int Bn, int Ho, int Wo) {
  const int C8 = Cd / 8;
  const int64_t n = (int64_t)Bn * Ho * Wo * C8;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C8) * 8;
  int64_t r = i / C8;
  const int xo = (int)(r % Wo);
  r /= Wo;
  const int yo = (int)(r % Ho);
  const int64_t b = r / Ho;
  const int W = 2 * Wo, H = 2 * Ho;
  const int64_t p = (b * H + 2 * yo) * W + 2 * xo;
  const float* s = gcat + p * Ccat + c;
  const int64_t dn = (int64_t)W * Ccat;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const f32x4 a0 = *(const f32x4*)(s + 4 * h), a1 = *(const f32x4*)(s + Ccat + 4 * h),
                a2 = *(const f32x4*)(s + dn + 4 * h), a3 = *(const f32x4*)(s + dn + Ccat + 4 * h);
    *(f32x4*)(gdeep + i * 8 + 4 * h) = (a0 + a1) + (a2 + a3);
  }
}

// gskip[b][y][x][c] = gcat[b][y][x][Cd + c] (if gcat) + gpool[b][y/2][x/2][c] / 4 (if gpool), float32
__global__ __launch_bounds__(256) void k_skip_grad(const float* __restrict__ gcat, int Ccat, int Cd,
                                                   const float* __restrict__ gpool, float* __restrict__ gskip,
                                                   int Cs, int Bn, int H, int W) {
  const int C8 = Cs / 8;
  const int64_t n = (int64_t)Bn * H * W * C8;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int c = (int)(i % C8) * 8;
  const int64_t p = i / C8;
  const int x = (int)(p % W);
  const int64_t r = p / W;
  const int y = (int)(r % H);
  const int64_t b = r / H;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
    if (gcat) v += *(const f32x4*)(gcat + p * Ccat + Cd + c + 4 * h);
    if (gpool) v += 0.25f * *(const f32x4*)(gpool + ((b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cs + c + 4 * h);
    *(f32x4*)(gskip + p * Cs + c + 4 * h) = v;
  }
}

// bias gradient: block b stores sum over its pixels of the ReLU-masked
// float32 gradient (g[p][c] where act[p][c] > 0) in part[b][c] (summed
// into db by k_sum_parts).  It sums the float32 gradient, not its bfloat16
// copy: a bias gradient is a sum over every pixel with much cancellation.
__global__ __launch_bounds__(256) void k_bias_grad(const float* __restrict__ g, const uint16_t* __restrict__ actv,
                                                   int C, int64_t P, int64_t px_per_block, float* __restrict__ part) {
  __shared__ float red[256];
  const int t = threadIdx.x;
  const int lanes_per_px = C < 256 ? C : 256;   // C is 32, 64, 128 or a multiple of 256
  const int rows = 256 / lanes_per_px;
  const int64_t pbeg = (int64_t)blockIdx.x * px_per_block;
  const int64_t pend = pbeg + px_per_block < P ? pbeg + px_per_block : P;
  for (int cbase = 0; cbase < C; cbase += lanes_per_px) {
    const int c = cbase + t % lanes_per_px, row = t / lanes_per_px;
    const bool act = row < rows && c < C;
    // four independent running sums (their loads in flight together),
    // combined in a fixed order
    float s4[4] = {0.f, 0.f, 0.f, 0.f};
    if (act) {
      int64_t p = pbeg + row;
      for (; p + 3 * rows < pend; p += 4 * rows) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int64_t q = p + u * rows;
          s4[u] += bf2f(actv[q * C + c]) > 0.f ? g[q * C + c] : 0.f;
        }
      }
      for (; p < pend; p += rows) s4[0] += bf2f(actv[p * C + c]) > 0.f ? g[p * C + c] : 0.f;
    }
    float s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    red[t] = s;
    __syncthreads();
    if (row == 0 && act) {
      for (int r = 1; r < rows; ++r) s += red[r * lanes_per_px + t];
      part[(int64_t)blockIdx.x * C + c] = s;
    }
    __syncthreads();
  }
}

// Head: out[p][j] = scale * (b[j] + sum_c w[j][c] x[p][c]) (+ gain *
// resid[p][1 + j] when a residual input is given), j = 0, 1 (float32 out).
__global__ __launch_bounds__(256) void k_head_fwd(const uint16_t* __restrict__ x, int C, const float* __restrict__ w,
                                                  const float* __restrict__ b, float scale,
                                                  const float* __restrict__ resid, int rc, float gain,
                                                  float* __restrict__ out, int64_t P) {
  const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  float s0 = 0.f, s1 = 0.f;
  for (int c = 0; c < C; c += 8) {
    const u16x8 a = *(const u16x8*)(x + p * C + c);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float v = bf2f(a[e]);
      s0 += w[c + e] * v;
      s1 += w[C + c + e] * v;
    }
  }
  float r0 = 0.f, r1 = 0.f;
  if (resid) {
    r0 = gain * resid[p * rc + 1];
    r1 = gain * resid[p * rc + 2];
  }
  out[2 * p] = scale * (b[0] + s0) + r0;
  out[2 * p + 1] = scale * (b[1] + s1) + r1;
}

// Mean squared error of the head output against the target field, and the
// head's backward: gx[p][c] = sum_j go[p][j] w[j][c] (bfloat16),
// dw[j][c] += sum_p go[p][j] x[p][c], db[j] += sum_p go[p][j],
// go = scale * 2 (out - target) / (2 P).  loss[0] += sum (out - target)^2 / (2 P).
// Block b stores its shares in part[b] = (dw [2][C], db [2]) and lpart[b]
// (the loss), summed by k_sum_parts / k_sum_parts_f64 in a fixed order.
__global__ __launch_bounds__(256) void k_head_bwd(const uint16_t* __restrict__ x, int C, const float* __restrict__ w,
                                                  float scale, const float* __restrict__ out,
                                                  const float* __restrict__ target, int64_t P,
                                                  float* __restrict__ gx, float* __restrict__ hpart,
                                                  double* __restrict__ lpart) {
  float* dw = hpart + (int64_t)blockIdx.x * (2 * C + 2);
  __shared__ float part[2][4][8];     // per-wave partial dw, 8 channels at a time
  __shared__ double lred[256];
  __shared__ float bred[2][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t p = (int64_t)blockIdx.x * 256 + t;
  const bool ok = p < P;
  const double inv = 1.0 / (2.0 * (double)P);
  float g0 = 0.f, g1 = 0.f;
  double l = 0.0;
  if (ok) {
    const float e0 = out[2 * p] - target[2 * p], e1 = out[2 * p + 1] - target[2 * p + 1];
    l = ((double)e0 * e0 + (double)e1 * e1) * inv;
    g0 = (float)(2.0 * inv) * e0 * scale;
    g1 = (float)(2.0 * inv) * e1 * scale;
  }
  lred[t] = l;
  bred[0][t] = g0;
  bred[1][t] = g1;
  for (int c = 0; c < C; c += 8) {
    u16x8 a;
    if (ok) a = *(const u16x8*)(x + p * C + c);
    else a = u16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (ok) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        f32x4 o;
#pragma unroll
        for (int e = 0; e < 4; ++e) o[e] = g0 * w[c + 4 * h + e] + g1 * w[C + c + 4 * h + e];
        *(f32x4*)(gx + p * C + c + 4 * h) = o;
      }
    }
    // dw partials: reduce over the block's pixels, 8 channels at a time
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float v = bf2f(a[e]);
      float s0 = g0 * v, s1 = g1 * v;
      for (int d = 32; d >= 1; d >>= 1) {
        s0 += __shfl_xor(s0, d, 64);
        s1 += __shfl_xor(s1, d, 64);
      }
      if (lane == 0) {
        part[0][wv][e] = s0;
        part[1][wv][e] = s1;
      }
    }
    __syncthreads();
    if (t < 16) {
      const int j = t >> 3, e = t & 7;
      float s = 0.f;
      for (int q = 0; q < 4; ++q) s += part[j][q][e];
      dw[j * C + c + e] = s;
    }
    __syncthreads();
  }
  for (int d = 128; d >= 1; d >>= 1) {
    if (t < d) {
      lred[t] += lred[t + d];
      bred[0][t] += bred[0][t + d];
      bred[1][t] += bred[1][t + d];
    }
    __syncthreads();
  }
  if (t == 0) {
    lpart[blockIdx.x] = lred[0];
    dw[2 * C] = bred[0][0];
    dw[2 * C + 1] = bred[1][0];
  }
}

// Adam with bias correction (Kingma and Ba): m, v float32.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bfloat16 copies of one conv layer's float32 weights W[o][k] (k = tap C_in + c):
// wA = W as is, wT[c][tap' C_out + o] = W[o][(8 - tap') C_in + c].
__global__ __launch_bounds__(256) void k_pack_w(const float* __restrict__ w, int Cin, int Cout,
                                                uint16_t* __restrict__ wA, uint16_t* __restrict__ wT) {
  const int64_t n = (int64_t)Cout * 9 * Cin;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int K = 9 * Cin;
  const int o = (int)(i / K), k = (int)(i - (int64_t)o * K);
  const int tap = k / Cin, c = k - tap * Cin;
  const uint16_t v = f2bf(w[i]);
  wA[i] = v;
  if (wT) wT[(int64_t)c * 9 * Cout + (8 - tap) * Cout + o] = v;
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ x, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = v;
}

// ---------------------------------------------------------------------------
// host launchers

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

bool conv3_supported(int Cin, int Cout) { return Cout % 32 == 0 && Cin >= 1; }

// deep != nullptr (the concatenation read in place) only where
// conv3_rows_ok holds and Cd % 32 == 0 (checked by the caller)
template <bool F32OUT>
static void conv3_t(const uint16_t* in, int Cin, const uint16_t* wA, const float* bias, void* out, int Cout, int Bn,
                    int H, int W, int relu, hipStream_t s, const uint16_t* deep = nullptr, int Cd = 0) {
  const int64_t P = (int64_t)Bn * H * W;
  const unsigned gx = (unsigned)((P + 255) / 256);
  const bool gen = Cin % 32 != 0;
  if (conv3_rows_ok(Cin, P, H, W)) {   // whole rows per block: P is a multiple of 256
    if (Cout % 64 == 0)
      hipLaunchKernelGGL((k_conv3_rows<4, F32OUT>), dim3(gx, Cout / 64), dim3(256), 0, s, in, Cin, deep, Cd, wA, bias,
                         out, Cout, P, H, W, relu);
    else
      hipLaunchKernelGGL((k_conv3_rows<2, F32OUT>), dim3(gx, Cout / 32), dim3(256), 0, s, in, Cin, deep, Cd, wA, bias,
                         out, Cout, P, H, W, relu);
    return;
  }
  if (Cout % 64 == 0) {
    dim3 grid(gx, Cout / 64);
    if (gen) hipLaunchKernelGGL((k_conv3<4, true, F32OUT>), grid, dim3(256), 0, s, in, Cin, wA, bias, out, Cout, P, H, W, relu);
    else hipLaunchKernelGGL((k_conv3<4, false, F32OUT>), grid, dim3(256), 0, s, in, Cin, wA, bias, out, Cout, P, H, W, relu);
  } else {
    dim3 grid(gx, Cout / 32);
    if (gen) hipLaunchKernelGGL((k_conv3<2, true, F32OUT>), grid, dim3(256), 0, s, in, Cin, wA, bias, out, Cout, P, H, W, relu);
    else hipLaunchKernelGGL((k_conv3<2, false, F32OUT>), grid, dim3(256), 0, s, in, Cin, wA, bias, out, Cout, P, H, W, relu);
  }
}

void launch_conv3(const uint16_t* in, int Cin, const uint16_t* wA, const float* bias, uint16_t* out, int Cout,
                  int Bn, int H, int W, int relu, hipStream_t s) {
  conv3_t<false>(in, Cin, wA, bias, out, Cout, Bn, H, W, relu, s);
}
// conv over [up(deep), skip] without the concatenation in memory; false
// (nothing launched) where the row-staged convolution does not apply
bool launch_conv3_upcat(const uint16_t* deep, int Cd, const uint16_t* skip, int Cs, const uint16_t* wA,
                        const float* bias, uint16_t* out, int Cout, int Bn, int H, int W, int relu, hipStream_t s) {
  if (Cd % 32 != 0 || !conv3_rows_ok(Cd + Cs, (int64_t)Bn * H * W, H, W)) return false;
  conv3_t<false>(skip, Cd + Cs, wA, bias, out, Cout, Bn, H, W, relu, s, deep, Cd);
  return true;
}

void launch_conv3_f32(const uint16_t* in, int Cin, const uint16_t* wA, float* out, int Cout, int Bn, int H, int W,
                      hipStream_t s) {
  conv3_t<true>(in, Cin, wA, nullptr, out, Cout, Bn, H, W, 0, s);
}

// Pixel shares of the weight gradient: enough to give the GPU ~4096
// blocks, at least 256 pixels each.
int64_t wgrad_splits(int64_t P, int Cin, int Cout, int64_t* px_per_block) {
  const int K = 9 * Cin;
  const int64_t kt = (K + 127) / 128, ot = Cout / 32;
  // (at most 256 shares: their fixed-order sum stays short)
  int64_t splits = 4096 / (kt * ot);
  if (splits > 256) splits = 256;
  if (splits < 1) splits = 1;
  int64_t ppb = (P + splits - 1) / splits;
  if (ppb < 256) ppb = 256;
  ppb = (ppb + kWgPix - 1) / kWgPix * kWgPix;
  if (px_per_block) *px_per_block = ppb;
  return (P + ppb - 1) / ppb;
}

// part: float [wgrad_splits(...)][Cout][9 Cin] scratch
void launch_conv3_wgrad(const uint16_t* in, int Cin, const uint16_t* g, int Cout, float* dW, float* part, int Bn,
                        int H, int W, hipStream_t s) {
  const int64_t P = (int64_t)Bn * H * W;
  const int K = 9 * Cin;
  const unsigned kt = (unsigned)((K + 127) / 128), ot = (unsigned)(Cout / 32);
  int64_t ppb = 0;
  const int64_t splits = wgrad_splits(P, Cin, Cout, &ppb);
  dim3 grid(kt, ot, (unsigned)splits);
  if (Cin % 8 == 0)
    hipLaunchKernelGGL((k_conv3_wgrad<false>), grid, dim3(256), 0, s, in, Cin, g, Cout, part, P, H, W, ppb);
  else
    hipLaunchKernelGGL((k_conv3_wgrad<true>), grid, dim3(256), 0, s, in, Cin, g, Cout, part, P, H, W, ppb);
  const int64_t n = (int64_t)Cout * K;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, part, n, (int)splits, dW);
}

void launch_to_bf16(const float* x, uint16_t* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nblk(n)), dim3(256), 0, s, x, y, n);
}
void launch_relu_mask(const float* g, const uint16_t* act, uint16_t* gm, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_relu_mask, dim3(nblk(n / 8)), dim3(256), 0, s, g, act, gm, n / 8);
}
void launch_pool(const uint16_t* x, uint16_t* y, int Bn, int H, int W, int C, hipStream_t s) {
  hipLaunchKernelGGL(k_pool, dim3(nblk((int64_t)Bn * (H / 2) * (W / 2) * (C / 8))), dim3(256), 0, s, x, y, Bn, H, W, C);
}
void launch_upcat(const uint16_t* deep, int Cd, const uint16_t* skip, int Cs, uint16_t* cat, int Bn, int H, int W,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_upcat, dim3(nblk((int64_t)Bn * H * W * ((Cd + Cs) / 8))), dim3(256), 0, s, deep, Cd, skip, Cs,
                     cat, Bn, H, W);
}
void launch_up_grad(const float* gcat, int Ccat, int Cd, float* gdeep, int Bn, int Ho, int Wo, hipStream_t s) {
  hipLaunchKernelGGL(k_up_grad, dim3(nblk((int64_t)Bn * Ho * Wo * (Cd / 8))), dim3(256), 0, s, gcat, Ccat, Cd, gdeep,
                     Bn, Ho, Wo);
}
void launch_skip_grad(const float* gcat, int Ccat, int Cd, const float* gpool, float* gskip, int Cs, int Bn,
                      int H, int W, hipStream_t s) {
  hipLaunchKernelGGL(k_skip_grad, dim3(nblk((int64_t)Bn * H * W * (Cs / 8))), dim3(256), 0, s, gcat, Ccat, Cd, gpool,
                     gskip, Cs, Bn, H, W);
}
// Blocks of the bias gradient (at most 256, at least 64 pixels each).
int64_t bias_blocks(int64_t P, int64_t* px_per_block) {
  int64_t blocks = 512;
  int64_t ppb = (P + blocks - 1) / blocks;
  if (ppb < 64) ppb = 64;
  if (px_per_block) *px_per_block = ppb;
  return (P + ppb - 1) / ppb;
}

// g: float32 gradient of the layer's output, act: its stored activation;
// part: float [bias_blocks(P)][C] scratch
void launch_bias_grad(const float* g, const uint16_t* act, int C, int64_t P, float* db, float* part, hipStream_t s) {
  int64_t ppb = 0;
  const int64_t blocks = bias_blocks(P, &ppb);
  hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)blocks), dim3(256), 0, s, g, act, C, P, ppb, part);
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((C + 63) / 64)), dim3(256), 0, s, part, (int64_t)C, (int)blocks, db);
}
void launch_head_fwd(const uint16_t* x, int C, const float* w, const float* b, float scale, const float* resid,
                     int rc, float gain, float* out, int64_t P, hipStream_t s) {
  hipLaunchKernelGGL(k_head_fwd, dim3(nblk(P)), dim3(256), 0, s, x, C, w, b, scale, resid, rc, gain, out, P);
}
// part: float [nblk(P)][2C + 2] and lpart: double [nblk(P)] scratch; dw
// and db are consecutive in the parameter layout (db = dw + 2C).
void launch_head_bwd(const uint16_t* x, int C, const float* w, float scale, const float* out, const float* target,
                     int64_t P, float* gx, float* dw, double* loss, float* part, double* lpart, hipStream_t s) {
  const unsigned blocks = nblk(P);
  hipLaunchKernelGGL(k_head_bwd, dim3(blocks), dim3(256), 0, s, x, C, w, scale, out, target, P, gx, part, lpart);
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)((2 * C + 2 + 63) / 64)), dim3(256), 0, s, part, (int64_t)(2 * C + 2),
                     (int)blocks, dw);
  if (loss) hipLaunchKernelGGL(k_sum_parts_f64, dim3(1), dim3(256), 0, s, lpart, (int)blocks, loss);
}
void launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}
void launch_pack_w(const float* w, int Cin, int Cout, uint16_t* wA, uint16_t* wT, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_w, dim3(nblk((int64_t)Cout * 9 * Cin)), dim3(256), 0, s, w, Cin, Cout, wA, wT);
}
void launch_fill_f32(float* x, int64_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_f32, dim3(nblk(n)), dim3(256), 0, s, x, n, v);
}

}  // namespace cgn
