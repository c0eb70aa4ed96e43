// Density, displacement, advection, areas and the stopping rule
// (paper: Method, Steps 1, 3, 5, 6, 7; Background, eqs.(2)-(3) and
// "Quality Measures").
#include "cg_dev.h"

namespace cgk {

// Step 3: density LUT.  d0 = sum s / sum o over map regions with o > 0,
// background density b*d0 (or from a prescribed background mass); the LUT is scaled so the texture mass is N^2
// (the map is invariant to a common scale of the density).
__global__ __launch_bounds__(256) void k_density(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_inst, KD_INST, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  __shared__ double red[256];
  const int t = threadIdx.x, R = I.R;
  auto count = [&](int v) -> double { return (double)I.counts[v]; };
  const double NN = (double)I.N * (double)I.N;
  const bool poly = I.area_source == CG_AREA_POLYGON;
  const double c0 = count(0);
  // one pass over the regions (every load of a region issued before any
  // is used; the thread's first region kept for the table): sum s, sum o
  // and sum s / o * count, whose total does not depend on d0
  double ss = 0.0, so = 0.0, cm = 0.0, q1 = 0.0;
  for (int v = 1 + t; v <= R; v += 256) {
    const double cnt = count(v);
    const double ar = I.areas[v];
    const double sv = (double)I.values[v - 1];
    const double o = poly ? ar * NN : cnt;
    const double q = o > 0.0 ? sv / o : 0.0;
    if (v == 1 + t) q1 = q;
    if (o > 0.0) {
      ss += sv;
      cm += q * cnt;
    }
    so += o;
  }
  ss = block_sum(ss, red);
  so = block_sum(so, red);
  const double d0 = so > 0.0 ? ss / so : 1.0;
  const double bdv = background_density(I, d0, c0);
  cm = block_sum(cm, red) + bdv * c0;
  const double kappa = cm > 0.0 ? NN / cm : 1.0;
  for (int v = 1 + t; v <= R; v += 256) {
    double q = q1;
    if (v != 1 + t) {
      const double o = poly ? I.areas[v] * NN : count(v);
      q = o > 0.0 ? (double)I.values[v - 1] / o : 0.0;
    }
    I.lut[v] = (float)(kappa * q);
  }
  for (int v = R + 1 + t; v < I.n_lut; v += 256) I.lut[v] = 0.f;
  if (t == 0) {
    I.lut[0] = (float)(kappa * bdv);
    I.st->d0 = d0;
    I.st->C = cm;
  }
}

// The anchor points of eq.(2) at (x, y).  Step 1's t(x, y; d0) for a
// constant density is in closed form (quadrant areas are products, wedge
// areas squares minus the parts the domain border cuts off) and enters
// node_disp below.
template <typename F>
__device__ __forceinline__ void anchors(F x, F y, F& q1x, F& q1y, F& q2x, F& q2y, F& q3x, F& q3y,
                                        F& q4x, F& q4y) {
  if (y < x) { q1x = 1; q1y = 1 + y - x; q3x = x - y; q3y = 0; }
  else { q1x = 1 - y + x; q1y = 1; q3x = 0; q3y = y - x; }
  if (x + y < 1) { q2x = x + y; q2y = 0; q4x = 0; q4y = x + y; }
  else { q2x = 1; q2y = x + y - 1; q4x = x + y - 1; q4y = 1; }
}

// Step 5 at one node (x, y) = (i, j) / N: D = t(.; d) - t(.; d0)
// (eqs.(2)-(3)) from the node's S and T, S at (i, N) and (N, j), the
// diagonal marginals HA[i + j] and HB[j - i + N], the total C and 1/(2C).
template <typename F>
__device__ __forceinline__ void node_disp(F x, F y, F s, F tt, F siN, F sNj, F ha, F hb, F C, F inv2C, F& dx,
                                          F& dy) {
  // eq.(2) for the density and for the constant density in one
  // combination: each coefficient is (integral / 2C) - (its constant-
  // density value / 2); the wedge areas need the squared positive parts
  // of z and -z for both diagonals: one max and one min each (one of the
  // two is zero)
  const F h = F(0.5);
  const F u = y - x, w = x + y - 1;
  const F up = fmax(u, F(0)), un = fmin(u, F(0)), wp = fmax(w, F(0)), wn = fmin(w, F(0));
  const F su = up * up, sv = un * un, sw = wp * wp, sz = wn * wn;   // wedges of y-x, x-y, x+y-1, 1-x-y
  const F a = s * inv2C - h * (x * y);
  const F b = (siN - s) * inv2C - h * (x * (1 - y));
  const F dl = (sNj - s) * inv2C - h * ((1 - x) * y);
  const F g = (C - siN - sNj + s) * inv2C - h * ((1 - x) * (1 - y));
  const F at = tt * inv2C - h * (y * y - h * su - h * sw);
  const F bt = (ha - tt) * inv2C - h * (x * x - h * sv - h * sw);
  const F gt = (C - ha - hb + tt) * inv2C - h * ((1 - y) * (1 - y) - h * sz - h * sv);
  const F dt = (hb - tt) * inv2C - h * ((1 - x) * (1 - x) - h * sz - h * su);
  F q1x, q1y, q2x, q2y, q3x, q3y, q4x, q4y;
  anchors(x, y, q1x, q1y, q2x, q2y, q3x, q3y, q4x, q4y);
  dx = a * q1x + b * q2x + g * q3x + dl * q4x + (at + gt) * x + bt;
  dy = a * q1y + b * q2y + g * q3y + dl * q4y + at + (bt + dt) * y;
}

// (S, T) of node (i, j): one load of the interleaved pair (ST = 2) or two.
template <typename F, int ST>
__device__ __forceinline__ void node_st(g_ptr<const F> S, g_ptr<const F> T, int64_t at, F& s, F& t) {
  if (ST == 2) {
    typedef F F2 __attribute__((ext_vector_type(2)));
    const F2 v = *(g_ptr<const F2>)(S + 2 * at);
    s = v[0];
    t = v[1];
  } else {
    s = S[at];
    t = T[at];
  }
}

// Step 6: bilinear interpolation of D at each point, clamp to [0,1]^2.
// The four corner nodes share their marginals: three consecutive HA and HB
// values, two values of row N and two of column N.
template <typename F, int ST>
__global__ __launch_bounds__(256) void k_map_points(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_pts, KD_PTS, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  const int64_t idx = (int64_t)(blockIdx.x - first) * 256 + threadIdx.x;
  if (idx >= I.n_pts) return;
  g_ptr<float2> ptr = idx < I.n_vert ? I.xy + idx : I.extra + (idx - I.n_vert);
  const float2 p = ld2(ptr);
  const int N = I.N;
  const F fN = F(N);
  const F u = fmin(fmax(F(p.x) * fN, F(0)), fN);
  const F v = fmin(fmax(F(p.y) * fN, F(0)), fN);
  const int i0 = min((int)floor(u), N - 1);
  const int j0 = min((int)floor(v), N - 1);
  const F fx = u - F(i0), fy = v - F(j0);
  g_ptr<const F> S = (g_ptr<const F>)I.S;
  g_ptr<const F> T = (g_ptr<const F>)I.T;
  g_ptr<const F> HA = (g_ptr<const F>)I.HA;
  g_ptr<const F> HB = (g_ptr<const F>)I.HB;
  const int64_t pitch = I.pitch;
  const F C = S[((int64_t)N * pitch + N) * ST];
  const F inv2C = F(1) / (F(2) * C), invN = F(1) / fN;
  const int64_t r0 = (int64_t)j0 * pitch + i0, r1 = r0 + pitch, rN = (int64_t)N * pitch + i0;
  F s00, t00, s10, t10, s01, t01, s11, t11;
  node_st<F, ST>(S, T, r0, s00, t00);
  node_st<F, ST>(S, T, r0 + 1, s10, t10);
  node_st<F, ST>(S, T, r1, s01, t01);
  node_st<F, ST>(S, T, r1 + 1, s11, t11);
  const F sN0 = S[rN * ST], sN1 = S[(rN + 1) * ST];                                   // (i0, N), (i0+1, N)
  const F s0N = S[((int64_t)j0 * pitch + N) * ST], s1N = S[((int64_t)(j0 + 1) * pitch + N) * ST];   // (N, j0), (N, j0+1)
  const int ia = i0 + j0, ib = j0 - i0 + N;
  const F ha0 = HA[ia], ha1 = HA[ia + 1], ha2 = HA[ia + 2];
  const F hb0 = HB[ib - 1], hb1 = HB[ib], hb2 = HB[ib + 1];
  const F x0 = F(i0) * invN, x1 = F(i0 + 1) * invN, y0 = F(j0) * invN, y1 = F(j0 + 1) * invN;
  F d00x, d00y, d10x, d10y, d01x, d01y, d11x, d11y;
  node_disp<F>(x0, y0, s00, t00, sN0, s0N, ha0, hb1, C, inv2C, d00x, d00y);
  node_disp<F>(x1, y0, s10, t10, sN1, s0N, ha1, hb0, C, inv2C, d10x, d10y);
  node_disp<F>(x0, y1, s01, t01, sN0, s1N, ha1, hb2, C, inv2C, d01x, d01y);
  node_disp<F>(x1, y1, s11, t11, sN1, s1N, ha2, hb1, C, inv2C, d11x, d11y);
  const F w00 = (1 - fx) * (1 - fy), w10 = fx * (1 - fy), w01 = (1 - fx) * fy, w11 = fx * fy;
  const F dx = w00 * d00x + w10 * d10x + w01 * d01x + w11 * d11x;
  const F dy = w00 * d00y + w10 * d10y + w01 * d01y + w11 * d11y;
  float2 o;
  o.x = (float)fmin(fmax(F(p.x) + dx, F(0)), F(1));
  o.y = (float)fmin(fmax(F(p.y) + dy, F(0)), F(1));
  st2(ptr, o);
}

// Warm start: move every point by alpha times a displacement field given
// at the pixel centres of a G x G grid ([G][G][2], centre (i + 1/2, j +
// 1/2) / G), interpolated bilinearly (constant beyond the outermost
// centres), then clamp to the unit square.  alpha < 0: the instance's
// chosen step (IterState::ws_alpha; 0 = no move).
__global__ __launch_bounds__(256) void k_apply_field(Batch B, float alpha) {
  int64_t first;
  const int k = find_inst(B, B.off_pts, KD_PTS, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (I.init_field == nullptr) return;
  const int64_t idx = (int64_t)(blockIdx.x - first) * 256 + threadIdx.x;
  if (idx >= I.n_pts) return;
  const float a = alpha < 0.f ? I.st->ws_alpha : alpha;
  if (a == 0.f) return;
  g_ptr<float2> ptr = idx < I.n_vert ? I.xy + idx : I.extra + (idx - I.n_vert);
  const float2 p = ld2(ptr);
  const int G = (int)I.init_G;
  g_ptr<const float2> F = (g_ptr<const float2>)I.init_field;
  float dx, dy;
  if (G == 1) {
    const float2 f0 = ld2(F);
    dx = f0.x;
    dy = f0.y;
  } else {
    const float u = fminf(fmaxf(p.x * G - 0.5f, 0.f), (float)(G - 1));
    const float v = fminf(fmaxf(p.y * G - 0.5f, 0.f), (float)(G - 1));
    const int i0 = min((int)floorf(u), G - 2), j0 = min((int)floorf(v), G - 2);
    const float fx = u - i0, fy = v - j0;
    const float2 a = ld2(F + (int64_t)j0 * G + i0), b = ld2(F + (int64_t)j0 * G + i0 + 1);
    const float2 c = ld2(F + (int64_t)(j0 + 1) * G + i0), d = ld2(F + (int64_t)(j0 + 1) * G + i0 + 1);
    const float w00 = (1 - fx) * (1 - fy), w10 = fx * (1 - fy), w01 = (1 - fx) * fy, w11 = fx * fy;
    dx = w00 * a.x + w10 * b.x + w01 * c.x + w11 * d.x;
    dy = w00 * a.y + w10 * b.y + w01 * c.y + w11 * d.y;
  }
  st2(ptr, make_float2(fminf(fmaxf(p.x + a * dx, 0.f), 1.f), fminf(fmaxf(p.y + a * dy, 0.f), 1.f)));
}

// Warm start: put the starting positions back (before the next trial step).
__global__ __launch_bounds__(256) void k_restore(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_pts, KD_PTS, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (I.init_field == nullptr) return;
  const int64_t idx = (int64_t)(blockIdx.x - first) * 256 + threadIdx.x;
  if (idx >= I.n_pts) return;
  if (idx < I.n_vert) {
    if (I.src_xy && I.src_xy != I.xy) st2(I.xy + idx, ld2(I.src_xy + idx));
  } else {
    const int64_t e = idx - I.n_vert;
    if (I.src_extra && I.src_extra != I.extra) st2(I.extra + e, ld2(I.src_extra + e));
  }
}

// Per-region log-density table of Step 3 from the pixel counts: lut[v] =
// log(d(v) / mean d), d(v) = s(v)/o(v), d(0) = shape * d0 (one block).
__global__ __launch_bounds__(256) void k_log_lut(const int64_t* counts, const float* values, int R, int N, float shape,
                                                 float* lut) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double ss = 0.0, so = 0.0;
  for (int v = 1 + t; v <= R; v += 256) {
    const int64_t o = counts[v];
    if (o > 0) {
      ss += (double)values[v - 1];
      so += (double)o;
    }
  }
  ss = block_sum(ss, red);
  so = block_sum(so, red);
  const double d0 = so > 0.0 ? ss / so : 1.0;
  const double bdv = (double)shape * d0;
  const double C = ss + bdv * (double)counts[0];
  const double mean = C / ((double)N * (double)N);
  const double tiny = 1e-30;
  for (int v = t; v <= R; v += 256) {
    double d;
    if (v == 0) d = bdv;
    else d = counts[v] > 0 ? (double)values[v - 1] / (double)counts[v] : 0.0;
    lut[v] = (float)log(fmax(d, tiny) / fmax(mean, tiny));
  }
}

__global__ __launch_bounds__(256) void k_log_density(const uint16_t* labels, const float* lut, int R, int64_t n,
                                                     float* out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int v = labels[i];
  out[i] = v <= R ? lut[v] : lut[0];
}

// Box average of a [G][G][2] field over f x f cells -> [G/f][G/f][2].
__global__ __launch_bounds__(256) void k_field_pool(int G, int f, const float2* in, float2* out) {
  const int g = G / f;
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)g * g) return;
  const int j = (int)(idx / g), i = (int)(idx - (int64_t)j * g);
  float sx = 0.f, sy = 0.f;
  for (int b = 0; b < f; ++b)
    for (int a = 0; a < f; ++a) {
      const float2 v = in[(int64_t)(j * f + b) * G + i * f + a];
      sx += v.x;
      sy += v.y;
    }
  const float w = 1.f / (float)(f * f);
  out[idx] = make_float2(sx * w, sy * w);
}

// Pixel-centre tracer grid, or the displacement of moved tracers from it.
__global__ __launch_bounds__(256) void k_tracer_field(int G, const float2* fin, float2* out) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= (int64_t)G * G) return;
  const int j = (int)(idx / G), i = (int)(idx - (int64_t)j * G);
  const float cx = ((float)i + 0.5f) / (float)G, cy = ((float)j + 0.5f) / (float)G;
  if (fin) out[idx] = make_float2(fin[idx].x - cx, fin[idx].y - cy);
  else out[idx] = make_float2(cx, cy);
}

// Shoelace area of every region (sum over its rings), FP64, fixed order.
__global__ __launch_bounds__(256) void k_areas(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_regions, KD_REGIONS, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  __shared__ double red[256];
  region_area(I, 1 + (int)(blockIdx.x - first), red);
}

// Cartographic errors and the stopping rule (Method, end of the static
// construction).  mode 0: update the iteration state; mode 1: evaluate
// only (eps, xi into the state, nothing else touched); modes 2-4 judge a
// warm start (instances with a field): 2 keeps xi as the error of the plain
// start, 3 records a trial step `alpha` if it is the best so far, 4 flags
// CG_FLAG_FALLBACK when no trial step beat the plain start.
__global__ __launch_bounds__(256) void k_err(Batch B, int mode, float alpha) {
  int64_t first;
  const int k = find_inst(B, B.off_inst, KD_INST, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  __shared__ double red[256];
  (void)stopping_rule(I, mode, alpha, red);
}

// Reset the iteration state and copy the starting positions.
__global__ __launch_bounds__(256) void k_init(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_pts, KD_PTS, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  const int64_t idx = (int64_t)(blockIdx.x - first) * 256 + threadIdx.x;
  if (idx == 0) {
    IterState z = {};
    z.best_xi = 1e300;
    static_assert(sizeof(IterState) % 4 == 0, "state is copied as 32-bit words");
    const uint32_t* src = (const uint32_t*)&z;
    g_ptr<uint32_t> dst = (g_ptr<uint32_t>)I.st;
    for (int w = 0; w < (int)(sizeof(IterState) / 4); ++w) dst[w] = src[w];
  }
  // the row counters are accumulated with atomics and cleared by their
  // consumers; scratch memory starts with arbitrary contents
  if (I.row_cnt) {
    const int64_t nth = (B.off_pts[k + 1] - first) * 256;
    for (int64_t q = idx; q < I.N; q += nth) I.row_cnt[q] = 0u;
  }
  if (idx >= I.n_pts) return;
  if (idx < I.n_vert) {
    if (I.src_xy && I.src_xy != I.xy) st2(I.xy + idx, ld2(I.src_xy + idx));
  } else {
    const int64_t e = idx - I.n_vert;
    if (I.src_extra && I.src_extra != I.extra) st2(I.extra + e, ld2(I.src_extra + e));
  }
}

__global__ __launch_bounds__(256) void k_export(Batch B, int64_t* contested, double* eps_xi) {
  const IterState* st = B.inst[0].st;
  if (threadIdx.x == 0) {
    if (contested) *contested = st->contested;
    if (eps_xi) {
      eps_xi[0] = st->eps;
      eps_xi[1] = st->xi;
    }
  }
}

// Transition frames: f = a + (k/K)(b - a), k = 1..K-1, for n points.
__global__ __launch_bounds__(256) void k_frames(const float2* a, const float2* b, float2* out, int64_t n, int K) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx >= n) return;
  const float2 pa = a[idx], pb = b[idx];
  for (int kk = 1; kk < K; ++kk) {
    const float w = (float)kk / (float)K;
    out[(int64_t)(kk - 1) * n + idx] = make_float2(pa.x + w * (pb.x - pa.x), pa.y + w * (pb.y - pa.y));
  }
}

// host launchers --------------------------------------------------------------

void launch_density(const Batch& B, hipStream_t s) {
  hipLaunchKernelGGL(k_density, dim3(B.n), dim3(256), 0, s, B);
}
void launch_map(const Batch& B, int prec, bool il, int64_t pt_blocks, hipStream_t s) {
  if (pt_blocks <= 0) return;
  if (prec == CG_F64) {
    if (il) hipLaunchKernelGGL((k_map_points<double, 2>), dim3(pt_blocks), dim3(256), 0, s, B);
    else hipLaunchKernelGGL((k_map_points<double, 1>), dim3(pt_blocks), dim3(256), 0, s, B);
  } else {
    if (il) hipLaunchKernelGGL((k_map_points<float, 2>), dim3(pt_blocks), dim3(256), 0, s, B);
    else hipLaunchKernelGGL((k_map_points<float, 1>), dim3(pt_blocks), dim3(256), 0, s, B);
  }
}
void launch_apply_field(const Batch& B, int64_t pt_blocks, float alpha, hipStream_t s) {
  if (pt_blocks > 0) hipLaunchKernelGGL(k_apply_field, dim3(pt_blocks), dim3(256), 0, s, B, alpha);
}
void launch_restore(const Batch& B, int64_t pt_blocks, hipStream_t s) {
  if (pt_blocks > 0) hipLaunchKernelGGL(k_restore, dim3(pt_blocks), dim3(256), 0, s, B);
}
void launch_log_density(const uint16_t* labels, const int64_t* counts, const float* values, int R, int N, float shape,
                        float* lut, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_log_lut, dim3(1), dim3(256), 0, s, counts, values, R, N, shape, lut);
  const int64_t n = (int64_t)N * N;
  hipLaunchKernelGGL(k_log_density, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, labels, lut, R, n, out);
}
void launch_field_pool(int G, int f, const float* in, float* out, hipStream_t s) {
  const int64_t n = (int64_t)(G / f) * (G / f);
  hipLaunchKernelGGL(k_field_pool, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, f, (const float2*)in,
                     (float2*)out);
}
void launch_tracer_field(int G, const float* fin, float* out, hipStream_t s) {
  const int64_t n = (int64_t)G * G;
  hipLaunchKernelGGL(k_tracer_field, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, G, (const float2*)fin,
                     (float2*)out);
}
void launch_areas(const Batch& B, int64_t region_blocks, hipStream_t s) {
  if (region_blocks > 0) hipLaunchKernelGGL(k_areas, dim3(region_blocks), dim3(256), 0, s, B);
}
void launch_err(const Batch& B, int mode, hipStream_t s, float alpha) {
  hipLaunchKernelGGL(k_err, dim3(B.n), dim3(256), 0, s, B, mode, alpha);
}
void launch_init(const Batch& B, int64_t pt_blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_init, dim3(pt_blocks), dim3(256), 0, s, B);
}
void launch_export(const Batch& B, int64_t* contested, double* eps_xi, hipStream_t s) {
  hipLaunchKernelGGL(k_export, dim3(1), dim3(64), 0, s, B, contested, eps_xi);
}
void launch_frames(const float* a, const float* b, float* out, int64_t n, int K, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  if (blocks > 0 && K > 1)
    hipLaunchKernelGGL(k_frames, dim3(blocks), dim3(256), 0, s, (const float2*)a, (const float2*)b,
                       (float2*)out, n, K);
}

}  // namespace cgk
