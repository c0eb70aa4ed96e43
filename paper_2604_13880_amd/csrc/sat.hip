// Node integral images of the density texture (paper: Background,
// "Integral Images", eq.(1); Method, Step 4).
//
// With R(x, q) the integral of row q over [0, x] and M(x, q) the integral up
// to the centre of pixel x (M = R + d/2), the tables are
//   S(i, j)  = sum_{q<j} R(i, q)                       (axis-aligned)
//   TA(u, j) = sum_{q<j} M(u - q, q)                   (anti-diagonal)
//   TB(v, j) = sum_{q<j} M(v + q, q)                   (diagonal)
//   T(i, j)  = TA(i+j-1, j) - TB(i-j, j)                (top wedge of node (i,j))
//   HA(s)    = TA(s-1, N),  HB(r) = C - TB(-r, N)       (diagonal marginals)
// because the top wedge cuts every row q < j in the interval
// [i - (j - y'), i + (j - y')] whose row integral averages to the two M
// values at its ends; a pixel bisected by a wedge side contributes half.
//
// Three passes over tiles of TW columns x TH rows (one block of TW threads
// per tile), reduce-then-scan:
//   k_sat_reduce  per tile: row totals, column prefix sums, cumulative
//                 masses along anti-diagonals and diagonals
//   k_sat_carry1  row carries across tile columns, tile-row prefix totals
//   k_sat_carry2  carries entering every tile row for S, TA, TB; HA, HB
//   k_sat_final   per tile with a TH-column halo on each side: row prefix
//                 sums staged in LDS, then a sweep down the tile's rows
//                 that accumulates S, TA, TB in registers and writes one
//                 row of S and T per step (coalesced stores)
// Accumulation precision: float, compensated float or double (PT<P>).
#include "cg_dev.h"

namespace cgk {

template <bool DENSE>
__device__ __forceinline__ float dens_at(const Inst& I, const float* lut_s, bool lut_lds, int p, int q) {
  const int N = I.N;
  if (p < 0 || p >= N || q < 0 || q >= N) return 0.f;
  if (DENSE) return I.density[(int64_t)q * N + p];
  const int lab = I.labels[(int64_t)q * N + p];
  if (lab >= I.n_lut) return 0.f;  // labels outside the LUT carry no mass
  return lut_lds ? lut_s[lab] : I.lut[lab];
}

template <typename A>
__device__ __forceinline__ A mid(const A& a, const A& b) {
  A s = a;
  acc_addv(s, b);
  return acc_half(s);
}

template <int P, int TW, int TH, bool DENSE>
__global__ __launch_bounds__(TW) void k_sat_reduce(Batch B) {
  typedef typename PT<P>::acc A;
  typedef typename PT<P>::carry Cy;
  const int64_t nb = B.off_tiles[B.n];
  const int64_t b = xcd_block(blockIdx.x, nb);
  const int k = find_inst(B.off_tiles, B.n, b);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  constexpr int NW = TW / 64, E = TW / 64, D = TW + TH - 1;
  __shared__ A Rs[TH][TW + 1];
  __shared__ float lut_s[kLutLds];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const SatLayout L = sat_layout(I.N, TW, TH);
  const int tile = (int)(b - B.off_tiles[k]);
  const int tx = tile % L.ntx, ty = tile / L.ntx;
  const int x0 = tx * TW, y0 = ty * TH;
  const bool lut_lds = !DENSE && I.n_lut <= kLutLds;
  if (lut_lds)
    for (int v = t; v < I.n_lut; v += TW) lut_s[v] = I.lut[v];
  __syncthreads();
  for (int r = w; r < TH; r += NW) {
    const int q = y0 + r;
    float dv[E];
    A loc;
    acc_zero(loc);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      dv[e] = dens_at<DENSE>(I, lut_s, lut_lds, x0 + lane * E + e, q);
      acc_add(loc, dv[e]);
    }
    A run = wave_exclusive_scan(loc, lane);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      Rs[r][lane * E + e] = run;
      acc_add(run, dv[e]);
    }
    if (lane == 63) Rs[r][TW] = run;
  }
  __syncthreads();
  Cy* agg = (Cy*)I.agg;
  const int64_t tid = (int64_t)ty * L.ntx + tx;
  for (int r = t; r < TH; r += TW) agg[L.rowTot + (int64_t)tx * L.NY + y0 + r] = to_carry(Rs[r][TW]);
  {
    A s;
    acc_zero(s);
    for (int r = 0; r < TH; ++r) acc_addv(s, Rs[r][t + 1]);
    agg[L.colsum + tid * (TW + 1) + t + 1] = to_carry(s);
    if (t == 0) agg[L.colsum + tid * (TW + 1)] = (Cy)0;
  }
  for (int c = t; c < D; c += TW) {
    A sa, sb;
    acc_zero(sa);
    acc_zero(sb);
    for (int r = 0; r < TH; ++r) {
      const int ca = c - r;                 // anti-diagonal u = x0+y0+c meets row y0+r at column x0+ca
      if (ca >= TW) acc_addv(sa, Rs[r][TW]);
      else if (ca >= 0) acc_addv(sa, mid(Rs[r][ca], Rs[r][ca + 1]));
      const int cb = c + r - TH + 1;        // diagonal v = x0-y0-TH+1+c meets it at column x0+cb
      if (cb >= TW) acc_addv(sb, Rs[r][TW]);
      else if (cb >= 0) acc_addv(sb, mid(Rs[r][cb], Rs[r][cb + 1]));
    }
    agg[L.cdfA + tid * D + c] = to_carry(sa);
    agg[L.cdfB + tid * D + c] = to_carry(sb);
  }
  if (t == 0) {
    A s;
    acc_zero(s);
    for (int r = 0; r < TH; ++r) acc_addv(s, Rs[r][TW]);
    agg[L.tileTot + tid] = to_carry(s);
  }
}

template <int P, int TW, int TH>
__global__ __launch_bounds__(256) void k_sat_carry1(Batch B) {
  typedef typename PT<P>::carry Cy;
  const int k = find_inst(B.off_carry1, B.n, blockIdx.x);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  const SatLayout L = sat_layout(I.N, TW, TH);
  const int64_t idx = (int64_t)(blockIdx.x - B.off_carry1[k]) * 256 + threadIdx.x;
  Cy* agg = (Cy*)I.agg;
  if (idx < L.NY) {
    const int q = (int)idx;
    Cy run = 0;
    for (int tx = 0; tx < L.ntx; ++tx) {
      const Cy v = agg[L.rowTot + (int64_t)tx * L.NY + q];
      agg[L.RC + (int64_t)tx * L.NY + q] = run;
      run += v;
    }
  } else if (idx < L.NY + L.nty) {
    const int ty = (int)(idx - L.NY);
    Cy run = 0;
    for (int tx = 0; tx < L.ntx; ++tx) {
      const Cy v = agg[L.tileTot + (int64_t)ty * L.ntx + tx];
      agg[L.prefTot + (int64_t)ty * (L.ntx + 1) + tx] = run;
      run += v;
    }
    agg[L.prefTot + (int64_t)ty * (L.ntx + 1) + L.ntx] = run;
  } else if (idx == L.NY + L.nty) {
    Cy C = 0;
    for (int ty = 0; ty < L.nty; ++ty) {
      Cy band = 0;
      for (int tx = 0; tx < L.ntx; ++tx) band += agg[L.tileTot + (int64_t)ty * L.ntx + tx];
      C += band;
    }
    agg[L.Cval] = C;
  }
}

template <int TW, int TH, typename Cy>
__device__ __forceinline__ Cy band_a(const Cy* agg, const SatLayout& L, int ty, int64_t u) {
  constexpr int D = TW + TH - 1;
  const int64_t y0 = (int64_t)ty * TH;
  int64_t klo = ceildiv(u - y0 - TW - TH + 2, TW);
  klo = klo < 0 ? 0 : (klo > L.ntx ? L.ntx : klo);
  int64_t khi = floordiv(u - y0, TW);
  if (khi > L.ntx - 1) khi = L.ntx - 1;
  Cy s = agg[L.prefTot + (int64_t)ty * (L.ntx + 1) + klo];
  for (int64_t tx = klo; tx <= khi; ++tx)
    s += agg[L.cdfA + ((int64_t)ty * L.ntx + tx) * D + (u - tx * TW - y0)];
  return s;
}

template <int TW, int TH, typename Cy>
__device__ __forceinline__ Cy band_b(const Cy* agg, const SatLayout& L, int ty, int64_t v) {
  constexpr int D = TW + TH - 1;
  const int64_t y0 = (int64_t)ty * TH;
  int64_t klo = ceildiv(v + y0 - TW + 1, TW);
  klo = klo < 0 ? 0 : (klo > L.ntx ? L.ntx : klo);
  int64_t khi = floordiv(v + y0 + TH - 1, TW);
  if (khi > L.ntx - 1) khi = L.ntx - 1;
  Cy s = agg[L.prefTot + (int64_t)ty * (L.ntx + 1) + klo];
  for (int64_t tx = klo; tx <= khi; ++tx)
    s += agg[L.cdfB + ((int64_t)ty * L.ntx + tx) * D + (v - tx * TW + y0 + TH - 1)];
  return s;
}

template <int P, int TW, int TH>
__global__ __launch_bounds__(256) void k_sat_carry2(Batch B) {
  typedef typename PT<P>::carry Cy;
  typedef typename PT<P>::store St;
  const int k = find_inst(B.off_carry2, B.n, blockIdx.x);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  const SatLayout L = sat_layout(I.N, TW, TH);
  const int N = I.N;
  const int64_t idx = (int64_t)(blockIdx.x - B.off_carry2[k]) * 256 + threadIdx.x;
  const Cy* agg = (const Cy*)I.agg;
  Cy* carry = (Cy*)I.carry;
  const int64_t nS = L.NX + 1;
  if (idx < nS) {
    const int i = (int)idx;
    int tx = i / TW;
    if (tx > L.ntx - 1) tx = L.ntx - 1;
    const int c = i - tx * TW;
    Cy run = 0;
#pragma unroll 4
    for (int ty = 0; ty < L.nty; ++ty) {
      const Cy band = agg[L.prefTot + (int64_t)ty * (L.ntx + 1) + tx] +
                      agg[L.colsum + ((int64_t)ty * L.ntx + tx) * (TW + 1) + c];
      carry[L.Stop + (int64_t)ty * nS + i] = run;
      run += band;
    }
  } else if (idx < nS + L.LA) {
    const int64_t a = idx - nS;
    const int64_t u = a - 1;
    Cy run = 0;
#pragma unroll 4
    for (int ty = 0; ty < L.nty; ++ty) {
      const Cy band = band_a<TW, TH>(agg, L, ty, u);
      carry[L.TAc + (int64_t)ty * L.LA + a] = run;
      run += band;
    }
    carry[L.TAc + (int64_t)L.nty * L.LA + a] = run;
    if (a <= 2 * N) ((St*)I.HA)[a] = (St)run;          // HA(s) = TA(s-1, N), s = a
  } else if (idx < nS + L.LA + L.LB) {
    const int64_t bi = idx - nS - L.LA;
    const int64_t v = bi - L.NY;
    Cy run = 0;
#pragma unroll 4
    for (int ty = 0; ty < L.nty; ++ty) {
      const Cy band = band_b<TW, TH>(agg, L, ty, v);
      carry[L.TBc + (int64_t)ty * L.LB + bi] = run;
      run += band;
    }
    carry[L.TBc + (int64_t)L.nty * L.LB + bi] = run;
    if (v >= -N && v <= N) ((St*)I.HB)[N - v] = (St)(agg[L.Cval] - run);   // HB(r) = C - TB(-r, N)
  }
}

template <int P, int TW, int TH, bool DENSE>
__global__ __launch_bounds__(TW) void k_sat_final(Batch B) {
  typedef typename PT<P>::acc A;
  typedef typename PT<P>::carry Cy;
  typedef typename PT<P>::store St;
  constexpr int NW = TW / 64;
  constexpr int XW = TW + 2 * TH;          // columns x0-TH .. x0+TW+TH-1
  constexpr int E = XW / 64 + 1;            // lanes cover c = 0..XW inclusive
  constexpr int NSL = TW + TH + 1;         // anti-diagonal / diagonal slots
  const int64_t nb = B.off_tiles[B.n];
  const int64_t b = xcd_block(blockIdx.x, nb);
  const int k = find_inst(B.off_tiles, B.n, b);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  __shared__ A Rs[TH][XW + 1];
  __shared__ A ta[2][NSL];
  __shared__ A tb[2][NSL];
  __shared__ float lut_s[kLutLds];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int N = I.N;
  const SatLayout L = sat_layout(N, TW, TH);
  const int tile = (int)(b - B.off_tiles[k]);
  const int tx = tile % L.ntx, ty = tile / L.ntx;
  const int x0 = tx * TW, y0 = ty * TH;
  const bool lut_lds = !DENSE && I.n_lut <= kLutLds;
  if (lut_lds)
    for (int v = t; v < I.n_lut; v += TW) lut_s[v] = I.lut[v];
  __syncthreads();
  const Cy* agg = (const Cy*)I.agg;
  const Cy* carry = (const Cy*)I.carry;
  // row prefix sums over the tile and its halo: R(x0-TH+c, q) for c in [0, XW]
  for (int r = w; r < TH; r += NW) {
    const int q = y0 + r;
    float dv[E];
    A loc;
    acc_zero(loc);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int c = lane * E + e;
      dv[e] = c < XW ? dens_at<DENSE>(I, lut_s, lut_lds, x0 - TH + c, q) : 0.f;
      acc_add(loc, dv[e]);
    }
    A run = wave_exclusive_scan(loc, lane);
    A lv[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      lv[e] = run;
      acc_add(run, dv[e]);
    }
    // R(c) = R(x0, q) + (L(c) - L(TH)) keeps R exact at the tile's left edge
    const A lth = shfl_acc(lv[TH % E], TH / E);
    A rc;
    from_carry(rc, agg[L.RC + (int64_t)tx * L.NY + q]);
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int c = lane * E + e;
      if (c <= XW) {
        A v = rc;
        acc_addv(v, acc_sub(lv[e], lth));
        Rs[r][c] = v;
      }
    }
  }
  // carries entering the tile
  A sacc, saccN;
  from_carry(sacc, carry[L.Stop + (int64_t)ty * (L.NX + 1) + x0 + t]);
  const bool extra = (x0 + TW == N) && t == 0;   // the tile column that ends at node column N
  if (extra) from_carry(saccN, carry[L.Stop + (int64_t)ty * (L.NX + 1) + N]);
  else acc_zero(saccN);
  A ra[2], rb[2];
  const int s1 = t + TW;
  const bool has1 = s1 < NSL;
  from_carry(ra[0], carry[L.TAc + (int64_t)ty * L.LA + x0 + y0 + t]);
  from_carry(rb[0], carry[L.TBc + (int64_t)ty * L.LB + (x0 - y0 - TH + L.NY) + t]);
  if (has1) {
    from_carry(ra[1], carry[L.TAc + (int64_t)ty * L.LA + x0 + y0 + s1]);
    from_carry(rb[1], carry[L.TBc + (int64_t)ty * L.LB + (x0 - y0 - TH + L.NY) + s1]);
  } else {
    acc_zero(ra[1]);
    acc_zero(rb[1]);
  }
  St* S = (St*)I.S;
  St* T = (St*)I.T;
  const int64_t pitch = I.pitch;
  const int i = x0 + t;
  if (ty == 0) {
    if (i <= N) {
      S[i] = (St)0;
      T[i] = (St)0;
    }
    if (extra) {
      S[N] = (St)0;
      T[N] = (St)0;
    }
  }
  __syncthreads();
  for (int r = 0; r < TH; ++r) {
    const int j = y0 + r + 1;
    acc_addv(sacc, Rs[r][t + TH]);
    if (extra) acc_addv(saccN, Rs[r][TW + TH]);
    {
      const int ca = t + TH - 1 - r;         // anti-diagonal slot t meets row y0+r here
      acc_addv(ra[0], mid(Rs[r][ca], Rs[r][ca + 1]));
      const int cb = t + r;                  // diagonal slot t
      acc_addv(rb[0], mid(Rs[r][cb], Rs[r][cb + 1]));
      ta[r & 1][t] = ra[0];
      tb[r & 1][t] = rb[0];
    }
    if (has1) {
      const int ca = s1 + TH - 1 - r;
      acc_addv(ra[1], mid(Rs[r][ca], Rs[r][ca + 1]));
      const int cb = s1 + r;
      acc_addv(rb[1], mid(Rs[r][cb], Rs[r][cb + 1]));
      ta[r & 1][s1] = ra[1];
      tb[r & 1][s1] = rb[1];
    }
    __syncthreads();
    if (j <= N) {
      const int64_t row = (int64_t)j * pitch;
      if (i <= N) {
        S[row + i] = to_store(sacc);
        T[row + i] = to_store(acc_sub(ta[r & 1][t + r + 1], tb[r & 1][t + TH - 1 - r]));
      }
      if (extra) {
        S[row + N] = to_store(saccN);
        T[row + N] = to_store(acc_sub(ta[r & 1][TW + r + 1], tb[r & 1][TW + TH - 1 - r]));
      }
    }
  }
}

// host launchers --------------------------------------------------------------

template <int P, int TW, int TH>
static void launch_sat_t(const Batch& B, bool dense, int64_t tiles, int64_t c1, int64_t c2,
                         hipStream_t s, StageHook h, void* u) {
  auto hk = [&](int st, int after) { if (h) h(st, after, u); };
  hk(ST_SAT_REDUCE, 0);
  if (dense) hipLaunchKernelGGL((k_sat_reduce<P, TW, TH, true>), dim3(tiles), dim3(TW), 0, s, B);
  else hipLaunchKernelGGL((k_sat_reduce<P, TW, TH, false>), dim3(tiles), dim3(TW), 0, s, B);
  hk(ST_SAT_REDUCE, 1);
  hk(ST_SAT_CARRY1, 0);
  hipLaunchKernelGGL((k_sat_carry1<P, TW, TH>), dim3(c1), dim3(256), 0, s, B);
  hk(ST_SAT_CARRY1, 1);
  hk(ST_SAT_CARRY2, 0);
  hipLaunchKernelGGL((k_sat_carry2<P, TW, TH>), dim3(c2), dim3(256), 0, s, B);
  hk(ST_SAT_CARRY2, 1);
  hk(ST_SAT_FINAL, 0);
  if (dense) hipLaunchKernelGGL((k_sat_final<P, TW, TH, true>), dim3(tiles), dim3(TW), 0, s, B);
  else hipLaunchKernelGGL((k_sat_final<P, TW, TH, false>), dim3(tiles), dim3(TW), 0, s, B);
  hk(ST_SAT_FINAL, 1);
}

template <int P>
static bool launch_sat_p(const Batch& B, int tw, int th, bool dense, int64_t tiles, int64_t c1,
                         int64_t c2, hipStream_t s, StageHook h, void* u) {
  if (tw == 64 && th == 16) launch_sat_t<P, 64, 16>(B, dense, tiles, c1, c2, s, h, u);
  else if (tw == 128 && th == 16) launch_sat_t<P, 128, 16>(B, dense, tiles, c1, c2, s, h, u);
  else if (tw == 128 && th == 32) launch_sat_t<P, 128, 32>(B, dense, tiles, c1, c2, s, h, u);
  else if (tw == 256 && th == 32) launch_sat_t<P, 256, 32>(B, dense, tiles, c1, c2, s, h, u);
  else return false;
  return true;
}

bool launch_sat(const Batch& B, int prec, int tw, int th, bool dense, int64_t tiles, int64_t c1,
                int64_t c2, hipStream_t s, StageHook h, void* u) {
  if (prec == CG_F32) return launch_sat_p<CG_F32>(B, tw, th, dense, tiles, c1, c2, s, h, u);
  if (prec == CG_COMP) return launch_sat_p<CG_COMP>(B, tw, th, dense, tiles, c1, c2, s, h, u);
  if (prec == CG_F64) return launch_sat_p<CG_F64>(B, tw, th, dense, tiles, c1, c2, s, h, u);
  return false;
}

bool sat_shape_supported(int tw, int th) {
  return (tw == 64 && th == 16) || (tw == 128 && th == 16) || (tw == 128 && th == 32) ||
         (tw == 256 && th == 32);
}

}  // namespace cgk
