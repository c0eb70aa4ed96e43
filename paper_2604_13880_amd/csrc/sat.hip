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
//   k_sat_reduce  per tile: row totals, column prefix sums, and masses
//                 below every anti-diagonal and diagonal (from line sums
//                 of the raw densities, no row scans)
//   k_sat_carry1  row carries across tile columns, tile-row prefix totals
//   k_sat_carry2  carries entering every tile row for S, TA, TB; HA, HB
//   k_sat_final   per tile (its own labels only; the parts of the
//                 tilted lines in the neighbouring tiles come from the
//                 reduce pass's line masses): row prefix sums staged in
//                 LDS, then a sweep down the tile's rows that accumulates
//                 S and the line sums in registers and writes one row of
//                 S and T per step (coalesced stores)
// Accumulation precision: float, compensated float or double (PT<P>).
#include "cg_dev.h"

namespace cgk {

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kSub_Rows = 4;   // rows staged in LDS at a time (a sub-band of the tile)
constexpr int kPrefLds = 1024;    // tile-row prefix totals the carry pass keeps in LDS

__device__ __forceinline__ float shfl_xor_acc(float v, int d) { return __shfl_xor(v, d, 64); }
__device__ __forceinline__ double shfl_xor_acc(double v, int d) { return __shfl_xor(v, d, 64); }
__device__ __forceinline__ Comp shfl_xor_acc(Comp v, int d) {
  return Comp{__shfl_xor(v.hi, d, 64), __shfl_xor(v.lo, d, 64)};
}

// Sum over the wavefront (butterfly: every lane gets the same value).
template <typename A>
__device__ __forceinline__ A wave_sum(A v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const A o = shfl_xor_acc(v, d);
    acc_addv(v, o);
  }
  return v;
}

// K exclusive scans over the block's threads at once, each in thread order
// (a fixed order; two barriers for all of them); `total` receives the
// block sums.  wt: LDS scratch of K * NW entries.
template <typename A, int NW, int K>
__device__ __forceinline__ void block_exclusive_scans(A (&v)[K], A* wt, A (&total)[K]) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  A ex[K];
#pragma unroll
  for (int k = 0; k < K; ++k) ex[k] = wave_exclusive_scan(v[k], lane);
  __syncthreads();
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      A inc = ex[k];
      acc_addv(inc, v[k]);
      wt[k * NW + w] = inc;
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    A pre;
    acc_zero(pre);
    acc_zero(total[k]);
#pragma unroll
    for (int i = 0; i < NW; ++i) {
      if (i < w) acc_addv(pre, wt[k * NW + i]);
      acc_addv(total[k], wt[k * NW + i]);
    }
    acc_addv(pre, ex[k]);
    v[k] = pre;
  }
}

// Local sums inside a tile (at most one tile row-strip of mass) use float
// in the float-stored modes and double in the double mode; the long sums
// (carries across tiles, row carries) use the mode's accumulator.
template <int P> struct LocalT { typedef float type; };
template <> struct LocalT<CG_F64> { typedef double type; };

// Inclusive scan over a wavefront with DPP row shifts and row broadcasts
// (no LDS traffic): within each row of 16 lanes by shifts of 1, 2, 4, 8,
// then row 0's total into row 1, row 2's into row 3, and lane 31's into
// rows 2 and 3.  Lanes whose source lies outside the row read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_take(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_take(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROWS, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
// Lane l takes lane l+1's value (lane 63 takes 0) / lane l-1's (lane 0 takes 0).
template <typename Lc>
__device__ __forceinline__ Lc take_right(Lc v) { return dpp_take<0x130, 0xf>(v); }   // wave_shl:1
template <typename Lc>
__device__ __forceinline__ Lc take_left(Lc v) { return dpp_take<0x138, 0xf>(v); }    // wave_shr:1
// One lane's value (uniform lane index) and a write into one lane.
__device__ __forceinline__ float lane_get(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_get(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
template <typename Lc>
__device__ __forceinline__ Lc lane_put(Lc x, int l, Lc old) { return (int)(threadIdx.x & 63) == l ? x : old; }

template <typename Lc>
__device__ __forceinline__ Lc wave_inclusive_scan_dpp(Lc x) {
  x += dpp_take<0x111, 0xf>(x);   // row_shr:1
  x += dpp_take<0x112, 0xf>(x);   // row_shr:2
  x += dpp_take<0x114, 0xf>(x);   // row_shr:4
  x += dpp_take<0x118, 0xf>(x);   // row_shr:8
  x += dpp_take<0x142, 0xa>(x);   // row_bcast:15 into rows 1 and 3
  x += dpp_take<0x143, 0xc>(x);   // row_bcast:31 into rows 2 and 3
  return x;
}

// Inclusive scan within segments of SEG lanes (16, 32 or 48/64; a
// segment starts at a 16-lane row): the row shifts, then the row-15
// broadcast only into rows that continue a segment, the row-31 broadcast
// only for segments longer than 32 lanes.
template <int SEG, typename Lc>
__device__ __forceinline__ Lc seg_inclusive_scan_dpp(Lc x) {
  static_assert(SEG == 16 || SEG == 32 || SEG == 48 || SEG == 64, "segments are whole DPP rows");
  x += dpp_take<0x111, 0xf>(x);
  x += dpp_take<0x112, 0xf>(x);
  x += dpp_take<0x114, 0xf>(x);
  x += dpp_take<0x118, 0xf>(x);
  if (SEG >= 32) x += dpp_take<0x142, 0xa>(x);
  if (SEG >= 48) x += dpp_take<0x143, 0xc>(x);
  return x;
}

typedef double f64x2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
// Buffer store of a 4, 8 or 16-byte value at voff + soff bytes, marked
// nontemporal (cache policy bit 1): the tables are written once and read
// by the next kernel, so they should not displace the labels and LUT
// that the writer's blocks are still reading.
template <typename T>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  constexpr int kNT = 2;
  if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), rs, voff, soff, kNT);
  else if constexpr (sizeof(T) == 8) __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), rs, voff, soff, kNT);
  else __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, v), rs, voff, soff, kNT);
}
// Four consecutive LDS values (16-byte aligned) in 16-byte stores.
__device__ __forceinline__ void store4(float* p, const float v[4]) { *(f32x4_t*)p = f32x4_t{v[0], v[1], v[2], v[3]}; }
__device__ __forceinline__ void store4(double* p, const double v[4]) {
  *(f64x2_t*)p = f64x2_t{v[0], v[1]};
  *(f64x2_t*)(p + 2) = f64x2_t{v[2], v[3]};
}

// One sub-band of kSub_Rows rows of a tile's W columns, one row per segment
// of W/4 lanes (16, 32 or 64), 4 consecutive columns per lane: wavefront w
// holds rows w*RPP .. w*RPP+RPP-1.  The labels (or densities) of a later
// sub-band are loaded while the current one is scanned.
template <bool DENSE, int W, int NW>
struct RowStage {
  static constexpr int LPR = W / 4;                    // lanes per row = segment
  static constexpr int RPP = 64 / LPR;                 // rows per wavefront
  static_assert(LPR == 16 || LPR == 32 || LPR == 64, "segments are whole DPP rows");
  static_assert(NW * RPP == kSub_Rows, "one pass covers the sub-band");
  // Labels and LUT entries are read with buffer loads: an offset past the
  // descriptor's byte count reads 0, so chunks outside the texture and
  // labels outside the LUT need no branch (kOut marks them).
  static constexpr uint32_t kOut = 0x80000000u;
  __amdgpu_buffer_rsrc_t lab_rs, lut_rs;
  u32x2_t lab;
  f32x4_t da;
  bool ok;
  int g, li;   // row of the sub-band, chunk of the row

  __device__ __forceinline__ void init(const InstG& I) {
    const int lane = threadIdx.x & 63;
    g = (threadIdx.x >> 6) * RPP + lane / LPR;
    li = lane % LPR;
    if (!DENSE) {
      lab_rs = __builtin_amdgcn_make_buffer_rsrc((void*)I.labels, (short)0, (int)(2 * (int64_t)I.N * I.N), 0x00020000);
      lut_rs = __builtin_amdgcn_make_buffer_rsrc((void*)I.lut, (short)0, 4 * I.n_lut, 0x00020000);
    }
  }
  __device__ __forceinline__ void load(const InstG& I, int xs, int y) {
    const int N = I.N, q = y + g, p = xs + 4 * li;
    ok = q < N && p < N;   // p >= 0; p and N multiples of 4: whole chunks
    if (DENSE) {
      if (ok) da = *(g_ptr<const f32x4_t>)(I.density + (int64_t)q * N + p);
    } else {
      const uint32_t off = ok ? (uint32_t)(2 * ((int64_t)q * N + p)) : kOut;   // N^2 * 2 < 2^31
      lab = __builtin_amdgcn_raw_buffer_load_b64(lab_rs, (int)off, 0, 0);
    }
  }
  // densities from a LUT copy in LDS (clamped index and a select)
  __device__ __forceinline__ void values_lds(const float* lut_s, int n_lut, float v[4]) const {
    const int nl = ok ? n_lut : 0;   // outside the texture: no mass
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int lb = (int)((lab[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
      const float x = lut_s[lb < kLutLds ? lb : 0];
      v[e] = lb < nl ? x : 0.f;   // labels outside the LUT carry no mass
    }
  }
  __device__ __forceinline__ void values(const InstG& I, float v[4]) const {
    if (DENSE) {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = ok ? da[e] : 0.f;
    } else {
      const uint32_t out = ok ? 0u : kOut;   // zero mass outside the texture
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t lb = (lab[e >> 1] >> (16 * (e & 1))) & 0xFFFFu;
        v[e] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(lut_rs, (int)((lb << 2) | out), 0, 0));
      }
    }
  }
};

template <typename A, typename Lc>
__device__ __forceinline__ void acc_add_local(A& a, Lc x) { acc_add(a, x); }
template <>
__device__ __forceinline__ void acc_add_local<double, double>(double& a, double x) { a += x; }

// Tile aggregates from line sums of the raw densities (no row scans):
// column totals, row totals, and the sums h_a(s) over the tile's
// anti-diagonals s = (p - x0) + (q - y0) and h_b(s) over its diagonals
// s = (p - x0) - (q - y0) + TH - 1.  The mass of the tile below an
// anti-diagonal slot c (pixels bisected by it count half) is then
// sum_{s<c} h_a(s) + h_a(c)/2, and likewise for the diagonals.
// Step 3 inside the reduce pass: every block builds the instance's density
// LUT in LDS from the pixel counts (or polygon areas) and the values, in
// one fixed order, so all blocks hold the same table; the instance's first
// block also publishes it (and d0, C) for the writer.  d0 = sum s / sum o
// over regions with o > 0, background density shape * d0 (or from a
// prescribed background mass), LUT scaled so the texture mass is N^2.
template <int NT>
__device__ __forceinline__ void density_lut(const InstG& I, float* lut_s, bool publish) {
  constexpr int NW = NT / 64;
  __shared__ double part[3][NW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6, R = I.R;
  const double NN = (double)I.N * (double)I.N;
  const bool poly = I.area_source == CG_AREA_POLYGON;
  const double c0 = (double)I.counts[0];   // background pixels, needed after the sums
  double ss = 0.0, so = 0.0, sc = 0.0;
  // the thread's first region is kept for the table (most instances have
  // at most one region per thread); every load of a region is issued
  // before any is used
  double q1 = 0.0;
  for (int v = 1 + t; v <= R; v += NT) {
    const double cnt = (double)I.counts[v];
    const double ar = I.areas[v];
    const double s = (double)I.values[v - 1];
    const double o = poly ? ar * NN : cnt;
    const double q = o > 0.0 ? s / o : 0.0;
    if (v == 1 + t) q1 = q;
    if (o > 0.0) {
      ss += s;
      sc += q * cnt;
    }
    so += o;
  }
  ss = wave_inclusive_scan_dpp(ss);   // lane 63: the wavefront's sum
  so = wave_inclusive_scan_dpp(so);
  sc = wave_inclusive_scan_dpp(sc);
  if (lane == 63) {
    part[0][w] = ss;
    part[1][w] = so;
    part[2][w] = sc;
  }
  __syncthreads();
  ss = so = sc = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    ss += part[0][i];
    so += part[1][i];
    sc += part[2][i];
  }
  const double d0 = so > 0.0 ? ss / so : 1.0;
  const double bdv = background_density(I, d0, c0);
  const double cm = sc + bdv * c0;
  const double kappa = cm > 0.0 ? NN / cm : 1.0;
  g_ptr<float> lut = (g_ptr<float>)I.lut;
  for (int v = 1 + t; v <= R; v += NT) {
    double q = q1;
    if (v != 1 + t) {
      const double o = poly ? I.areas[v] * NN : (double)I.counts[v];
      q = o > 0.0 ? (double)I.values[v - 1] / o : 0.0;
    }
    const float x = (float)(kappa * q);
    lut_s[v] = x;
    if (publish) lut[v] = x;
  }
  if (t == 0) {
    const float x0 = (float)(kappa * bdv);
    lut_s[0] = x0;
    if (publish) {
      lut[0] = x0;
      I.st->d0 = d0;
      I.st->C = cm;
    }
  }
}

template <int P, int TW, int TH, bool DENSE>
__global__ __launch_bounds__(TW, 8) void k_sat_reduce(Batch B) {
  typedef typename PT<P>::acc A;
  typedef typename PT<P>::carry Cy;
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);   // one block per tile of the batch
  int64_t first;
  const int k = find_inst(B, B.off_tiles, KD_TILES, b, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  typedef typename LocalT<P>::type Lc;
  typedef RowStage<DENSE, TW, TW / 64> Stage;
  constexpr int NW = TW / 64, D = TW + TH - 1;
  constexpr int LPR = Stage::LPR, NG = kSub_Rows;   // lanes per row; rows per step = row classes
  static_assert(TH <= TW, "tiles are at least as wide as they are tall");
  static_assert(TH % NG == 0, "whole steps");
  __shared__ A rsum[TH];
  __shared__ A wt[5 * NW];
  __shared__ float lut_s[kLutLds];
  __shared__ Lc hpa[NG][D];    // line sums of one row class: anti-diagonals s = p + r
  __shared__ Lc hpb[NG][D];    // diagonals s = p - r + TH - 1
  __shared__ __align__(16) Lc colp[NG][TW];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const SatLayout L = sat_layout(I.N, TW, TH);
  const int tile = (int)(b - first);
  const int tx = tile % L.ntx, ty = tile / L.ntx;
  const int x0 = tx * TW, y0 = ty * TH;
  const bool lut_lds = !DENSE && I.n_lut <= kLutLds;
  Stage stg;
  stg.init(I);
  stg.load(I, x0, y0);   // the first labels are in flight while the density table is built
  if (!DENSE && B.make_lut) density_lut<TW>(I, lut_s, tile == 0);   // R + 1 <= kLutLds (host)
  else if (lut_lds)
    for (int v = t; v < I.n_lut; v += TW) lut_s[v] = I.lut[v];
  for (int e = t; e < NG * D; e += TW) {   // lines a row class never meets stay 0
    (&hpa[0][0])[e] = (Lc)0;
    (&hpb[0][0])[e] = (Lc)0;
  }
  __syncthreads();
  // Every step covers NG rows: row r0 + g of the tile is held by one
  // segment of LPR lanes, 4 consecutive columns per lane, so each lane
  // sees every NG-th row of the same 4 columns.  Per lane and column it
  // keeps the column sum of its rows and the sums of the anti-diagonal and
  // the diagonal through that column: NG rows down, both lines have moved
  // NG = 4 columns, i.e. one lane (DPP wave shift), left / right.  A line
  // about to leave the tile is written to its row class's table; after the
  // last step the lines still inside are.  No barrier inside the loop.
  const int g = stg.g, li = stg.li;
  auto values = [&](float v[4]) {
    if (lut_lds) stg.values_lds(lut_s, I.n_lut, v);
    else stg.values(I, v);
  };
  Lc cs[4] = {0, 0, 0, 0}, la[4] = {0, 0, 0, 0}, lb[4] = {0, 0, 0, 0};
  float dnext[4];
  values(dnext);
  if (NG < TH) stg.load(I, x0, y0 + NG);
  for (int r0 = 0; r0 < TH; r0 += NG) {
    const int r = r0 + g;
    float dv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) dv[e] = dnext[e];
    if (r0 + NG < TH) {   // densities of the next step, labels of the one after
      values(dnext);
      if (r0 + 2 * NG < TH) stg.load(I, x0, y0 + r0 + 2 * NG);
    }
    Lc s4 = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) s4 += (Lc)dv[e];
    const Lc rt = seg_inclusive_scan_dpp<LPR>(s4);   // the segment's last lane: the row total
    if (li == LPR - 1) {
      acc_zero(rsum[r]);
      acc_add_local(rsum[r], rt);
    }
    if (r0 > 0) {   // lines leaving at the left (anti-diagonal) or right (diagonal) edge
      if (li == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) hpa[g][c + r - NG] = la[c];
      }
      if (li == LPR - 1) {
#pragma unroll
        for (int c = 0; c < 4; ++c) hpb[g][TW - 4 + c - (r - NG) + TH - 1] = lb[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      Lc ia = take_right(la[c]), ib = take_left(lb[c]);
      if (LPR < 64) {   // segments hold different rows: new lines enter at the ends
        ia = li == LPR - 1 ? (Lc)0 : ia;
        ib = li == 0 ? (Lc)0 : ib;
      }
      la[c] = ia + (Lc)dv[c];
      lb[c] = ib + (Lc)dv[c];
      cs[c] += (Lc)dv[c];
    }
  }
  {
    const int rl = TH - NG + g;   // last row of this class
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      hpa[g][4 * li + c + rl] = la[c];
      hpb[g][4 * li + c - rl + TH - 1] = lb[c];
    }
    store4(&colp[g][4 * li], cs);
  }
  __syncthreads();
  // per thread: column t's total and the line sums of slots t and t + TW,
  // row classes in order
  Lc col = 0;
#pragma unroll
  for (int gg = 0; gg < NG; ++gg) col += colp[gg][t];
  auto line = [&](const Lc (*hp)[D], int sl) -> Lc {
    Lc v = 0;
#pragma unroll
    for (int gg = 0; gg < NG; ++gg) v += hp[gg][sl];
    return v;
  };
  const int c1 = t + TW;
  const bool has1 = c1 < D;
  const Lc ha0 = line(hpa, t), hb0 = line(hpb, t);
  const Lc ha1 = has1 ? line(hpa, c1) : (Lc)0, hb1 = has1 ? line(hpb, c1) : (Lc)0;
  __syncthreads();
  g_ptr<Cy> agg = (g_ptr<Cy>)I.agg;
  const int64_t tid = (int64_t)ty * L.ntx + tx;
  for (int r = t; r < TH; r += TW) agg[L.rowTot + (int64_t)tx * L.NY + y0 + r] = to_carry(rsum[r]);
  A z, colA, ha0A, ha1A, hb0A, hb1A;
  acc_zero(z);
  acc_zero(colA); acc_add_local(colA, col);
  acc_zero(ha0A); acc_add_local(ha0A, ha0);
  acc_zero(ha1A); acc_add_local(ha1A, ha1);
  acc_zero(hb0A); acc_add_local(hb0A, hb0);
  acc_zero(hb1A); acc_add_local(hb1A, hb1);
  // column prefix, and the line masses below every anti-diagonal / diagonal slot
  A sc[5] = {colA, ha0A, has1 ? ha1A : z, hb0A, has1 ? hb1A : z}, stot[5];
  block_exclusive_scans<A, NW, 5>(sc, wt, stot);
  A ex = sc[0], tot = stot[0], ea0 = sc[1], tA0 = stot[1], ea1 = sc[2], eb0 = sc[3], tB0 = stot[3], eb1 = sc[4];
  acc_addv(ex, colA);
  agg[L.colsum + tid * (TW + 1) + t + 1] = to_carry(ex);
  if (t == 0) {
    agg[L.colsum + tid * (TW + 1)] = (Cy)0;
    agg[L.tileTot + tid] = to_carry(tot);
  }
  acc_addv(ea0, acc_half(ha0A));
  acc_addv(eb0, acc_half(hb0A));
  agg[L.cdfA + tid * D + t] = to_carry(ea0);
  agg[L.cdfB + tid * D + t] = to_carry(eb0);
  if (has1) {
    A a1 = tA0, b1 = tB0;
    acc_addv(a1, ea1);
    acc_addv(a1, acc_half(ha1A));
    acc_addv(b1, eb1);
    acc_addv(b1, acc_half(hb1A));
    agg[L.cdfA + tid * D + c1] = to_carry(a1);
    agg[L.cdfB + tid * D + c1] = to_carry(b1);
  }
}

template <int P, int TW, int TH>
__global__ __launch_bounds__(256) void k_sat_carry1(Batch B) {
  typedef typename PT<P>::carry Cy;
  int64_t first;
  const int k = find_inst(B, B.off_carry1, KD_CARRY1, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  const SatLayout L = sat_layout(I.N, TW, TH);
  const int64_t idx = (int64_t)(blockIdx.x - first) * 256 + threadIdx.x;
  g_ptr<Cy> agg = (g_ptr<Cy>)I.agg;
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
  }
}

// Mass of tile row ty on the anti-diagonal side u (tiles fully below u give
// their totals through the tile-row prefix, at most two tiles are cut),
// in two parts: the tile-row prefix entry (its index into the [tile row]
// [ntx + 1] prefix table) and the one or two cut tiles' line masses (0
// where a tile is not cut), so that the line masses can be loaded before
// the prefix table is complete.  Likewise on the diagonal side v.
template <int TW, int TH, typename Cy>
__device__ __forceinline__ int band_a_parts(g_ptr<const Cy> agg, const SatLayout& L, int ty, int64_t u, Cy& a1, Cy& a2) {
  constexpr int D = TW + TH - 1;
  const int64_t y0 = (int64_t)ty * TH;
  int64_t klo = ceildiv(u - y0 - TW - TH + 2, TW);
  klo = klo < 0 ? 0 : (klo > L.ntx ? L.ntx : klo);
  int64_t khi = floordiv(u - y0, TW);
  if (khi > L.ntx - 1) khi = L.ntx - 1;
  const int64_t base = L.cdfA + (int64_t)ty * L.ntx * D;
  a1 = klo <= khi ? agg[base + klo * D + (u - klo * TW - y0)] : (Cy)0;
  a2 = klo + 1 <= khi ? agg[base + (klo + 1) * D + (u - (klo + 1) * TW - y0)] : (Cy)0;
  return ty * (L.ntx + 1) + (int)klo;
}

template <int TW, int TH, typename Cy>
__device__ __forceinline__ int band_b_parts(g_ptr<const Cy> agg, const SatLayout& L, int ty, int64_t v, Cy& a1, Cy& a2) {
  constexpr int D = TW + TH - 1;
  const int64_t y0 = (int64_t)ty * TH;
  int64_t klo = ceildiv(v + y0 - TW + 1, TW);
  klo = klo < 0 ? 0 : (klo > L.ntx ? L.ntx : klo);
  int64_t khi = floordiv(v + y0 + TH - 1, TW);
  if (khi > L.ntx - 1) khi = L.ntx - 1;
  const int64_t base = L.cdfB + (int64_t)ty * L.ntx * D;
  a1 = klo <= khi ? agg[base + klo * D + (v - klo * TW + y0 + TH - 1)] : (Cy)0;
  a2 = klo + 1 <= khi ? agg[base + (klo + 1) * D + (v - (klo + 1) * TW + y0 + TH - 1)] : (Cy)0;
  return ty * (L.ntx + 1) + (int)klo;
}

// Carries entering every tile row: for each index (node column i for S,
// anti-diagonal u for TA, diagonal v for TB) an exclusive scan over the tile
// rows of the band values.  A block holds IPB indices x CH chunks of
// kCarryRows tile rows; chunk sums are joined by an LDS scan.
template <int P, int TW, int TH, bool PREF_LDS>
__global__ __launch_bounds__(256) void k_sat_carry2(Batch B) {
  typedef typename PT<P>::carry Cy;
  typedef typename PT<P>::store St;
  int64_t first;
  const int k = find_inst(B, B.off_carry2, KD_CARRY2, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  __shared__ Cy part[256];
  __shared__ Cy partC[256];
  __shared__ Cy pref_s[PREF_LDS ? kPrefLds : 1];
  const SatLayout L = sat_layout(I.N, TW, TH);
  const int N = I.N, nty = L.nty;
  const int CH = L.carry_ch, IPB = 256 / CH;
  const int t = threadIdx.x, ch = t / IPB, j = t - ch * IPB;
  const int64_t idx = (int64_t)(blockIdx.x - first) * IPB + j;
  g_ptr<const Cy> agg = (g_ptr<const Cy>)I.agg;
  g_ptr<Cy> carry = (g_ptr<Cy>)I.carry;
  const int64_t nS = L.NX + 1;
  const int seg = idx < nS ? 0 : (idx < nS + L.LA ? 1 : (idx < nS + L.LA + L.LB ? 2 : 3));
  const int ty0 = ch * kCarryRows;
  // the band values' tile parts first (they do not need the prefix table),
  // then the tile-row prefix entries
  int pidx[kCarryRows];
  Cy a1[kCarryRows], a2[kCarryRows];
#pragma unroll
  for (int d = 0; d < kCarryRows; ++d) {
    const int ty = ty0 + d;
    pidx[d] = 0;
    a1[d] = a2[d] = (Cy)0;
    if (ty < nty) {
      if (seg == 0) {
        const int i = (int)idx;
        int tx = i / TW;
        if (tx > L.ntx - 1) tx = L.ntx - 1;
        pidx[d] = ty * (L.ntx + 1) + tx;
        a1[d] = agg[L.colsum + ((int64_t)ty * L.ntx + tx) * (TW + 1) + (i - tx * TW)];
      } else if (seg == 1) {
        pidx[d] = band_a_parts<TW, TH, Cy>(agg, L, ty, idx - nS - 1, a1[d], a2[d]);
      } else if (seg == 2) {
        pidx[d] = band_b_parts<TW, TH, Cy>(agg, L, ty, idx - nS - L.LA - L.NY, a1[d], a2[d]);
      }
    }
  }
  if (PREF_LDS) {
    // tile-row prefix totals, one thread per tile row (the order of the
    // row-carry pass): nty <= 256 and nty (ntx + 1) <= kPrefLds here
    g_ptr<const Cy> ag = (g_ptr<const Cy>)I.agg;
    for (int ty = threadIdx.x; ty < L.nty; ty += 256) {
      Cy run = 0;
      for (int c0 = 0; c0 < L.ntx; c0 += 8) {   // loads issued 8 at a time, summed in tile order
        Cy v[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) v[c] = c0 + c < L.ntx ? ag[L.tileTot + (int64_t)ty * L.ntx + c0 + c] : (Cy)0;
#pragma unroll
        for (int c = 0; c < 8; ++c)
          if (c0 + c < L.ntx) {
            pref_s[ty * (L.ntx + 1) + c0 + c] = run;
            run += v[c];
          }
      }
      pref_s[ty * (L.ntx + 1) + L.ntx] = run;
    }
    __syncthreads();
  }
  auto prefix = [&](int pi) -> Cy { return PREF_LDS ? pref_s[pi] : agg[L.prefTot + pi]; };
  Cy band[kCarryRows], tot[kCarryRows];
  Cy sum = 0, sumC = 0;
#pragma unroll
  for (int d = 0; d < kCarryRows; ++d) {
    const int ty = ty0 + d;
    Cy v = 0, w = 0;
    if (ty < nty && seg < 3) {
      v = prefix(pidx[d]);   // + the cut tiles, in the order of the band sums
      v += a1[d];
      v += a2[d];
      if (seg == 2) w = prefix(ty * (L.ntx + 1) + L.ntx);
    }
    band[d] = v;
    tot[d] = w;
    sum += v;
    sumC += w;
  }
  part[t] = sum;
  partC[t] = sumC;
  __syncthreads();
  if (seg == 3) return;
  Cy run = 0, C = 0;
  for (int cc = 0; cc < ch; ++cc) {
    run += part[cc * IPB + j];
    C += partC[cc * IPB + j];
  }
#pragma unroll
  for (int d = 0; d < kCarryRows; ++d) {
    const int ty = ty0 + d;
    if (ty < nty) {
      if (seg == 0) carry[L.Stop + (int64_t)ty * nS + idx] = run;
      else if (seg == 1) carry[L.TAc + (int64_t)ty * L.LA + (idx - nS)] = run;
      else carry[L.TBc + (int64_t)ty * L.LB + (idx - nS - L.LA)] = run;
      run += band[d];
      C += tot[d];        // the total in the order the diagonal sums use
    }
  }
  if (ch == CH - 1) {
    if (seg == 1) {
      const int64_t a = idx - nS;
      carry[L.TAc + (int64_t)nty * L.LA + a] = run;
      if (a <= 2 * N) ((g_ptr<St>)I.HA)[a] = (St)run;                 // HA(s) = TA(s-1, N), s = a
    } else if (seg == 2) {
      const int64_t bi = idx - nS - L.LA, v = bi - L.NY;
      carry[L.TBc + (int64_t)nty * L.LB + bi] = run;
      if (v >= -N && v <= N) ((g_ptr<St>)I.HB)[N - v] = (St)(C - run);  // HB(r) = C - TB(-r, N)
    }
  }
}

// Writer pass.  Per tile (TW threads, one per node column, TH rows; the
// tile's own labels only):
//   S(i, j) = Stop(i) + sum_{rows < j} rc(q) + sum_{rows < j} Rloc(i, q)
//   TA(s, j) = TAc(s) + sum_{rows < j} rc(q) + la(s, j)   (likewise TB)
//   T = TA - TB = (TAc - TBc) + (la - lb)   (the row-carry sums cancel)
// where rc(q) is the row integral left of the tile, Rloc the row integral
// from the tile's left edge to the node and la, lb the sums of Mloc (the
// row integral from the tile's left edge to a pixel centre) along the
// anti-diagonal / diagonal through the node over the tile's rows above it.
// Those lines may start in a neighbouring tile of the same tile row; their
// part there is known from the reduce pass: an anti-diagonal that lies in
// the right tile up to row k adds the tile's own row totals of rows 0..k
// plus the right tile's mass below its anti-diagonal k; a diagonal that
// lies in the left tile adds that tile's mass below the diagonal minus
// its total (Mloc is negative left of the tile).  Inside the tile the
// line sums run in shift registers: after every row the anti-diagonal sums
// move one lane left, the diagonal sums one lane right, and every lane adds
// the Mloc of its column.  Each wavefront sums its own 64-column strip; the
// sums leaving a strip's edge are kept per row in LDS and added to the
// lines' values in the neighbouring strip when T is formed.  Rloc, Mloc,
// la, lb stay within one tile and are kept in the local type; Stop, TAc,
// TBc and the row-carry sum in the accumulator.
template <typename St> struct Pair;
template <> struct Pair<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct Pair<double> { typedef double type __attribute__((ext_vector_type(2))); };

// IL: S and T interleaved in one table of (S, T) pairs (the series driver's
// own buffers: one store per node, and the mapping kernel gathers both
// values of a node from one cache line); else two separate tables.
// Occupancy: asked for 7 wavefronts per SIMD, the compensated mode fits
// 64 registers (8 wavefronts, no spills: the uneven batch's writer 694 ->
// 676 us); the double-accumulator mode does not (spills, slower), so it
// keeps the compiler's choice.
template <int P, int TW, int TH, bool DENSE, bool IL>
__global__ __launch_bounds__(TW, P == CG_COMP ? 7 : 1) void k_sat_final(Batch B) {
  typedef typename PT<P>::acc A;
  typedef typename PT<P>::carry Cy;
  typedef typename PT<P>::store St;
  typedef typename LocalT<P>::type Lc;
  constexpr int NW = TW / 64, SB = kSub_Rows;
  constexpr int NSL = TW + TH + 1;         // anti-diagonal / diagonal slots
  constexpr int D = TW + TH - 1;           // line masses per tile in the reduce pass's table
  constexpr int PP = TW + 4;               // row pitch of Pn (16-byte aligned rows)
  constexpr int OP = 64 + TH;              // rows of the strip-edge tables, 64 leading zeros
  static_assert(TH <= 64 && TH <= TW, "a line crosses at most one strip edge inside a tile row");
  const int64_t b = xcd_block(blockIdx.x, gridDim.x);   // one block per tile of the batch
  int64_t first;
  const int k = find_inst(B, B.off_tiles, KD_TILES, b, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  // One barrier per sub-band for short tiles (a latency-bound single
  // texture: 1024^2 writer 13.8 -> 13.3 us), two for tall ones (the large
  // batches are 2% faster with them): see the loop below.
  constexpr bool ONE = TH <= 16;
  __shared__ __align__(16) Lc Pn[ONE ? 2 : 1][SB][PP];  // exclusive row prefix at node columns 0..TW (TW: the row total)
  __shared__ Lc oa_s[NW + 1][OP];          // [w][64 + r]: anti-diagonal sum leaving strip w's left edge after row r
  __shared__ Lc ob_s[NW + 1][OP];          // [w + 1][64 + r]: diagonal sum leaving strip w's right edge after row r
  __shared__ Lc ea_s[TH];                  // right tile's mass below its anti-diagonal r
  __shared__ Lc eb_s[TH];                  // left tile's line at its last column in row r: mass below - total
  __shared__ A ca_s[NSL];
  __shared__ A cb_s[NSL];
  __shared__ A rc_s[TH];
  __shared__ Lc laN_s[TH];                 // node column N: the rows' totals so far (its anti-diagonal)
  __shared__ St sN_s[TH];                  // node column N: S, stored with T (interleaved float tables)
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int N = I.N;
  const SatLayout L = sat_layout(N, TW, TH);
  const int tile = (int)(b - first);
  const int tx = tile % L.ntx, ty = tile / L.ntx;
  const int x0 = tx * TW, y0 = ty * TH;
  g_ptr<const Cy> agg = (g_ptr<const Cy>)I.agg;
  g_ptr<const Cy> carry = (g_ptr<const Cy>)I.carry;
  typedef RowStage<DENSE, TW, NW> Stage;
  Stage stg;
  stg.init(I);
  stg.load(I, x0, y0);   // the first labels are in flight during the set-up
  // carries entering the tile
  A stop, stopN;
  from_carry(stop, carry[L.Stop + (int64_t)ty * (L.NX + 1) + x0 + t]);
  const bool xcol = x0 + TW == N;                 // the tile column that ends at node column N (block-uniform)
  const bool extra = xcol && t == 0;
  if (extra) from_carry(stopN, carry[L.Stop + (int64_t)ty * (L.NX + 1) + N]);
  else acc_zero(stopN);
  for (int sl = t; sl < NSL; sl += TW) {
    from_carry(ca_s[sl], carry[L.TAc + (int64_t)ty * L.LA + x0 + y0 + sl]);
    from_carry(cb_s[sl], carry[L.TBc + (int64_t)ty * L.LB + (x0 - y0 - TH + L.NY) + sl]);
  }
  for (int r = t; r < TH; r += TW) {   // row carries: the rows' totals in the tile columns to the left
    Cy run = 0;                          // (loads issued 8 at a time, summed in column order)
    for (int c0 = 0; c0 < tx; c0 += 8) {
      Cy v[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] = c0 + c < tx ? agg[L.rowTot + (int64_t)(c0 + c) * L.NY + y0 + r] : (Cy)0;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c0 + c < tx) run += v[c];
    }
    from_carry(rc_s[r], run);
    // lines from the neighbouring tiles of this tile row (tile-local masses)
    Lc ea = 0, eb = 0;
    if (tx + 1 < L.ntx) ea = (Lc)agg[L.cdfA + ((int64_t)ty * L.ntx + tx + 1) * D + r];
    if (tx > 0) {
      const int64_t tl = (int64_t)ty * L.ntx + tx - 1;
      eb = (Lc)(agg[L.cdfB + tl * D + (TW + TH - 2 - r)] - agg[L.tileTot + tl]);
    }
    ea_s[r] = ea;
    eb_s[r] = eb;
  }
  for (int e = t; e < (NW + 1) * OP; e += TW) {   // rows before the tile row and the outer strips read 0
    (&oa_s[0][0])[e] = (Lc)0;
    (&ob_s[0][0])[e] = (Lc)0;
  }
  typedef typename Pair<St>::type St2;
  g_ptr<St> S = (g_ptr<St>)I.S;
  g_ptr<St> T = (g_ptr<St>)I.T;
  const int64_t pitch = I.pitch;
  const int i = x0 + t;
  // tiles are never wider than max(64, N) and the pitch holds every tile
  // column: columns past N are row padding, written without a bound check
  if (ty == 0) {
    if (IL) {
      S[2 * i] = (St)0;
      S[2 * i + 1] = (St)0;
      if (extra) {
        S[2 * N] = (St)0;
        S[2 * N + 1] = (St)0;
      }
    } else {
      S[i] = (St)0;
      T[i] = (St)0;
      if (extra) {
        S[N] = (St)0;
        T[N] = (St)0;
      }
    }
  }
  St sv[SB];               // S of the sub-band's rows, stored with T (interleaved tables)
  Lc dl[SB];               // strip sums of the lines through the sub-band's nodes: la - lb
  A sb = stop, sbN = stopN;   // column carry plus the row carries of the rows done
  Lc rsum = 0, rsumN = 0, rpre = 0;
  Lc ra = 0, rb = 0;       // shift registers: anti-diagonal through this column, diagonal arriving here
  // stores of whole rows: buffer stores, the row offset in a scalar register
  // (tables are below 2 GiB: checked on the host)
  const int64_t tab_bytes = (int64_t)(N + 1) * I.pitch * (IL ? (int64_t)sizeof(St2) : (int64_t)sizeof(St));
  const __amdgpu_buffer_rsrc_t s_rs = __builtin_amdgcn_make_buffer_rsrc((void*)I.S, (short)0, (int)tab_bytes, 0x00020000);
  const __amdgpu_buffer_rsrc_t t_rs = __builtin_amdgcn_make_buffer_rsrc(IL ? (void*)I.S : (void*)I.T, (short)0, (int)tab_bytes, 0x00020000);
  // Interleaved (S, T) pairs of floats go out as one 8-byte store in the T
  // pass.  Pairs of doubles are written in two phases, S in the sweep and T
  // in the T pass (barriers between them, so the compiler cannot merge the
  // halves): after a merged 16-byte store the compiler may rewrite the
  // store's data registers in the next instruction, and with several writer
  // blocks per CU such stores wrote the new values (double-precision series
  // runs were not reproducible).
  constexpr bool kSplit = IL && sizeof(St) == 8;
  // T of the rows of sub-band r0: carries, strip sums and the parts of the
  // lines in the neighbouring strips (rows before the line entered)
  auto t_pass = [&](int r0) {
#pragma unroll
    for (int rr = 0; rr < SB; ++rr) {
      const int r = r0 + rr, j = y0 + r + 1;   // j <= N: N is a multiple of TH
      const int sa = t + r + 1, sbl = t + TH - 1 - r;
      A v = acc_sub(ca_s[sa], cb_s[sbl]);
      // the lines' parts in the neighbouring strips: row r - 64 + lane of
      // strip w + 1 (anti-diagonal), row r - lane of strip w - 1 (diagonal)
      acc_add_local(v, dl[rr] + (oa_s[w + 1][r + lane] - ob_s[w][64 + r - lane]));
      if (kSplit) bstore((St)to_store(v), t_rs, i * (int)sizeof(St2) + (int)sizeof(St), (int)(j * pitch * (int64_t)sizeof(St2)));
      else if (IL) bstore(St2{sv[rr], (St)to_store(v)}, t_rs, i * (int)sizeof(St2), (int)(j * pitch * (int64_t)sizeof(St2)));
      else bstore((St)to_store(v), t_rs, i * (int)sizeof(St), (int)(j * pitch * (int64_t)sizeof(St)));
    }
    if (extra) {
#pragma unroll
      for (int rr = 0; rr < SB; ++rr) {
        const int r = r0 + rr;
        const int64_t row = (int64_t)(y0 + r + 1) * pitch;
        A v = acc_sub(ca_s[TW + r + 1], cb_s[TW + TH - 1 - r]);
        acc_add_local(v, laN_s[r] - ob_s[NW][64 + r]);   // diagonal: the last strip's edge sum
        if (kSplit) S[2 * (row + N) + 1] = (St)to_store(v);
        else if (IL) ((g_ptr<St2>)I.S)[row + N] = St2{sN_s[r], (St)to_store(v)};
        else T[row + N] = to_store(v);
      }
    }
  };
  // pipeline: the labels of the sub-band after next and the densities
  // (table lookups) of the next one are in flight while a sub-band is done
  float dnext[4];
  stg.values(I, dnext);
  if (SB < TH) stg.load(I, x0, y0 + SB);
  // Per sub-band: the exclusive row prefixes into LDS, a barrier, the
  // sweep; T of the previous sub-band needs its strip-edge sums, written by
  // all wavefronts before a barrier.  Two barriers: T of the previous
  // sub-band first, then the scan, barrier, sweep, barrier.  One barrier
  // (ONE): the prefixes alternate between two buffers (the other one may
  // still be read by a slower wavefront's sweep of the sub-band before),
  // and T of the previous sub-band comes after the scan's barrier.
  for (int r0 = 0; r0 < TH; r0 += SB) {
    Lc (*const Pb)[PP] = Pn[ONE ? (r0 / SB) & 1 : 0];
    float dv[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) dv[e] = dnext[e];
    if (r0 + SB < TH) {
      stg.values(I, dnext);
      if (r0 + 2 * SB < TH) stg.load(I, x0, y0 + r0 + 2 * SB);
    }
    if (!ONE && r0 > 0) t_pass(r0 - SB);
    {   // each row scanned by one segment of a wavefront
      Lc loc = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) loc += (Lc)dv[e];
      const Lc x = seg_inclusive_scan_dpp<Stage::LPR>(loc);
      Lc run = x - loc, pv[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        pv[e] = run;
        run += (Lc)dv[e];
      }
      store4(&Pb[stg.g][4 * stg.li], pv);
      if (stg.li == Stage::LPR - 1) Pb[stg.g][TW] = x;   // the row total
    }
    __syncthreads();
    if (ONE && r0 > 0) t_pass(r0 - SB);
#pragma unroll
    for (int rr = 0; rr < SB; ++rr) {
      const int r = r0 + rr, j = y0 + r + 1;
      const Lc p0 = Pb[rr][t], p1 = Pb[rr][t + 1];
      const Lc m = (Lc)0.5 * (p0 + p1);                        // Mloc at this column
      acc_addv(sb, rc_s[r]);
      rsum += p0;                                              // Rloc at node column i
      A v = sb;
      acc_add_local(v, rsum);
      sv[rr] = (St)to_store(v);
      if (!IL) bstore(sv[rr], s_rs, i * (int)sizeof(St), (int)(j * pitch * (int64_t)sizeof(St)));
      else if (kSplit) bstore(sv[rr], s_rs, i * (int)sizeof(St2), (int)(j * pitch * (int64_t)sizeof(St2)));
      // anti-diagonals move one lane left; the last strip's lane 63 takes
      // the line arriving from the right tile (its part there: the row
      // totals of the rows done plus the right tile's mass below it)
      Lc ia = take_right(ra);
      if (w == NW - 1) {
        const Lc e = r > 0 ? rpre + ea_s[r - 1] : (Lc)0;
        ia = lane == 63 ? e : ia;
        rpre += Pb[rr][TW];
      }
      ra = ia + m;
      if (lane == 0) oa_s[w][64 + r] = ra;
      // diagonals: the line at this column after row r, then one lane
      // right; strip 0's lane 0 takes the line arriving from the left tile
      const Lc z = rb + m;
      if (lane == 63) ob_s[w + 1][64 + r] = z;
      Lc ib = take_left(z);
      if (w == 0) ib = lane == 0 ? eb_s[r] : ib;
      rb = ib;
      dl[rr] = ra - rb;
    }
    if (extra) {
#pragma unroll
      for (int rr = 0; rr < SB; ++rr) {
        const int r = r0 + rr, j = y0 + r + 1;
        acc_addv(sbN, rc_s[r]);
        rsumN += Pb[rr][TW];                                   // column N: the whole row lies left of it
        laN_s[r] = rsumN;                                      // its anti-diagonal: the rows' totals
        A v = sbN;
        acc_add_local(v, rsumN);
        const St sN = (St)to_store(v);
        if (!IL) S[(int64_t)j * pitch + N] = sN;
        else if (kSplit) S[2 * ((int64_t)j * pitch + N)] = sN;
        else sN_s[r] = sN;
      }
    }
    if (!ONE) __syncthreads();
  }
  if (ONE) __syncthreads();
  t_pass(TH - SB);
}

// host launchers --------------------------------------------------------------

template <int P, int TW, int TH>
static void launch_sat_t(const Batch& B, bool dense, bool il, int64_t tiles, int64_t c1, int64_t c2,
                         hipStream_t s, StageHook h, void* u) {
  auto hk = [&](int st, int after) { if (h) h(st, after, u); };
  hk(ST_SAT_REDUCE, 0);
  if (dense) hipLaunchKernelGGL((k_sat_reduce<P, TW, TH, true>), dim3(tiles), dim3(TW), 0, s, B);
  else hipLaunchKernelGGL((k_sat_reduce<P, TW, TH, false>), dim3(tiles), dim3(TW), 0, s, B);
  hk(ST_SAT_REDUCE, 1);
  // the carry pass builds the tile-row prefix totals in LDS when every
  // instance's table fits; otherwise the row-carry pass writes them
  const SatLayout Lm = sat_layout(B.max_n, TW, TH);
  const bool pref_lds = Lm.nty <= 256 && (int64_t)Lm.nty * (Lm.ntx + 1) <= kPrefLds;
  if (!pref_lds) {
    hk(ST_SAT_CARRY1, 0);
    hipLaunchKernelGGL((k_sat_carry1<P, TW, TH>), dim3(c1), dim3(256), 0, s, B);
    hk(ST_SAT_CARRY1, 1);
  }
  hk(ST_SAT_CARRY2, 0);
  if (pref_lds) hipLaunchKernelGGL((k_sat_carry2<P, TW, TH, true>), dim3(c2), dim3(256), 0, s, B);
  else hipLaunchKernelGGL((k_sat_carry2<P, TW, TH, false>), dim3(c2), dim3(256), 0, s, B);
  hk(ST_SAT_CARRY2, 1);
  hk(ST_SAT_FINAL, 0);
  if (dense) hipLaunchKernelGGL((k_sat_final<P, TW, TH, true, false>), dim3(tiles), dim3(TW), 0, s, B);
  else if (il) hipLaunchKernelGGL((k_sat_final<P, TW, TH, false, true>), dim3(tiles), dim3(TW), 0, s, B);
  else hipLaunchKernelGGL((k_sat_final<P, TW, TH, false, false>), dim3(tiles), dim3(TW), 0, s, B);
  hk(ST_SAT_FINAL, 1);
}

template <int P>
static bool launch_sat_p(const Batch& B, int tw, int th, bool dense, bool il, int64_t tiles, int64_t c1,
                         int64_t c2, hipStream_t s, StageHook h, void* u) {
  if (tw == 64 && th == 16) launch_sat_t<P, 64, 16>(B, dense, il, tiles, c1, c2, s, h, u);
  else if (tw == 128 && th == 16) launch_sat_t<P, 128, 16>(B, dense, il, tiles, c1, c2, s, h, u);
  else if (tw == 128 && th == 32) launch_sat_t<P, 128, 32>(B, dense, il, tiles, c1, c2, s, h, u);
  else if (tw == 256 && th == 32) launch_sat_t<P, 256, 32>(B, dense, il, tiles, c1, c2, s, h, u);
  else if (tw == 256 && th == 64) launch_sat_t<P, 256, 64>(B, dense, il, tiles, c1, c2, s, h, u);
  else return false;
  return true;
}

bool launch_sat(const Batch& B, int prec, int tw, int th, bool dense, bool il, int64_t tiles, int64_t c1,
                int64_t c2, hipStream_t s, StageHook h, void* u) {
  if (prec == CG_F32) return launch_sat_p<CG_F32>(B, tw, th, dense, il, tiles, c1, c2, s, h, u);
  if (prec == CG_COMP) return launch_sat_p<CG_COMP>(B, tw, th, dense, il, tiles, c1, c2, s, h, u);
  if (prec == CG_F64) return launch_sat_p<CG_F64>(B, tw, th, dense, il, tiles, c1, c2, s, h, u);
  if (prec == CG_F64ACC) return launch_sat_p<CG_F64ACC>(B, tw, th, dense, il, tiles, c1, c2, s, h, u);
  return false;
}

bool sat_shape_supported(int tw, int th) {
  return (tw == 64 && th == 16) || (tw == 128 && th == 16) || (tw == 128 && th == 32) ||
         (tw == 256 && th == 32) || (tw == 256 && th == 64);
}

}  // namespace cgk
