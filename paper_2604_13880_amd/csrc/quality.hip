// Geographic-distortion measures of a cartogram against its original map
// (paper: Background, "Quality Measures"):
//   * topology distortion tau = 1 - |E_c n E_m| / |E_c u E_m| over the
//     region adjacencies of the two rasters (regions whose pixels share a
//     pixel side; the background is not a region);
//   * shape distortion of every region: the symmetric difference of its
//     pixel sets in the two rasters over their union, minimised over all
//     translations by whole pixels (the cartogram's set moved);
//   * relative position error R: the mean absolute angle between the
//     vectors joining region barycentres in the cartogram and in the map,
//     over ordered pairs, divided by pi.
//
// GPU design.  One pass over each label map finds every region's bounding
// box (atomics only where a run of equal labels starts or ends) and sets
// the bit of every adjacent region pair in an (R+1)^2 bitmap (an atomic OR
// only when the bit is not yet seen).  Each region's pixel set is then
// packed into 64-bit rows of its bounding box (one wavefront ballot per
// word).  The best overlap over translations is an exact integer search:
// the overlap of a translation is a sum of popcounts of ANDed, shifted bit
// rows; a translation is skipped when an upper bound of its overlap (the
// row-count and column-count overlaps, min over the rows / columns) does
// not exceed the best overlap found so far, which starts from the
// translations that align the two pixel centroids.  Skipping never changes
// the maximum, so the result equals the full search.  Barycentres and the
// pair angles are FP64 sums in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "cg.h"
#include "host.h"

using cgh::align_up;
using cgh::fail;

namespace cgq {

constexpr int kMaxRegions = 4095;     // adjacency bitmap of (R+1)^2 bits: 2 MiB per raster
constexpr int kSmWords = 6144;        // bit images kept in LDS when both fit (48 KiB)
constexpr int64_t kWorkPerBlock = (int64_t)1 << 21;   // word operations a search block is sized for

// Bit images and bounds of one region (offsets in words of the shared buffers).
struct QReg {
  int32_t ha, wa, Wa, hb, wb, Wb;   // rows, columns, 64-bit words per row: map (a), cartogram (b)
  int32_t ax0, ay0, bx0, by0;       // bounding-box origins in the label maps
  int64_t abits, bbits;             // word offsets of the bit images
  int64_t prof;                     // int32 offset of ra[ha], rb[hb], ca[wa], cb[wb]
  int64_t uoff, voff;               // int32 offsets of U[ha+hb-1], V[wa+wb-1]
};

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}
// Block (256 threads) sums: lane exchanges within each wavefront, then the
// four wavefront totals in a fixed order.
__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* red) {
  v = wave_sum_i64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const int64_t r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_sum_f64(double v, double* red) {
  v = wave_sum_f64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max_f64(double v, double* red) {
  v = wave_max_f64(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return r;
}

// Empty bounding boxes, cleared bitmaps and overlaps.
__global__ __launch_bounds__(256) void k_q_init(int4* box, int nbox, uint32_t* bits, int64_t nwords, uint32_t* best,
                                                int nbest, uint32_t* err) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x, stride = (int64_t)gridDim.x * 256;
  for (int64_t i = g; i < nbox; i += stride) box[i] = make_int4(INT32_MAX, INT32_MAX, -1, -1);
  for (int64_t i = g; i < nwords; i += stride) bits[i] = 0u;
  for (int64_t i = g; i < nbest; i += stride) best[i] = 0u;
  if (g == 0) *err = 0u;
}

__device__ __forceinline__ void set_pair(uint32_t* bits, int R, int a, int b) {
  const int u = min(a, b), v = max(a, b);
  const int64_t bit = (int64_t)u * (R + 1) + v;
  uint32_t* w = bits + (bit >> 5);
  const uint32_t m = 1u << (bit & 31);
  if ((__atomic_load_n(w, __ATOMIC_RELAXED) & m) == 0u) atomicOr(w, m);
}

// One pass over a label map (blockIdx.y = 0: map, 1: cartogram): bounding
// boxes from the runs of equal labels and the adjacency bitmap.  A thread
// takes 8 pixels of a row and the 8 below them.
__global__ __launch_bounds__(256) void k_q_scan(const uint16_t* lab0, const uint16_t* lab1, int N, int R, int4* box,
                                                uint32_t* bits, int64_t nwords, uint32_t* err) {
  const int r = blockIdx.y;
  const uint16_t* lab = r ? lab1 : lab0;
  int4* bx = box + (size_t)r * (R + 1);
  uint32_t* bm = bits + (size_t)r * nwords;
  const int chunks = N >> 3;
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (g >= (int64_t)N * chunks) return;
  const int q = (int)(g / chunks), p0 = (int)(g % chunks) * 8;
  const uint16_t* row = lab + (size_t)q * N;
  uint16_t v[8], dn[8];
  {
    const uint4 a = *(const uint4*)(row + p0);
    memcpy(v, &a, 16);
    if (q + 1 < N) {
      const uint4 b = *(const uint4*)(row + N + p0);
      memcpy(dn, &b, 16);
    } else {
      for (int i = 0; i < 8; ++i) dn[i] = 0;
    }
  }
  const int left = p0 > 0 ? row[p0 - 1] : 0;
  const int right = p0 + 8 < N ? row[p0 + 8] : 0;
  for (int i = 0; i < 8; ++i) {
    const int a = v[i];
    if (a == 0) continue;
    if (a > R) {
      atomicOr(err, 1u);
      continue;
    }
    const int prev = i ? v[i - 1] : left;
    const int next = i < 7 ? v[i + 1] : right;
    const int p = p0 + i;
    if (prev != a) {
      atomicMin(&bx[a].x, p);
      atomicMin(&bx[a].y, q);
      atomicMax(&bx[a].w, q);
    }
    if (next != a) {
      atomicMax(&bx[a].z, p);
      if (next > 0 && next <= R) set_pair(bm, R, a, next);
    }
    const int c = dn[i];
    if (c != a && c > 0 && c <= R) set_pair(bm, R, a, c);
  }
}

// Bit images: word w of row y of region v's image (map or cartogram) holds
// pixels x0 + 64 w + l, l = 0..63, of label-map row y0 + y; one wavefront
// per word (ballot).  seg[2(v-1)] / seg[2(v-1)+1] are the first words of
// v's map / cartogram image, seg[2R] the total.
__global__ __launch_bounds__(256) void k_q_pack(const uint16_t* lab0, const uint16_t* lab1, int N, int R,
                                                const QReg* regs, const int64_t* seg, uint64_t* out) {
  const int lane = threadIdx.x & 63;
  const int64_t word = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t total = seg[2 * R];
  if (word >= total) return;
  int lo = 0, hi = 2 * R;   // seg[lo] <= word < seg[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (seg[mid] <= word) lo = mid; else hi = mid;
  }
  const int v = 1 + (lo >> 1), r = lo & 1;
  const QReg g = regs[v];
  const int W = r ? g.Wb : g.Wa, w = r ? g.wb : g.wa;
  const int x0 = r ? g.bx0 : g.ax0, y0 = r ? g.by0 : g.ay0;
  const int64_t k = word - seg[lo];
  const int y = (int)(k / W), wi = (int)(k % W);
  const int xr = 64 * wi + lane;
  const uint16_t* lab = r ? lab1 : lab0;
  const bool in = xr < w && lab[(size_t)(y0 + y) * N + x0 + xr] == v;
  const uint64_t m = __ballot(in);
  if (lane == 0) out[(r ? g.bbits : g.abits) + k] = m;
}

// Overlap |A n (B + (dy, dx))|: pixel (yb, xb) of B lies on pixel
// (yb + dy, xb + dx) of A (bounding-box coordinates).
__device__ __forceinline__ uint32_t overlap_at(const uint64_t* A, int ha, int wa, int Wa, const uint64_t* B, int hb,
                                               int wb, int Wb, int dy, int dx) {
  const int y0 = max(0, dy), y1 = min(ha, hb + dy);
  const int x0 = max(0, dx), x1 = min(wa, wb + dx);
  if (y0 >= y1 || x0 >= x1) return 0u;
  const int w0 = x0 >> 6, w1 = (x1 - 1) >> 6;
  uint32_t c = 0;
  for (int y = y0; y < y1; ++y) {
    const uint64_t* ar = A + (size_t)y * Wa;
    const uint64_t* br = B + (size_t)(y - dy) * Wb;
    for (int w = w0; w <= w1; ++w) {
      const int s = 64 * w - dx;   // B column under A column 64 w
      const int q = s >> 6, sh = s & 63;
      const uint64_t lo = (q >= 0 && q < Wb) ? br[q] : 0ull;
      const uint64_t hi = (q + 1 >= 0 && q + 1 < Wb) ? br[q + 1] : 0ull;
      const uint64_t bb = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
      c += (uint32_t)__popcll(ar[w] & bb);
    }
  }
  return c;
}

// Per region (one block): pixel counts, row and column counts, the bounds
// U(dy) = sum_y min(ra[y], rb[y - dy]) and V(dx) likewise over columns, and
// the overlap at the 3 x 3 translations around the one that aligns the two
// pixel centroids (the search's starting best).
__global__ __launch_bounds__(256) void k_q_bound(const QReg* regs, const uint64_t* bits, int32_t* prof, int32_t* UV,
                                                 uint32_t* best, int64_t* pixels, int R) {
  const int v = 1 + blockIdx.x;
  const int t = threadIdx.x;
  const QReg g = regs[v];
  __shared__ int64_t red[4];
  __shared__ double redd[4];
  const uint64_t* A = bits + g.abits;
  const uint64_t* B = bits + g.bbits;
  int32_t* ra = prof + g.prof;
  int32_t* rb = ra + g.ha;
  int32_t* ca = rb + g.hb;
  int32_t* cb = ca + g.wa;
  int64_t na = 0, nb = 0;
  double sya = 0, syb = 0, sxa = 0, sxb = 0;
  for (int y = t; y < g.ha; y += 256) {
    int c = 0;
    for (int w = 0; w < g.Wa; ++w) c += __popcll(A[(size_t)y * g.Wa + w]);
    ra[y] = c;
    na += c;
    sya += (double)y * c;
  }
  for (int y = t; y < g.hb; y += 256) {
    int c = 0;
    for (int w = 0; w < g.Wb; ++w) c += __popcll(B[(size_t)y * g.Wb + w]);
    rb[y] = c;
    nb += c;
    syb += (double)y * c;
  }
  for (int x = t; x < g.wa; x += 256) {
    int c = 0;
    for (int y = 0; y < g.ha; ++y) c += (int)((A[(size_t)y * g.Wa + (x >> 6)] >> (x & 63)) & 1ull);
    ca[x] = c;
    sxa += (double)x * c;
  }
  for (int x = t; x < g.wb; x += 256) {
    int c = 0;
    for (int y = 0; y < g.hb; ++y) c += (int)((B[(size_t)y * g.Wb + (x >> 6)] >> (x & 63)) & 1ull);
    cb[x] = c;
    sxb += (double)x * c;
  }
  na = block_sum_i64(na, red);
  nb = block_sum_i64(nb, red);
  sya = block_sum_f64(sya, redd);
  syb = block_sum_f64(syb, redd);
  sxa = block_sum_f64(sxa, redd);
  sxb = block_sum_f64(sxb, redd);
  if (t == 0) {
    pixels[v] = na;
    pixels[R + 1 + v] = nb;
  }
  if (na == 0 || nb == 0) return;   // uniform: no overlap is possible
  __syncthreads();                  // row and column counts visible to the block
  const int ndy = g.ha + g.hb - 1, ndx = g.wa + g.wb - 1;
  int32_t* U = UV + g.uoff;
  int32_t* V = UV + g.voff;
  for (int i = t; i < ndy; i += 256) {
    const int dy = i - (g.hb - 1);
    int s = 0;
    for (int y = max(0, dy); y < min(g.ha, g.hb + dy); ++y) s += min(ra[y], rb[y - dy]);
    U[i] = s;
  }
  for (int i = t; i < ndx; i += 256) {
    const int dx = i - (g.wb - 1);
    int s = 0;
    for (int x = max(0, dx); x < min(g.wa, g.wb + dx); ++x) s += min(ca[x], cb[x - dx]);
    V[i] = s;
  }
  // starting best: translations around the centroid alignment
  const int dyc = (int)rint(sya / (double)na - syb / (double)nb);
  const int dxc = (int)rint(sxa / (double)na - sxb / (double)nb);
  int64_t top = 0;
  for (int c = 0; c < 9; ++c) {
    const int dy = min(max(dyc + c / 3 - 1, -(g.hb - 1)), g.ha - 1);
    const int dx = min(max(dxc + c % 3 - 1, -(g.wb - 1)), g.wa - 1);
    const int y0 = max(0, dy), y1 = min(g.ha, g.hb + dy);
    const int x0 = max(0, dx), x1 = min(g.wa, g.wb + dx);
    int64_t o = 0;
    if (y0 < y1 && x0 < x1) {
      const int w0 = x0 >> 6, nw = ((x1 - 1) >> 6) - w0 + 1;
      const int64_t n = (int64_t)(y1 - y0) * nw;
      for (int64_t i = t; i < n; i += 256) {
        const int y = y0 + (int)(i / nw), w = w0 + (int)(i % nw);
        const int s = 64 * w - dx;
        const int q = s >> 6, sh = s & 63;
        const uint64_t* br = B + (size_t)(y - dy) * g.Wb;
        const uint64_t lo = (q >= 0 && q < g.Wb) ? br[q] : 0ull;
        const uint64_t hi = (q + 1 >= 0 && q + 1 < g.Wb) ? br[q + 1] : 0ull;
        const uint64_t bb = sh ? ((lo >> sh) | (hi << (64 - sh))) : lo;
        o += __popcll(A[(size_t)y * g.Wa + w] & bb);
      }
    }
    o = block_sum_i64(o, red);
    top = max(top, o);
  }
  if (t == 0) atomicMax(best + v, (uint32_t)top);
}

// Exhaustive translation search of one region over the rows [lo, hi) of
// its dy range (work item (v, lo, hi)); translations whose bound does not
// exceed the best overlap found so far are skipped.
__global__ __launch_bounds__(256) void k_q_search(const QReg* regs, const int4* work, const uint64_t* bits,
                                                  const int32_t* UV, uint32_t* best) {
  const int4 wk = work[blockIdx.x];
  const int v = wk.x;
  const QReg g = regs[v];
  __shared__ uint64_t sm[kSmWords];
  __shared__ uint32_t sbest;
  const uint64_t* A = bits + g.abits;
  const uint64_t* B = bits + g.bbits;
  const int t = threadIdx.x;
  const int64_t nA = (int64_t)g.ha * g.Wa, nB = (int64_t)g.hb * g.Wb;
  if (nA + nB <= kSmWords) {
    for (int i = t; i < nA; i += 256) sm[i] = A[i];
    for (int i = t; i < nB; i += 256) sm[nA + i] = B[i];
    A = sm;
    B = sm + nA;
  }
  if (t == 0) sbest = __atomic_load_n(best + v, __ATOMIC_RELAXED);
  __syncthreads();
  const int32_t* U = UV + g.uoff;
  const int32_t* V = UV + g.voff;
  const int ndx = g.wa + g.wb - 1;
  uint32_t mine = 0;
  for (int iy = wk.y; iy < wk.z; ++iy) {
    const uint32_t cur = sbest;
    if ((uint32_t)U[iy] > cur) {
      const int dy = iy - (g.hb - 1);
      for (int ix = t; ix < ndx; ix += 256)
        if ((uint32_t)V[ix] > cur)
          mine = max(mine, overlap_at(A, g.ha, g.wa, g.Wa, B, g.hb, g.wb, g.Wb, dy, ix - (g.wb - 1)));
    }
    const uint32_t wm = wave_max_u32(mine);
    if ((t & 63) == 0 && wm > cur) atomicMax(&sbest, wm);
    __syncthreads();
  }
  if (t == 0) atomicMax(best + v, sbest);
}

// Barycentre of every region in both position sets (grid R x 2): the
// first moments of its rings over their signed area, as FP64 sums.
__global__ __launch_bounds__(256) void k_q_bary(const int32_t* reg_pair_off, const int2* reg_pairs, const float2* xy0,
                                                const float2* xy1, double* bary, int R) {
#pragma clang fp contract(off)   // the moments' products rounded one by one, as in a plain evaluation
  const int v = 1 + blockIdx.x, r = blockIdx.y;
  const float2* xy = r ? xy1 : xy0;
  __shared__ double red[4];
  double s0 = 0, sx = 0, sy = 0;
  for (int e = reg_pair_off[v - 1] + threadIdx.x; e < reg_pair_off[v]; e += 256) {
    const int2 pr = reg_pairs[e];
    const float2 a = xy[pr.x], b = xy[pr.y];
    const double c = (double)a.x * (double)b.y - (double)b.x * (double)a.y;
    s0 += c;
    sx += ((double)a.x + (double)b.x) * c;
    sy += ((double)a.y + (double)b.y) * c;
  }
  s0 = block_sum_f64(s0, red);
  sx = block_sum_f64(sx, red);
  sy = block_sum_f64(sy, red);
  if (threadIdx.x == 0) {
    double* o = bary + ((size_t)r * (R + 1) + v) * 2;
    o[0] = sx / (3.0 * s0);
    o[1] = sy / (3.0 * s0);
  }
}

// Sum over v != u of |angle(b_c(u,v), b_m(u,v))| for u = 1 + blockIdx.x.
__global__ __launch_bounds__(256) void k_q_relpos(const double* bary, int R, double* part) {
#pragma clang fp contract(off)   // products rounded one by one: equal vectors give an exact 0 angle
  const int u = 1 + blockIdx.x;
  __shared__ double red[4];
  const double* bm = bary;
  const double* bc = bary + (size_t)(R + 1) * 2;
  double s = 0;
  for (int v = 1 + threadIdx.x; v <= R; v += 256) {
    if (v == u) continue;
    const double mx = bm[2 * v] - bm[2 * u], my = bm[2 * v + 1] - bm[2 * u + 1];
    const double cx = bc[2 * v] - bc[2 * u], cy = bc[2 * v + 1] - bc[2 * u + 1];
    s += fabs(atan2(mx * cy - my * cx, mx * cx + my * cy));
  }
  s = block_sum_f64(s, red);
  if (threadIdx.x == 0) part[u] = s;
}

// tau, per-region shape distortion, its mean and max, R (one block).
__global__ __launch_bounds__(256) void k_q_final(const uint32_t* bits, int64_t nwords, const uint32_t* best,
                                                 const int64_t* pixels, const double* part, int R, int64_t* adjacency,
                                                 int64_t* overlap, double* shape, double* summary) {
  const int t = threadIdx.x;
  __shared__ int64_t red[4];
  __shared__ double redd[4];
  int64_t em = 0, ec = 0, both = 0;
  for (int64_t i = t; i < nwords; i += 256) {
    const uint32_t a = bits[i], b = bits[nwords + i];
    em += __popc(a);
    ec += __popc(b);
    both += __popc(a & b);
  }
  em = block_sum_i64(em, red);
  ec = block_sum_i64(ec, red);
  both = block_sum_i64(both, red);
  double hs = 0, hm = 0;
  for (int v = t; v <= R; v += 256) {
    const int64_t o = v ? (int64_t)best[v] : 0;
    const int64_t na = pixels[v], nb = pixels[R + 1 + v];
    const int64_t un = na + nb - o;
    const double h = (v == 0 || un == 0) ? 0.0 : (double)(na + nb - 2 * o) / (double)un;
    overlap[v] = o;
    shape[v] = h;
    if (v) {
      hs += h;
      hm = fmax(hm, h);
    }
  }
  hs = block_sum_f64(hs, redd);
  hm = block_max_f64(hm, redd);
  if (t != 0) return;
  const int64_t un = em + ec - both;
  double rp = 0;
  for (int u = 1; u <= R; ++u) rp += part[u];
  adjacency[0] = em;
  adjacency[1] = ec;
  adjacency[2] = both;
  summary[0] = un ? 1.0 - (double)both / (double)un : 0.0;
  summary[1] = R ? hs / R : 0.0;
  summary[2] = hm;
  summary[3] = R > 1 ? rp / (3.141592653589793 * (double)R * (double)(R - 1)) : 0.0;
}

}  // namespace cgq

extern "C" int cg_quality(cg_ctx* c, const cg_map* map, int N, const uint16_t* labels_map,
                          const uint16_t* labels_cart, const float* xy_map, const float* xy_cart,
                          cg_quality_out* out, void* stream) {
  using namespace cgq;
  if (!c) return CG_EINVAL;
  if (!map || !labels_map || !labels_cart || !xy_map || !xy_cart || !out)
    return fail(c, CG_EINVAL, "cg_quality: null argument");
  if (!out->adjacency || !out->overlap || !out->pixels || !out->shape || !out->summary)
    return fail(c, CG_EINVAL, "cg_quality: null output array");
  if (!cgh::pow2_ok(N)) return fail(c, CG_EINVAL, "cg_quality: N must be a power of two in [16, 8192]");
  if ((((uintptr_t)labels_map) | ((uintptr_t)labels_cart)) & 15)
    return fail(c, CG_EINVAL, "cg_quality: label maps must be 16-byte aligned");
  const int R = map->R;
  if (R < 1 || R > kMaxRegions)
    return fail(c, CG_EUNSUPPORTED, "cg_quality: needs 1 <= R <= " + std::to_string(kMaxRegions));
  hipSetDevice(c->device);
  hipStream_t st = cgh::pick_stream(c, stream);
  const int64_t nwords = ((int64_t)(R + 1) * (R + 1) + 31) / 32;
  // scratch: boxes [2][R+1], bitmaps [2][nwords], best [R+1], error word,
  // pixel counts [2][R+1], angle partials [R+1], barycentres [2][R+1][2]
  const size_t o_box = 0;
  const size_t o_bits = o_box + align_up(sizeof(int4) * 2 * (R + 1));
  const size_t o_best = o_bits + align_up(sizeof(uint32_t) * 2 * nwords);
  const size_t o_err = o_best + align_up(sizeof(uint32_t) * (R + 1));
  const size_t o_pix = o_err + align_up(sizeof(uint32_t));
  const size_t o_part = o_pix + align_up(sizeof(int64_t) * 2 * (R + 1));
  const size_t o_bary = o_part + align_up(sizeof(double) * (R + 1));
  const size_t fixed = o_bary + align_up(sizeof(double) * 4 * (R + 1));
  char* ws = nullptr;
  int rc = cgh::get_buf(c, "quality:fixed", fixed, st, &ws);
  if (rc) return rc;
  int4* d_box = (int4*)(ws + o_box);
  uint32_t* d_bits = (uint32_t*)(ws + o_bits);
  uint32_t* d_best = (uint32_t*)(ws + o_best);
  uint32_t* d_err = (uint32_t*)(ws + o_err);
  int64_t* d_pix = (int64_t*)(ws + o_pix);
  double* d_part = (double*)(ws + o_part);
  double* d_bary = out->bary ? out->bary : (double*)(ws + o_bary);
  {
    const int64_t n = std::max<int64_t>(2 * nwords, 2 * (R + 1));
    const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(k_q_init, dim3(blocks), dim3(256), 0, st, d_box, 2 * (R + 1), d_bits, 2 * nwords, d_best,
                       R + 1, d_err);
    const int64_t chunks = (int64_t)N * N / 8;
    hipLaunchKernelGGL(k_q_scan, dim3((unsigned)((chunks + 255) / 256), 2), dim3(256), 0, st, labels_map,
                       labels_cart, N, R, d_box, d_bits, nwords, d_err);
  }
  std::vector<int4> box(2 * (R + 1));
  uint32_t err = 0;
  HIP_OK(c, hipMemcpyAsync(box.data(), d_box, sizeof(int4) * box.size(), hipMemcpyDeviceToHost, st));
  HIP_OK(c, hipMemcpyAsync(&err, d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
  HIP_OK(c, hipStreamSynchronize(st));
  if (err) return fail(c, CG_EINVAL, "cg_quality: a label map holds a label above the map's region count");
  // layout of the bit images, counts and bounds; search work items
  std::vector<QReg> regs(R + 1);
  std::vector<int64_t> seg(2 * R + 1);
  std::vector<int4> work;
  int64_t words = 0, prof = 0, uv = 0;
  for (int v = 1; v <= R; ++v) {
    QReg& g = regs[v];
    memset(&g, 0, sizeof(g));
    const int4 a = box[v], b = box[R + 1 + v];
    const bool ea = a.z < a.x, eb = b.z < b.x;
    g.ax0 = ea ? 0 : a.x;
    g.ay0 = ea ? 0 : a.y;
    g.wa = ea ? 0 : a.z - a.x + 1;
    g.ha = ea ? 0 : a.w - a.y + 1;
    g.bx0 = eb ? 0 : b.x;
    g.by0 = eb ? 0 : b.y;
    g.wb = eb ? 0 : b.z - b.x + 1;
    g.hb = eb ? 0 : b.w - b.y + 1;
    g.Wa = (g.wa + 63) / 64;
    g.Wb = (g.wb + 63) / 64;
    seg[2 * (v - 1)] = words;
    g.abits = words;
    words += (int64_t)g.ha * g.Wa;
    seg[2 * (v - 1) + 1] = words;
    g.bbits = words;
    words += (int64_t)g.hb * g.Wb;
    g.prof = prof;
    prof += g.ha + g.hb + g.wa + g.wb;
    if (!ea && !eb) {
      const int ndy = g.ha + g.hb - 1, ndx = g.wa + g.wb - 1;
      g.uoff = uv;
      uv += ndy;
      g.voff = uv;
      uv += ndx;
      const int64_t per_row = (int64_t)ndx * std::min(g.ha, g.hb) * (std::min(g.Wa, g.Wb) + 1);
      const int rows = (int)std::max<int64_t>(1, std::min<int64_t>(ndy, kWorkPerBlock / std::max<int64_t>(per_row, 1)));
      for (int lo = 0; lo < ndy; lo += rows) work.push_back(make_int4(v, lo, std::min(ndy, lo + rows), 0));
    }
  }
  seg[2 * R] = words;
  if (work.size() > (size_t)INT32_MAX) return fail(c, CG_EUNSUPPORTED, "cg_quality: search too large");
  const size_t o_regs = 0;
  const size_t o_seg = o_regs + align_up(sizeof(QReg) * regs.size());
  const size_t o_work = o_seg + align_up(sizeof(int64_t) * seg.size());
  const size_t o_words = o_work + align_up(sizeof(int4) * std::max<size_t>(1, work.size()));
  const size_t o_prof = o_words + align_up(sizeof(uint64_t) * std::max<int64_t>(1, words));
  const size_t o_uv = o_prof + align_up(sizeof(int32_t) * std::max<int64_t>(1, prof));
  const size_t dyn = o_uv + align_up(sizeof(int32_t) * std::max<int64_t>(1, uv));
  char* wd = nullptr;
  if ((rc = cgh::get_buf(c, "quality:images", dyn, st, &wd))) return rc;
  QReg* d_regs = (QReg*)(wd + o_regs);
  int64_t* d_seg = (int64_t*)(wd + o_seg);
  int4* d_work = (int4*)(wd + o_work);
  uint64_t* d_words = (uint64_t*)(wd + o_words);
  int32_t* d_prof = (int32_t*)(wd + o_prof);
  int32_t* d_uv = (int32_t*)(wd + o_uv);
  HIP_OK(c, hipMemcpyAsync(d_regs, regs.data(), sizeof(QReg) * regs.size(), hipMemcpyHostToDevice, st));
  HIP_OK(c, hipMemcpyAsync(d_seg, seg.data(), sizeof(int64_t) * seg.size(), hipMemcpyHostToDevice, st));
  if (!work.empty())
    HIP_OK(c, hipMemcpyAsync(d_work, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice, st));
  if (words > 0)
    hipLaunchKernelGGL(k_q_pack, dim3((unsigned)((words + 3) / 4)), dim3(256), 0, st, labels_map, labels_cart, N, R,
                       (const QReg*)d_regs, (const int64_t*)d_seg, d_words);
  hipLaunchKernelGGL(k_q_bound, dim3(R), dim3(256), 0, st, (const QReg*)d_regs, (const uint64_t*)d_words, d_prof,
                     d_uv, d_best, d_pix, R);
  if (!work.empty())
    hipLaunchKernelGGL(k_q_search, dim3((unsigned)work.size()), dim3(256), 0, st, (const QReg*)d_regs,
                       (const int4*)d_work, (const uint64_t*)d_words, (const int32_t*)d_uv, d_best);
  hipLaunchKernelGGL(k_q_bary, dim3(R, 2), dim3(256), 0, st, (const int32_t*)map->d_reg_pair_off,
                     (const int2*)map->d_reg_pairs, (const float2*)xy_map, (const float2*)xy_cart, d_bary, R);
  hipLaunchKernelGGL(k_q_relpos, dim3(R), dim3(256), 0, st, (const double*)d_bary, R, d_part);
  hipLaunchKernelGGL(k_q_final, dim3(1), dim3(256), 0, st, (const uint32_t*)d_bits, nwords, (const uint32_t*)d_best,
                     (const int64_t*)d_pix, (const double*)d_part, R, out->adjacency, out->overlap, out->shape,
                     out->summary);
  if (out->pixels)
    HIP_OK(c, hipMemcpyAsync(out->pixels, d_pix, sizeof(int64_t) * 2 * (R + 1), hipMemcpyDeviceToDevice, st));
  HIP_OK(c, hipGetLastError());
  // host tables above are read by the copies: finish before they go
  HIP_OK(c, hipStreamSynchronize(st));
  return CG_OK;
}
