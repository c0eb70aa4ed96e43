// Rasterisation of the region polygons into a label map and per-region
// pixel counts (paper: Method, Step 2 -- region area by pixel counting).
//
// Membership rule: a pixel centre belongs to region v when the number of
// v's boundary edges crossing the centre's row at or left of the centre is
// odd.  Coordinates are snapped to 1/256 pixel (X = rint(x*256N)); an edge
// crosses row q when exactly one endpoint has Y <= 256q+128; its first
// pixel p0 is the smallest p whose centre is at or right of the crossing.
// Every unique edge separates two regions (0 = outside), so one crossing
// toggles the membership of both.  Toggles commute, so a row only needs its
// crossings ordered by p0: walking them maintains the set of regions that
// claim the current run of pixels.  A run claimed by several regions (the
// map has folded) takes the highest id and is counted as contested.
//
// Kernels (one launch each per iteration, covering every instance):
//   k_raster_count  one thread per edge: crossings per row (int atomics)
//   k_raster_scan   one block per instance: row offsets, counter resets
//   k_raster_emit   one thread per edge: (p0, region A, region B) records
//   k_raster_fill   one wavefront per row: sort by p0, walk, write labels,
//                   per-region counts aggregated in LDS
#include "cg_dev.h"

namespace cgk {

constexpr int kFillRows = 4;      // rows per block (one wavefront each)
constexpr int kFillXing = 512;    // crossings per row held in LDS

__device__ __forceinline__ int snapc(float v, float scale) { return (int)rintf(v * scale); }

// rows q with lo <= 256q + 128 < hi
__device__ __forceinline__ void crossed_rows(int ya, int yb, int N, int& q0, int& q1) {
  int lo = min(ya, yb), hi = max(ya, yb);
  q0 = max((lo - kSub / 2 + kSub - 1) >> 8, 0);
  q1 = min((hi - kSub / 2 + kSub - 1) >> 8, N);
}

__global__ __launch_bounds__(256) void k_raster_count(Batch B) {
  const int k = find_inst(B.off_edges, B.n, blockIdx.x);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  const int64_t e = (int64_t)(blockIdx.x - B.off_edges[k]) * 256 + threadIdx.x;
  if (e >= I.n_edges) return;
  const int4 E = I.edges[e];
  const float scale = (float)(kSub * I.N);
  const int ya = snapc(I.xy[E.x].y, scale), yb = snapc(I.xy[E.y].y, scale);
  int q0, q1;
  crossed_rows(ya, yb, I.N, q0, q1);
  for (int q = q0; q < q1; ++q) atomicAdd(&I.row_cnt[q], 1u);
}

__global__ __launch_bounds__(1024) void k_raster_scan(Batch B) {
  const int k = find_inst(B.off_inst, B.n, blockIdx.x);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  __shared__ uint32_t wsum[16];
  const int N = I.N, t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int per = (N + 1023) / 1024;
  const int base = t * per;
  uint32_t loc[8];
  uint32_t sum = 0;
  for (int c = 0; c < per; ++c) {
    const int q = base + c;
    const uint32_t v = q < N ? I.row_cnt[q] : 0u;
    loc[c] = v;
    sum += v;
  }
  // block exclusive scan of the per-thread sums
  uint32_t x = sum;
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t wpre = 0, total = 0;
  for (int i = 0; i < 16; ++i) {
    if (i < w) wpre += wsum[i];
    total += wsum[i];
  }
  uint32_t run = wpre + x - sum;
  for (int c = 0; c < per; ++c) {
    const int q = base + c;
    if (q < N) {
      I.row_off[q] = run;
      I.row_cnt[q] = 0u;
    }
    run += loc[c];
  }
  if (t == 0) {
    I.row_off[N] = total;
    I.st->xings = total;
    I.st->contested = 0;
    if ((int64_t)total > I.xing_cap) atomicOr(&I.st->flags, CG_FLAG_OVERFLOW);
  }
  for (int v = t; v <= I.R; v += 1024) I.counts[v] = 0;
}

__global__ __launch_bounds__(256) void k_raster_emit(Batch B) {
  const int k = find_inst(B.off_edges, B.n, blockIdx.x);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  const int64_t e = (int64_t)(blockIdx.x - B.off_edges[k]) * 256 + threadIdx.x;
  if (e >= I.n_edges) return;
  const int4 E = I.edges[e];
  const int N = I.N;
  const float scale = (float)(kSub * N);
  const float2 pa = I.xy[E.x], pb = I.xy[E.y];
  int ax = snapc(pa.x, scale), ay = snapc(pa.y, scale);
  int bx = snapc(pb.x, scale), by = snapc(pb.y, scale);
  int q0, q1;
  crossed_rows(ay, by, N, q0, q1);
  if (q0 >= q1) return;
  if (ay > by) {  // orient so that dy > 0; the crossing abscissa is unchanged
    int tx = ax; ax = bx; bx = tx;
    int ty = ay; ay = by; by = ty;
  }
  const int64_t dy = by - ay, dx = bx - ax;
  const int64_t den = (int64_t)kSub * dy;
  const uint64_t regs = ((uint64_t)(uint16_t)E.z << 16) | ((uint64_t)(uint16_t)E.w << 32);
  for (int q = q0; q < q1; ++q) {
    const int64_t yc = (int64_t)kSub * q + kSub / 2;
    // centre p is at or right of the crossing iff 256 p dy >= num
    const int64_t num = (yc - ay) * dx - ((int64_t)(kSub / 2) - ax) * dy;
    int64_t p0 = num <= 0 ? 0 : (num + den - 1) / den;
    if (p0 > N) p0 = N;
    const uint32_t slot = I.row_off[q] + atomicAdd(&I.row_cnt[q], 1u);
    if ((int64_t)slot < I.xing_cap) I.xing[slot] = (uint64_t)p0 | regs;
  }
}

__device__ __forceinline__ void set_toggle(int* set, int& n, int r, bool& over) {
  if (r == 0) return;
  for (int i = 0; i < n; ++i) {
    if (set[i] == r) {
      set[i] = set[n - 1];
      --n;
      return;
    }
  }
  if (n < kSetCap) set[n++] = r; else over = true;
}

__global__ __launch_bounds__(256) void k_raster_fill(Batch B) {
  const int k = find_inst(B.off_rows, B.n, blockIdx.x);
  const Inst& I = B.inst[k];
  if (inst_done(B, I)) return;
  __shared__ uint64_t xs[kFillRows][kFillXing];
  __shared__ uint64_t srt[kFillRows][kFillXing];
  __shared__ uint16_t sp_start[kFillRows][kFillXing + 2];
  __shared__ uint16_t sp_lab[kFillRows][kFillXing + 2];
  __shared__ int sp_n[kFillRows];
  __shared__ uint32_t lcount[kLutLds];
  __shared__ unsigned long long contested_blk;
  const int N = I.N, R = I.R;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const bool lds_counts = (R + 1) <= kLutLds;
  if (lds_counts)
    for (int v = t; v <= R; v += 256) lcount[v] = 0u;
  if (t == 0) contested_blk = 0ull;
  const int q = (int)(blockIdx.x - B.off_rows[k]) * kFillRows + w;
  const bool row_ok = q < N;
  uint32_t cnt = 0, off = 0;
  bool bad = false;
  if (row_ok) {
    cnt = I.row_cnt[q];
    off = I.row_off[q];
    if (cnt > (uint32_t)kFillXing || (int64_t)off + cnt > I.xing_cap) bad = true;
  }
  if (row_ok && !bad) {
    for (uint32_t i = lane; i < cnt; i += 64) xs[w][i] = I.xing[off + i];
  }
  __syncthreads();
  if (row_ok && !bad) {
    // rank sort by (p0, slot): ranks are unique, so srt is a permutation
    for (uint32_t i = lane; i < cnt; i += 64) {
      const uint64_t a = xs[w][i];
      const uint32_t pa = (uint32_t)(a & 0xFFFFu);
      uint32_t rank = 0;
      for (uint32_t j = 0; j < cnt; ++j) {
        const uint32_t pj = (uint32_t)(xs[w][j] & 0xFFFFu);
        rank += (pj < pa) || (pj == pa && j < i);
      }
      srt[w][rank] = a;
    }
  }
  __syncthreads();
  if (row_ok && lane == 0) {
    int set[kSetCap];
    int ns = 0, nsp = 0;
    bool over = false;
    uint32_t prev = 0;
    unsigned long long cont = 0;
    if (!bad) {
      for (uint32_t i = 0; i <= cnt; ++i) {
        const uint32_t p0 = i < cnt ? (uint32_t)(srt[w][i] & 0xFFFFu) : (uint32_t)N;
        if (p0 > prev) {
          int lab = 0;
          for (int s = 0; s < ns; ++s) lab = max(lab, set[s]);
          sp_start[w][nsp] = (uint16_t)prev;
          sp_lab[w][nsp] = (uint16_t)lab;
          ++nsp;
          const uint32_t len = p0 - prev;
          if (ns > 1) cont += len;
          if (lds_counts) atomicAdd(&lcount[lab], len);
          else atomicAdd((unsigned long long*)&I.counts[lab], (unsigned long long)len);
          prev = p0;
        }
        if (i < cnt) {
          const uint64_t r = srt[w][i];
          set_toggle(set, ns, (int)((r >> 16) & 0xFFFFu), over);
          set_toggle(set, ns, (int)((r >> 32) & 0xFFFFu), over);
        }
      }
    } else {
      sp_start[w][0] = 0;
      sp_lab[w][0] = 0;
      nsp = 1;
      if (lds_counts) atomicAdd(&lcount[0], (uint32_t)N);
      else atomicAdd((unsigned long long*)&I.counts[0], (unsigned long long)N);
    }
    if (nsp == 0) {  // N == 0 cannot happen; keep the span list well formed
      sp_start[w][0] = 0;
      sp_lab[w][0] = 0;
      nsp = 1;
    }
    sp_n[w] = nsp;
    if (cont) atomicAdd(&contested_blk, cont);
    if (bad || over) atomicOr(&I.st->flags, CG_FLAG_OVERFLOW);
    if (cont) atomicOr(&I.st->flags, CG_FLAG_CONTESTED);
  }
  __syncthreads();
  if (row_ok) {
    // fill: lane handles 8 consecutive pixels per step
    const int nsp = sp_n[w];
    uint16_t* row = I.labels + (int64_t)q * N;
    for (int p = lane * 8; p < N; p += 64 * 8) {
      // span containing pixel p: last start <= p
      int lo = 0, hi = nsp;
      while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (sp_start[w][mid] <= p) lo = mid; else hi = mid;
      }
      uint16_t v[8];
      int s = lo;
      for (int c = 0; c < 8; ++c) {
        while (s + 1 < nsp && sp_start[w][s + 1] <= p + c) ++s;
        v[c] = sp_lab[w][s];
      }
      if (p + 8 <= N) {
        uint4 pk;
        pk.x = v[0] | ((uint32_t)v[1] << 16);
        pk.y = v[2] | ((uint32_t)v[3] << 16);
        pk.z = v[4] | ((uint32_t)v[5] << 16);
        pk.w = v[6] | ((uint32_t)v[7] << 16);
        *(uint4*)(row + p) = pk;
      } else {
        for (int c = 0; c < 8 && p + c < N; ++c) row[p + c] = v[c];
      }
    }
    if (lane == 0) I.row_cnt[q] = 0u;
  }
  __syncthreads();
  if (lds_counts) {
    for (int v = t; v <= R; v += 256)
      if (lcount[v]) atomicAdd((unsigned long long*)&I.counts[v], (unsigned long long)lcount[v]);
  }
  if (t == 0 && contested_blk) atomicAdd((unsigned long long*)&I.st->contested, contested_blk);
}

// host launchers --------------------------------------------------------------

void launch_raster(const Batch& B, int64_t edge_blocks, int64_t row_blocks, hipStream_t s, StageHook h,
                   void* u) {
  auto hk = [&](int st, int after) { if (h) h(st, after, u); };
  if (edge_blocks > 0) {
    hk(ST_RASTER_COUNT, 0);
    hipLaunchKernelGGL(k_raster_count, dim3(edge_blocks), dim3(256), 0, s, B);
    hk(ST_RASTER_COUNT, 1);
  }
  hk(ST_RASTER_SCAN, 0);
  hipLaunchKernelGGL(k_raster_scan, dim3(B.n), dim3(1024), 0, s, B);
  hk(ST_RASTER_SCAN, 1);
  if (edge_blocks > 0) {
    hk(ST_RASTER_EMIT, 0);
    hipLaunchKernelGGL(k_raster_emit, dim3(edge_blocks), dim3(256), 0, s, B);
    hk(ST_RASTER_EMIT, 1);
  }
  hk(ST_RASTER_FILL, 0);
  hipLaunchKernelGGL(k_raster_fill, dim3(row_blocks), dim3(256), 0, s, B);
  hk(ST_RASTER_FILL, 1);
}

}  // namespace cgk
