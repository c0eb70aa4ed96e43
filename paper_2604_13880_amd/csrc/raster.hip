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
//   k_raster_emit   one thread per edge: (p0, region A, region B) records
//                   appended to the bucket of every row the edge crosses
//                   (kFillXing records per row; an integer atomic per
//                   crossing picks the slot); in launches of single-edge
//                   blocks also a block that clears the fill's totals and
//                   one block per region for the previous iteration's areas
//   k_raster_fill   one wavefront per row: rank sort by p0, claim sets by
//                   lane scans, write labels, per-region counts aggregated
//                   in LDS; in those launches also a block for the previous
//                   iteration's stopping rule
#include "cg_dev.h"

namespace cgk {

__device__ __forceinline__ int snapc(float v, float scale) { return (int)rintf(v * scale); }

// rows q with lo <= 256q + 128 < hi
__device__ __forceinline__ void crossed_rows(int ya, int yb, int N, int& q0, int& q1) {
  int lo = min(ya, yb), hi = max(ya, yb);
  q0 = max((lo - kSub / 2 + kSub - 1) >> 8, 0);
  q1 = min((hi - kSub / 2 + kSub - 1) >> 8, N);
}

// One thread per EPT edges (e0 + 256 j): all their loads are issued before
// any is used, which shortens the chain of dependent loads per edge when a
// launch has many rounds of blocks.  TOT = 0: the instance's first block
// also clears the totals the fill accumulates.  TOT = 1, 2 (launches of
// single-edge blocks): every instance has R + 1 blocks more than its edges
// need: first the totals block, which clears the totals, then one block
// per region, which with TOT = 2 computes the region's area from the
// positions the previous iteration's mapping left (Step 7; the stopping
// rule of that iteration then runs inside the fill, and the iteration
// needs no launch of its own for either).  The totals block also records
// the flags as they are before the fill, which is what that rule reads.
template <int EPT, int TOT>
__global__ __launch_bounds__(256) void k_raster_emit(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_edges, KD_EDGES, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  int64_t bi = blockIdx.x - first;
  if (TOT == 0 && bi == 0) {
    for (int v = threadIdx.x; v <= I.R; v += 256) I.counts[v] = 0;
    if (threadIdx.x == 0) I.st->contested = 0;
  }
  if (TOT != 0) {
    if (bi == 0) {   // the totals block
      for (int v = threadIdx.x; v <= I.R; v += 256) I.counts[v] = 0;
      if (threadIdx.x == 0) {
        I.st->contested = 0;
        if (TOT == 2) I.st->flags_rule = I.st->flags;
      }
      return;
    }
    if (bi <= I.R) {   // region bi's area
      if (TOT == 2) {
        __shared__ double red[256];
        region_area(I, (int)bi, red);
      }
      return;
    }
    bi -= 1 + I.R;
  }
  const int64_t e0 = bi * (256 * EPT) + threadIdx.x;
  if (e0 >= I.n_edges) return;
  const int N = I.N;
  const float scale = (float)(kSub * N);
  int4 E[EPT];
  float2 pa[EPT], pb[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) E[j] = ld4(I.edges + min(e0 + 256 * j, (int64_t)I.n_edges - 1));
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    pa[j] = ld2(I.xy + E[j].x);
    pb[j] = ld2(I.xy + E[j].y);
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    if (e0 + 256 * j >= I.n_edges) break;
    int ax = snapc(pa[j].x, scale), ay = snapc(pa[j].y, scale);
    int bx = snapc(pb[j].x, scale), by = snapc(pb[j].y, scale);
    int q0, q1;
    crossed_rows(ay, by, N, q0, q1);
    if (q0 >= q1) continue;
    if (ay > by) {  // orient so that dy > 0; the crossing abscissa is unchanged
      int tx = ax; ax = bx; bx = tx;
      int ty = ay; ay = by; by = ty;
    }
    const int64_t dy = by - ay, dx = bx - ax;
    const int64_t den = (int64_t)kSub * dy;
    const uint64_t regs = ((uint64_t)(uint16_t)E[j].z << 16) | ((uint64_t)(uint16_t)E[j].w << 32);
    // rows in groups of 8: the group's slot claims are all in flight before
    // the first one is used (a stretched edge crosses many rows, and one
    // claim at a time made its thread the launch's longest chain)
    for (int qb = q0; qb < q1; qb += 8) {
      uint32_t slot[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        slot[u] = qb + u < q1 ? g_atomic_add(&I.row_cnt[qb + u], 1u) : (uint32_t)kFillXing;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int q = qb + u;
        if (q >= q1) break;
        const int64_t yc = (int64_t)kSub * q + kSub / 2;
        // centre p is at or right of the crossing iff 256 p dy >= num
        const int64_t num = (yc - ay) * dx - ((int64_t)(kSub / 2) - ax) * dy;
        int64_t p0 = num <= 0 ? 0 : (num + den - 1) / den;
        if (p0 > N) p0 = N;
        // a full bucket is the fill's overflow
        if (slot[u] < (uint32_t)kFillXing) I.xing[(int64_t)q * kFillXing + slot[u]] = (uint64_t)p0 | regs;
      }
    }
  }
}

// Claim set of the current pixel run.  The common case (at most one
// claiming region) is a single label `cur`; a run claimed by several regions
// switches to a small slot array kept in registers (every index is a
// compile-time constant after unrolling; 0 marks a free slot).
struct Claims {
  int cur;           // the claiming region while `multi` is false
  bool multi;
  int set[kSetCap];
};

__device__ __forceinline__ void claims_toggle(Claims& c, int r, bool& over) {
  if (r == 0) return;
  if (!c.multi) {
    if (c.cur == 0) { c.cur = r; return; }
    if (c.cur == r) { c.cur = 0; return; }
    c.multi = true;
#pragma unroll
    for (int i = 0; i < kSetCap; ++i) c.set[i] = 0;
    c.set[0] = c.cur;
  }
  bool found = false;
#pragma unroll
  for (int i = 0; i < kSetCap; ++i)
    if (c.set[i] == r) {
      c.set[i] = 0;
      found = true;
    }
  if (!found) {
    bool placed = false;
#pragma unroll
    for (int i = 0; i < kSetCap; ++i)
      if (!placed && c.set[i] == 0) {
        c.set[i] = r;
        placed = true;
      }
    if (!placed) over = true;
  }
  int n = 0, any = 0;
#pragma unroll
  for (int i = 0; i < kSetCap; ++i) {
    n += c.set[i] != 0;
    any = max(any, c.set[i]);
  }
  if (n <= 1) {  // back to a single claim
    c.multi = false;
    c.cur = any;
  }
}

// The set {a} (empty for a = 0) toggled by b and by c (0 toggles
// nothing) holds at most one region.
__device__ __forceinline__ bool single_claim_ok(uint32_t a, uint32_t b, uint32_t c) {
  const int na = a != 0u ? ((1 + (b == a) + (c == a)) & 1) : 0;
  const int nb = (b != 0u && b != a) ? ((1 + (c == b)) & 1) : 0;
  const int nc = (c != 0u && c != a && c != b) ? 1 : 0;
  return na + nb + nc <= 1;
}

__device__ __forceinline__ void claims_label(const Claims& c, int& lab, int& n) {
  if (!c.multi) {
    lab = c.cur;
    n = c.cur != 0;
    return;
  }
  lab = 0;
  n = 0;
#pragma unroll
  for (int i = 0; i < kSetCap; ++i) {
    lab = max(lab, c.set[i]);
    n += c.set[i] != 0;
  }
}

// Bitonic sort of one 32-bit key per lane over the first SZ lanes
// (ascending there; lanes beyond SZ sort among themselves).
template <int SZ>
__device__ __forceinline__ uint32_t bitonic_sort(uint32_t key, int lane) {
#pragma unroll
  for (int size = 2; size <= SZ; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const uint32_t other = (uint32_t)__shfl_xor((int)key, stride, 64);
      const bool up = (lane & size) == 0;      // ascending half of this bitonic sequence
      const bool low = (lane & stride) == 0;   // lower partner
      key = (up == low) ? min(key, other) : max(key, other);
    }
  }
  return key;
}

// Cross-lane moves by DPP (no LDS traffic).  wave_shr1: lane l reads lane
// l-1 (lane 0 reads `edge`); wave_shl1: lane l reads lane l+1 (lane 63
// reads `edge`).
__device__ __forceinline__ uint32_t wave_shr1(uint32_t v, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ uint32_t wave_shl1(uint32_t v, uint32_t edge) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)edge, (int)v, 0x130, 0xf, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, false);
}
// Inclusive xor / sum scans over the wavefront: row shifts 1, 2, 4, 8, then
// row 0's total into row 1 and row 2's into row 3, then lane 31's into
// rows 2 and 3 (lanes whose source lies outside the row read 0).
__device__ __forceinline__ uint32_t wave_xor_scan(uint32_t x) {
  x ^= dpp_u32<0x111, 0xf>(x);
  x ^= dpp_u32<0x112, 0xf>(x);
  x ^= dpp_u32<0x114, 0xf>(x);
  x ^= dpp_u32<0x118, 0xf>(x);
  x ^= dpp_u32<0x142, 0xa>(x);
  x ^= dpp_u32<0x143, 0xc>(x);
  return x;
}
__device__ __forceinline__ uint32_t wave_add_scan(uint32_t x) {
  x += dpp_u32<0x111, 0xf>(x);
  x += dpp_u32<0x112, 0xf>(x);
  x += dpp_u32<0x114, 0xf>(x);
  x += dpp_u32<0x118, 0xf>(x);
  x += dpp_u32<0x142, 0xa>(x);
  x += dpp_u32<0x143, 0xc>(x);
  return x;
}

// One wavefront per row (up to 64 crossings one per lane, up to 256 four
// per lane).  Crossings rank-sorted by (p0, slot); t = A xor B for every
// crossing; the inclusive xor-scan X gives the claiming region after every
// prefix as long as at most one region claims (the claim set starts empty
// at the left border).  A crossing alone at its p0 keeps the set a
// singleton iff the label before it is one of its two regions.  Rows that
// fail this test, or have several crossings at one p0 (a boundary wiggling
// inside one pixel, or a folded map), take exact claim sets: for every
// distinct region of the row (a bitmap in LDS), its membership after
// crossing k is the parity of the crossings <= k with that region on one
// side only (a ballot and a popcount).  The serial walk of the claim set
// remains for long rows of maps with more regions than the bitmap holds.
//
// LEAD (launches of single-edge emit blocks): every instance has one block
// more, its first, which with RULE runs the stopping rule of the previous
// iteration (the emit pass before has computed that iteration's areas and
// recorded the flags as they were before this fill, which the rule reads
// instead of the flags the other blocks are setting).  The rows of an
// instance the rule ends are still filled in this launch; no kernel after
// it reads them, and the run's positions are final.
template <bool LEAD, bool RULE>
__global__ __launch_bounds__(256) void k_raster_fill(Batch B) {
  int64_t first;
  const int k = find_inst(B, B.off_rows, KD_ROWS, blockIdx.x, first);
  const InstG I = inst_of(B, k);  // register copy: stores below cannot alias it
  if (inst_done(B, k)) return;
  if (LEAD && blockIdx.x == first) {
    if (RULE) {
      __shared__ double red[256];
      (void)stopping_rule(I, 0, 0.f, red, true);
    }
    return;
  }
  constexpr int RPW = kFillRows / 4;   // rows per wavefront
  __shared__ uint64_t xs[4][kFillXing];
  uint64_t (*const srt)[kFillXing] = xs;   // sorted in place: every lane holds its records before any is written
  __shared__ uint16_t sp_start[4][kFillXing + 2];
  __shared__ uint16_t sp_lab[4][kFillXing + 2];
  __shared__ uint32_t lcount[kLutLds];
  __shared__ uint32_t rbits[4][kLutLds / 32];   // regions of a row (exact claim sets)
  __shared__ unsigned long long contested_blk;
  const int N = I.N, R = I.R;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int q0 = (int)(blockIdx.x - first - (LEAD ? 1 : 0)) * kFillRows;
  const bool lds_counts = (R + 1) <= kLutLds;
  // the first row's crossing count and its bucket's first 64 slots are
  // read together (the slots exist whatever the count)
  uint32_t cnt_first = 0;
  uint64_t rec_first = 0;
  if (q0 + w * RPW < N) {
    cnt_first = I.row_cnt[q0 + w * RPW];
    rec_first = I.xing[(int64_t)(q0 + w * RPW) * kFillXing + lane];
  }
  if (lds_counts)
    for (int v = t; v <= R; v += 256) lcount[v] = 0u;
  if (t == 0) contested_blk = 0ull;
  __syncthreads();
  for (int rr = 0; rr < RPW; ++rr) {
    const int q = q0 + w * RPW + rr;
    const bool row_ok = q < N;
    uint32_t cnt = 0, off = 0;
    bool bad = false;
    if (row_ok) {
      cnt = rr == 0 ? cnt_first : I.row_cnt[q];
      off = (uint32_t)q * (uint32_t)kFillXing;
      if (cnt > (uint32_t)kFillXing) bad = true;
      if (bad) cnt = 0;
      uint32_t i0 = lane;
      if (rr == 0) {
        if (lane < (int)cnt) xs[w][lane] = rec_first;
        i0 += 64;
      }
      for (uint32_t i = i0; i < cnt; i += 64) xs[w][i] = I.xing[off + i];
    }
    // Every LDS array of the row loop belongs to one wavefront, whose LDS
    // accesses take effect in program order: no block barrier inside the
    // loop (a row's wavefront never waits for the block's other rows), only
    // a barrier against the compiler moving accesses across the phases.
    __builtin_amdgcn_wave_barrier();
    cnt = (uint32_t)__builtin_amdgcn_readfirstlane((int)cnt);   // one row per wavefront
    if (row_ok) {
      // rank sort by the keys (p0, slot): every key is compared with all
      // others, read by lane (rows up to 64 crossings) or as LDS
      // broadcasts (longer rows, up to four keys per lane)
      if (cnt <= 64) {
        const uint64_t rec = lane < (int)cnt ? xs[w][lane] : 0ull;
        const uint32_t key = lane < (int)cnt ? (((uint32_t)(rec & 0xFFFFull) << 8) | (uint32_t)lane) : ~0u;
        uint32_t rank = 0;
        for (uint32_t j = 0; j < cnt; ++j) rank += (uint32_t)__builtin_amdgcn_readlane((int)key, (int)j) < key;
        if (lane < (int)cnt) srt[w][rank] = rec;
      } else {
        uint64_t rec[4];
        uint32_t key[4], rank[4] = {0u, 0u, 0u, 0u};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          const uint32_t i = (uint32_t)(lane + 64 * m);
          rec[m] = i < cnt ? xs[w][i] : 0ull;
          key[m] = i < cnt ? (((uint32_t)(rec[m] & 0xFFFFull) << 8) | i) : ~0u;
        }
        for (uint32_t j = 0; j < cnt; ++j) {
          const uint32_t kj = ((uint32_t)(xs[w][j] & 0xFFFFull) << 8) | j;
#pragma unroll
          for (int m = 0; m < 4; ++m) rank[m] += kj < key[m];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < 4; ++m)
          if ((uint32_t)(lane + 64 * m) < cnt) srt[w][rank[m]] = rec[m];
      }
    }
    __builtin_amdgcn_wave_barrier();
    if (row_ok) {
    uint32_t ngroups = 0;
    bool serial = false;     // the exact serial walk decides the row
    if (cnt <= 64) {
      // one crossing per lane, sorted by p0
      const bool live = lane < (int)cnt;
      const uint64_t rec = live ? srt[w][lane] : 0ull;
      const uint32_t p0 = (uint32_t)(rec & 0xFFFFu);
      const uint32_t ra = (uint32_t)((rec >> 16) & 0xFFFFu), rb = (uint32_t)((rec >> 32) & 0xFFFFu);
      const uint32_t pnext = wave_shl1(p0, 0u);
      const bool last = live && (lane + 1 == (int)cnt || pnext != p0);
      const uint32_t x = wave_xor_scan(live ? (ra ^ rb) : 0u);
      // every group a single crossing: the claim set before it is {xb}
      // (empty when xb = 0), after it the odd-multiplicity members of
      // {xb, ra, rb}; the xor label is exact iff at most one remains.  Rows
      // with several crossings at one p0 (a boundary wiggling inside one
      // pixel: most rows of fractal maps) check whole groups: the claim set
      // after a group is the one before it, {xb}, with the regions the
      // group toggles an odd number of times flipped, so it stays a
      // singleton (or empty) iff in the multiset {xb} + the group's region
      // ids at most one id, the group's xor label, has an odd count.  Each
      // lane counts its own ids and xb over its group (groups of up to 8
      // crossings); rows that fail take the exact claim sets below.
      bool ok = !bad;
      const uint32_t pprev = wave_shr1(p0, 0u);
      const bool first = live && (lane == 0 || pprev != p0);
      if (__all(!last || first)) {
        if (last) ok = ok && single_claim_ok(x ^ ra ^ rb, ra, rb);
      } else {
        constexpr int kMaxGroup = 8;
        const uint64_t fm = __ballot(first), lm = __ballot(last);
        const uint64_t below = fm & ((2ull << lane) - 1ull);   // lane 63: every bit
        const uint64_t above = lm & ~((1ull << lane) - 1ull);
        const int g0 = below ? 63 - __clzll((long long)below) : lane;   // the group's first and last crossing
        const int g1 = above ? __ffsll((long long)above) - 1 : lane;
        const uint32_t xb = __shfl(x ^ ra ^ rb, g0, 64);    // the label before the group
        const uint32_t xa = __shfl(x, g1, 64);              // and after it
        int gmax = live ? g1 - g0 + 1 : 0;
        for (int o = 32; o >= 1; o >>= 1) gmax = max(gmax, __shfl_xor(gmax, o, 64));
        if (gmax > kMaxGroup) {
          ok = false;
        } else {
          uint32_t ca = xb == ra, cb = xb == rb, cx = 1u;   // counts of ra, rb and xb in the multiset
          for (int d = 0; d < gmax; ++d) {
            const int j = g0 + d;
            const uint32_t raj = __shfl(ra, min(j, 63), 64), rbj = __shfl(rb, min(j, 63), 64);
            if (j <= g1) {
              ca += (raj == ra) + (rbj == ra);
              cb += (raj == rb) + (rbj == rb);
              cx += (raj == xb) + (rbj == xb);
            }
          }
          // an id other than 0 has an odd count iff it is the label after the group
          auto parity_ok = [&](uint32_t v, uint32_t c) { return v == 0u || ((v == xa) == ((c & 1u) != 0u)); };
          ok = ok && (!live || (parity_ok(ra, ca) && parity_ok(rb, cb) && parity_ok(xb, cx)));
        }
      }
      uint32_t label = x, nclaim = x != 0u;
      if (__any(!ok) && lds_counts) {
        // exact claim sets in parallel: for every distinct region v of the
        // row (from a bitmap of the row's regions), its parity after
        // crossing k is the parity of the crossings <= k that toggle it
        // (an edge with v on one side only)
        label = 0u;
        nclaim = 0u;
        const uint64_t upto = (2ull << lane) - 1ull;
        if (lane < kLutLds / 32) rbits[w][lane] = 0u;
        if (live) {
          if (ra) atomicOr(&rbits[w][ra >> 5], 1u << (ra & 31u));
          if (rb) atomicOr(&rbits[w][rb >> 5], 1u << (rb & 31u));
        }
        const int nwords = (R + 32) >> 5;       // words holding ids 0..R
        for (int wi = 0; wi < nwords; ++wi) {
          uint32_t bits = (uint32_t)__builtin_amdgcn_readfirstlane((int)rbits[w][wi]);
          while (bits) {
            const uint32_t v = (uint32_t)wi * 32u + (uint32_t)__builtin_ctz(bits);
            bits &= bits - 1u;
            const uint64_t mv = __ballot(live && ((ra == v) != (rb == v)));
            if (live && (__popcll(mv & upto) & 1)) {
              ++nclaim;
              label = max(label, v);
            }
          }
        }
      } else if (__any(!ok)) {
        // the same without the bitmap (more regions than it holds)
        label = 0u;
        nclaim = 0u;
        const uint64_t upto = (2ull << lane) - 1ull;
        for (int j = 0; j < (int)cnt; ++j) {
          const uint32_t raj = (uint32_t)__builtin_amdgcn_readlane((int)ra, j);
          const uint32_t rbj = (uint32_t)__builtin_amdgcn_readlane((int)rb, j);
          for (int side = 0; side < 2; ++side) {
            const uint32_t v = side ? rbj : raj;
            if (v == 0u) continue;
            const uint64_t seen = __ballot(live && (ra == v || rb == v));
            if ((int)(__ffsll((long long)seen) - 1) < j || (side == 1 && raj == v)) continue;
            const uint64_t m = __ballot(live && ((ra == v) != (rb == v)));
            if (live && (__popcll(m & upto) & 1)) {
              ++nclaim;
              label = max(label, v);
            }
          }
        }
      }
      // runs: [0, first p0) is background; every group's last crossing starts one
      const uint64_t lastmask = __ballot(last);
      const uint32_t before = __popcll(lastmask & ((1ull << lane) - 1ull));
      unsigned long long cont = 0;
      if (last) {
        sp_start[w][1 + before] = (uint16_t)p0;
        sp_lab[w][1 + before] = (uint16_t)label;
        const uint32_t en = lane + 1 == (int)cnt ? (uint32_t)N : pnext;
        if (en > p0) {
          if (lds_counts) atomicAdd(&lcount[label], en - p0);
          else g_atomic_add((g_ptr<unsigned long long>)&I.counts[label], (unsigned long long)(en - p0));
          if (nclaim > 1) cont = en - p0;
        }
      }
      if (lane == 0) {
        sp_start[w][0] = 0;
        sp_lab[w][0] = 0;
        const uint32_t first = cnt ? (uint32_t)(srt[w][0] & 0xFFFFu) : (uint32_t)N;
        if (first > 0) {
          if (lds_counts) atomicAdd(&lcount[0], first);
          else g_atomic_add((g_ptr<unsigned long long>)&I.counts[0], (unsigned long long)first);
        }
      }
      if (__any(cont != 0ull)) {
        for (int d = 32; d >= 1; d >>= 1) cont += __shfl_xor(cont, d, 64);
        if (lane == 0) {
          atomicAdd(&contested_blk, cont);
          g_atomic_or(&I.st->flags, (int32_t)CG_FLAG_CONTESTED);
        }
      }
      if (lane == 0 && bad) g_atomic_or(&I.st->flags, (int32_t)CG_FLAG_OVERFLOW);
      ngroups = __popcll(lastmask);
    } else {
      // long rows: four consecutive sorted crossings i = 4 lane + m per
      // lane; the same xor labels and single-claim test as above, on every
      // crossing alone at its p0 (rows with coincident crossings, or whose
      // test fails, take the serial walk)
      uint32_t p[4], ra[4], rb[4], lx[4];
      bool live[4];
      uint32_t acc = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint32_t i = 4 * (uint32_t)lane + m;
        live[m] = i < cnt;
        const uint64_t rec = live[m] ? srt[w][i] : 0ull;
        p[m] = (uint32_t)(rec & 0xFFFFu);
        ra[m] = (uint32_t)((rec >> 16) & 0xFFFFu);
        rb[m] = (uint32_t)((rec >> 32) & 0xFFFFu);
        acc ^= live[m] ? (ra[m] ^ rb[m]) : 0u;
        lx[m] = acc;
      }
      const uint32_t xin = wave_xor_scan(acc);
      const uint32_t xex = xin ^ acc;                  // xor of the crossings of the lanes before
      const uint32_t pbefore = wave_shr1(p[3], 0u);    // p0 of crossing 4 lane - 1
      const uint32_t pafter = wave_shl1(p[0], 0u);     // p0 of crossing 4 lane + 4
      bool single = true, ok = true;
      uint32_t nlast = 0;
      bool last[4];
      uint32_t x[4], pn[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const uint32_t i = 4 * (uint32_t)lane + m;
        x[m] = xex ^ lx[m];
        const uint32_t pv = m == 0 ? pbefore : p[m - 1];
        pn[m] = m == 3 ? pafter : p[m + 1];
        const bool has_next = i + 1 < cnt;
        last[m] = live[m] && (!has_next || pn[m] != p[m]);
        const bool first = live[m] && (i == 0 || pv != p[m]);
        single = single && (!live[m] || (last[m] && first));
        if (last[m]) ok = ok && single_claim_ok(x[m] ^ ra[m] ^ rb[m], ra[m], rb[m]);
        nlast += last[m] ? 1u : 0u;
      }
      uint32_t lab[4], ncl[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        lab[m] = x[m];
        ncl[m] = x[m] != 0u;
      }
      bool exact_ok = true;
      if (!__all(single && ok)) {
        if (lds_counts) {
          // exact claim sets, as for short rows: parity of every distinct
          // region after crossing i = parity of the crossings <= i toggling
          // it (lanes before: one ballot; this lane: a running xor)
          const uint64_t before = (1ull << lane) - 1ull;
          if (lane < kLutLds / 32) rbits[w][lane] = 0u;
#pragma unroll
          for (int m = 0; m < 4; ++m) {
            lab[m] = 0u;
            ncl[m] = 0u;
            if (live[m]) {
              if (ra[m]) atomicOr(&rbits[w][ra[m] >> 5], 1u << (ra[m] & 31u));
              if (rb[m]) atomicOr(&rbits[w][rb[m] >> 5], 1u << (rb[m] & 31u));
            }
          }
          const int nwords = (R + 32) >> 5;
          for (int wi = 0; wi < nwords; ++wi) {
            uint32_t bits = (uint32_t)__builtin_amdgcn_readfirstlane((int)rbits[w][wi]);
            while (bits) {
              const uint32_t v = (uint32_t)wi * 32u + (uint32_t)__builtin_ctz(bits);
              bits &= bits - 1u;
              uint32_t t[4], par = 0u;
#pragma unroll
              for (int m = 0; m < 4; ++m) {
                t[m] = (live[m] && ((ra[m] == v) != (rb[m] == v))) ? 1u : 0u;
                par ^= t[m];
              }
              uint32_t run = (uint32_t)__popcll(__ballot(par != 0u) & before) & 1u;
#pragma unroll
              for (int m = 0; m < 4; ++m) {
                run ^= t[m];
                if (live[m] && run) {
                  ++ncl[m];
                  lab[m] = max(lab[m], v);
                }
              }
            }
          }
        } else {
          exact_ok = false;   // more regions than the bitmap holds: serial walk
        }
      }
      if (__all(exact_ok)) {
        const uint32_t incl = wave_add_scan(nlast);
        uint32_t idx = incl - nlast;       // groups before this lane's first crossing
        unsigned long long cont = 0;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          if (!last[m]) continue;
          sp_start[w][1 + idx] = (uint16_t)p[m];
          sp_lab[w][1 + idx] = (uint16_t)lab[m];
          ++idx;
          const uint32_t i = 4 * (uint32_t)lane + m;
          const uint32_t en = i + 1 == cnt ? (uint32_t)N : pn[m];
          if (en > p[m]) {
            if (lds_counts) atomicAdd(&lcount[lab[m]], en - p[m]);
            else g_atomic_add((g_ptr<unsigned long long>)&I.counts[lab[m]], (unsigned long long)(en - p[m]));
            if (ncl[m] > 1) cont += en - p[m];
          }
        }
        if (lane == 0) {
          sp_start[w][0] = 0;
          sp_lab[w][0] = 0;
          if (p[0] > 0) {
            if (lds_counts) atomicAdd(&lcount[0], p[0]);
            else g_atomic_add((g_ptr<unsigned long long>)&I.counts[0], (unsigned long long)p[0]);
          }
        }
        if (__any(cont != 0ull)) {
          for (int d = 32; d >= 1; d >>= 1) cont += __shfl_xor(cont, d, 64);
          if (lane == 0) {
            atomicAdd(&contested_blk, cont);
            g_atomic_or(&I.st->flags, (int32_t)CG_FLAG_CONTESTED);
          }
        }
        ngroups = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
      } else {
        serial = true;
      }
    }
    if (serial && lane == 0) {
      // exact serial walk of the claim set
      Claims cl;
      cl.cur = 0;
      cl.multi = false;
#pragma unroll
      for (int i = 0; i < kSetCap; ++i) cl.set[i] = 0;
      bool over = false;
      uint32_t nsp = 0, prev = 0;
      unsigned long long cont = 0;
      for (uint32_t i = 0; i <= cnt; ++i) {
        uint64_t rec = 0;
        uint32_t p0 = (uint32_t)N;
        if (i < cnt) {
          rec = srt[w][i];
          p0 = (uint32_t)(rec & 0xFFFFu);
        }
        if (p0 > prev || (i == cnt && nsp == 0)) {
          int lab, n;
          claims_label(cl, lab, n);
          sp_start[w][nsp] = (uint16_t)prev;
          sp_lab[w][nsp] = (uint16_t)lab;
          ++nsp;
          const uint32_t len = p0 - prev;
          if (n > 1) cont += len;
          if (len) {
            if (lds_counts) atomicAdd(&lcount[lab], len);
            else g_atomic_add((g_ptr<unsigned long long>)&I.counts[lab], (unsigned long long)len);
          }
          prev = p0;
        }
        if (i < cnt) {
          claims_toggle(cl, (int)((rec >> 16) & 0xFFFFu), over);
          claims_toggle(cl, (int)((rec >> 32) & 0xFFFFu), over);
        }
      }
      ngroups = nsp - 1;
      if (cont) {
        atomicAdd(&contested_blk, cont);
        g_atomic_or(&I.st->flags, (int32_t)CG_FLAG_CONTESTED);
      }
      if (bad || over) g_atomic_or(&I.st->flags, (int32_t)CG_FLAG_OVERFLOW);
    }
      ngroups = __shfl(ngroups, 0, 64);
      // fill: spans 0..ngroups, the last span with start <= p holds pixel p
      const int nsp = (int)ngroups + 1;
      g_ptr<uint16_t> row = I.labels + (int64_t)q * N;
      int steps = 0;                       // binary-search steps over the spans (uniform)
      while ((1 << steps) < nsp) ++steps;
      constexpr int U = 4;                 // chunks searched in lockstep per lane
      for (int pb = lane * 8; pb < N; pb += 64 * 8 * U) {
        int los[U];
#pragma unroll
        for (int u = 0; u < U; ++u) los[u] = 0;
        for (int st = 0, span = 1 << (steps > 0 ? steps - 1 : 0); st < steps; ++st, span >>= 1) {
#pragma unroll
          for (int u = 0; u < U; ++u) {   // invariant: sp_start[los] <= p
            const int mid = los[u] + span;
            const bool in = mid < nsp;
            const int sp = sp_start[w][in ? mid : 0];
            los[u] = (in && sp <= pb + u * 512) ? mid : los[u];
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
        const int p = pb + u * 512;
        if (p >= N) break;
        const int lo = los[u];
        uint16_t v[8];
        // the next three span starts (N past the last span), read together;
        // the chunk's labels follow by selects when at most two spans start
        // inside it
        const int i1 = min(lo + 1, nsp - 1), i2 = min(lo + 2, nsp - 1), i3 = min(lo + 3, nsp - 1);
        const int s1 = lo + 1 < nsp ? (int)sp_start[w][i1] : N;
        const int s2 = lo + 2 < nsp ? (int)sp_start[w][i2] : N;
        const int s3 = lo + 3 < nsp ? (int)sp_start[w][i3] : N;
        const uint16_t l0 = sp_lab[w][lo], l1 = sp_lab[w][i1], l2 = sp_lab[w][i2];
        if (s3 >= p + 8) {
#pragma unroll
          for (int c = 0; c < 8; ++c) v[c] = p + c < s1 ? l0 : (p + c < s2 ? l1 : l2);
        } else {               // three or more spans start in these 8 pixels
          int sx = lo;
#pragma unroll
          for (int c = 0; c < 8; ++c) {
            while (sx + 1 < nsp && sp_start[w][sx + 1] <= p + c) ++sx;
            v[c] = sp_lab[w][sx];
          }
        }
        typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
        u32x4_t pk;
        pk.x = v[0] | ((uint32_t)v[1] << 16);
        pk.y = v[2] | ((uint32_t)v[3] << 16);
        pk.z = v[4] | ((uint32_t)v[5] << 16);
        pk.w = v[6] | ((uint32_t)v[7] << 16);
        __builtin_nontemporal_store(pk, (g_ptr<u32x4_t>)(row + p));   // N is a multiple of 8; streamed
        }
      }
      if (lane == 0) I.row_cnt[q] = 0u;
    }
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
  // the block's counts into the instance totals (integer sums: order-independent)
  if (lds_counts)
    for (int v = t; v <= R; v += 256)
      if (lcount[v]) g_atomic_add((g_ptr<unsigned long long>)&I.counts[v], (unsigned long long)lcount[v]);
  if (t == 0 && contested_blk) g_atomic_add((g_ptr<unsigned long long>)&I.st->contested, (unsigned long long)contested_blk);
}

void launch_raster(const Batch& B, int ept, int64_t edge_blocks, int64_t row_blocks, hipStream_t s, StageHook h,
                   void* u, bool rule) {
  auto hk = [&](int st, int after) { if (h) h(st, after, u); };
  // with single-edge blocks (few blocks, where a launch of its own costs
  // most) the plan gives every instance its totals, area and rule blocks;
  // with four edges per thread the extra blocks per instance made the
  // 64 x 2048^2 emit 9% slower, so those plans have none
  const bool one = ept != kEmitEdges;
  if (edge_blocks > 0) {
    hk(ST_RASTER_EMIT, 0);
    if (!one)
      hipLaunchKernelGGL((k_raster_emit<kEmitEdges, 0>), dim3(edge_blocks), dim3(256), 0, s, B);
    else if (rule)
      hipLaunchKernelGGL((k_raster_emit<1, 2>), dim3(edge_blocks), dim3(256), 0, s, B);
    else
      hipLaunchKernelGGL((k_raster_emit<1, 1>), dim3(edge_blocks), dim3(256), 0, s, B);
    hk(ST_RASTER_EMIT, 1);
  }
  hk(ST_RASTER_FILL, 0);
  if (!one) hipLaunchKernelGGL((k_raster_fill<false, false>), dim3(row_blocks), dim3(256), 0, s, B);
  else if (rule) hipLaunchKernelGGL((k_raster_fill<true, true>), dim3(row_blocks), dim3(256), 0, s, B);
  else hipLaunchKernelGGL((k_raster_fill<true, false>), dim3(row_blocks), dim3(256), 0, s, B);
  hk(ST_RASTER_FILL, 1);
}

}  // namespace cgk
