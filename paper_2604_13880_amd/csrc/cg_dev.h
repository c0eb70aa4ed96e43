// Device-side types shared by the HIP kernels of libcg.
//
// Every kernel works on a batch of independent cartogram instances.  A
// launch covers all instances: blockIdx.x is mapped to (instance, local
// block) through a per-kind prefix table of block counts, so one code path
// serves a single cartogram, all time steps of a series and uneven batches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cg.h"

namespace cgk {

constexpr int kSub = 256;          // fixed-point subdivisions per pixel (rasteriser)
constexpr int kLutLds = 1024;      // LUT entries kept in LDS by the scan / fill kernels
constexpr int kFillXing = 256;     // crossings one row may hold (its bucket; LDS of the fill kernel)
constexpr int kSetCap = 8;         // simultaneous claims tracked per pixel run
constexpr int kEmitEdges = 4;      // edges per emit thread in large launches
constexpr int kFillRows = 4;       // label rows per fill block (one per wavefront)
constexpr int kCarryRows = 8;      // tile rows one carry thread sums

// Pipeline stages of one iteration (for per-stage timing hooks).
enum Stage {
  ST_RASTER_EMIT = 0, ST_RASTER_FILL, ST_DENSITY,
  ST_SAT_REDUCE, ST_SAT_CARRY1, ST_SAT_CARRY2, ST_SAT_FINAL, ST_MAP, ST_AREAS, ST_ERR, ST_COUNT
};
// Called on the host right before (after = 0) and after (after = 1) a
// stage's kernel is enqueued.
typedef void (*StageHook)(int stage, int after, void* user);

// Iteration state of one instance (written by the kernels, polled by the host).
struct IterState {
  int32_t iter;       // moves done so far
  int32_t best_k;     // iteration of the smallest max error seen
  int32_t done;       // stopping rule met
  int32_t status;     // CG_STATUS_*
  int32_t flags;      // CG_FLAG_*
  int32_t evaluated;  // the error of the starting positions is known
  int64_t contested;  // contested pixels in the latest label map
  double xi, eps, best_xi;
  double d0, C;       // density parameters of the latest iteration
  double xi0;         // max error of the plain (not warm-started) start
  double ws_best;     // lowest max error among the warm start's trial steps
  float ws_alpha;     // chosen warm-start step (0: plain start)
  int32_t flags_rule; // flags as the emit pass found them (read by the rule run inside the fill)
};

// Pointer policies of the instance descriptor: the host fills generic
// pointers; kernels view the same bits as global-address-space pointers so
// that their loads, stores and atomics compile to global (not flat)
// instructions, which do not stall on LDS traffic.
#define CG_GLOBAL __attribute__((address_space(1)))
#define CG_CONST __attribute__((address_space(4)))
template <typename T> using g_ptr = T CG_GLOBAL*;
struct PlainPtr {
  template <typename T> using p = T*;
};
struct GlobalPtr {
  template <typename T> using p = T CG_GLOBAL*;
};

template <typename PP>
struct InstT {
  int32_t N, R, n_vert, n_pts;        // n_pts = vertices + tracer points
  int32_t n_edges, n_rings, n_lut, pad0;
  int32_t tw, th, ntx, nty;           // integral-image tiling
  int32_t area_source, patience, max_iters, fixed_iters;
  float shape, tol;
  int64_t pitch;
  double bg_mass;                     // prescribed background mass M_b (eq.(4)), or < 0: BDV = shape * d0
  // topology
  typename PP::template p<const int4> edges;                  // (v0, v1, region A, region B)
  typename PP::template p<const int32_t> reg_pair_off;        // [R+1] region -> its ring edges
  typename PP::template p<const int2> reg_pairs;              // ring edges (a, b) of every region, ring order
  // state and buffers
  typename PP::template p<float2> xy;                         // [n_vert] vertex positions (iterated in place)
  typename PP::template p<float2> extra;                      // [n_pts - n_vert] tracer points moved along
  typename PP::template p<const float2> src_xy;               // starting positions copied in by k_init (or null)
  typename PP::template p<const float2> src_extra;
  typename PP::template p<const float> init_field;            // warm-start displacement [G][G][2] at pixel centres, or null
  int64_t init_G;
  typename PP::template p<const float> values;                // [R]
  typename PP::template p<uint32_t> row_cnt;                  // [N] crossings per row (bucket fill)
  typename PP::template p<uint64_t> xing;                     // [N][kFillXing] crossing buckets
  typename PP::template p<uint16_t> labels;                   // [N][N]
  typename PP::template p<int64_t> counts;                    // [R+1]
  typename PP::template p<float> lut;                         // [n_lut]
  typename PP::template p<const float> density;               // dense texture (replaces labels + lut) or null
  typename PP::template p<void> S;
  typename PP::template p<void> T;
  typename PP::template p<void> HA;
  typename PP::template p<void> HB;
  typename PP::template p<void> agg;                          // integral-image tile aggregates
  typename PP::template p<void> carry;                        // integral-image carries
  typename PP::template p<double> areas;                      // [R+1]
  typename PP::template p<IterState> st;
};

using Inst = InstT<PlainPtr>;
using InstG = InstT<GlobalPtr>;
static_assert(sizeof(Inst) == sizeof(InstG), "descriptor views share one layout");

// Per-kind block offsets over the instances of a batch ([n+1] each).
// Kinds of per-instance work; each has its own block numbering.
enum Kind { KD_EDGES = 0, KD_ROWS, KD_TILES, KD_CARRY1, KD_CARRY2, KD_PTS, KD_REGIONS, KD_INST, KD_COUNT };

struct Batch {
  const Inst* inst;
  int32_t n;
  int32_t skip_done;                  // 1: instances whose state says done are skipped
  int32_t max_n;                      // largest texture of the batch
  int32_t make_lut;                   // 1: the integral-image reduce pass builds the density LUT (Step 3)
  int32_t stride[KD_COUNT];           // blocks per instance of each kind when all instances have as many, else 0
  const IterState* states;            // [n] iteration states (instance k's is states + k)
  const uint32_t* where[KD_COUNT];    // stride 0: per block of the kind, (instance, its first block)
  const int64_t* off_edges;
  const int64_t* off_rows;
  const int64_t* off_tiles;
  const int64_t* off_carry1;
  const int64_t* off_carry2;
  const int64_t* off_pts;
  const int64_t* off_regions;
  const int64_t* off_inst;
};

// Instance of block b of work kind kd, and that instance's first block.
// When every instance has the same number of blocks of the kind this is a
// division; otherwise one load from the batch's block table (a binary
// search over the block offsets `off` if there is none).  The instance is
// made explicitly wave-uniform so descriptor fields are fetched with
// scalar loads.
__device__ __forceinline__ int find_inst(const Batch& B, const int64_t* off, int kd, int64_t b, int64_t& first) {
  const uint32_t s = (uint32_t)B.stride[kd];
  if (s > 0u) {   // block indices are below 2^32
    const int k = __builtin_amdgcn_readfirstlane((int)((uint32_t)b / s));
    first = (int64_t)k * s;
    return k;
  }
  if (B.where[kd] != nullptr) {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    const u2 e = ((const u2 CG_CONST*)B.where[kd])[b];
    first = (int64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)e.y);
    return __builtin_amdgcn_readfirstlane((int)e.x);
  }
  int lo = 0, hi = B.n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (off[mid] <= b) lo = mid; else hi = mid;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  first = off[lo];
  return lo;
}

// Background density of Step 3: shape * d0, or, with a prescribed
// background mass M_b (eq.(4) of the steering section), shape * M_b / o_bg
// so that the o_bg background pixels hold M_b (shape * d0 when there are none).
template <typename I_>
__device__ __forceinline__ double background_density(const I_& I, double d0, double o_bg) {
  return (double)I.shape * ((I.bg_mass >= 0.0 && o_bg > 0.0) ? I.bg_mass / o_bg : d0);
}

// Descriptor k of a batch in registers (scalar loads; read-only in kernels).
__device__ __forceinline__ InstG inst_of(const Batch& B, int k) {
  return __builtin_bit_cast(InstG, ((const Inst CG_CONST*)B.inst)[k]);
}

// Loads and stores of HIP vector types through global-space pointers.
__device__ __forceinline__ int4 ld4(g_ptr<const int4> p) {
  typedef int v4 __attribute__((ext_vector_type(4)));
  const v4 v = *(g_ptr<const v4>)p;
  return make_int4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ float2 ld2(g_ptr<const float2> p) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(g_ptr<const v2>)p;
  return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2(g_ptr<float2> p, float2 a) {
  typedef float v2 __attribute__((ext_vector_type(2)));
  *(g_ptr<v2>)p = v2{a.x, a.y};
}

// Global-space atomics (relaxed, device scope).
template <typename T>
__device__ __forceinline__ T g_atomic_add(g_ptr<T> p, T v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T g_atomic_or(g_ptr<T> p, T v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether instance k has met its stopping rule (skipped when the batch
// says so).  Read from the state array directly, so the load does not wait
// for the descriptor's.
__device__ __forceinline__ bool inst_done(const Batch& B, int k) {
  return B.skip_done && ((g_ptr<const IterState>)B.states)[k].done != 0;
}

// Fixed-order block reductions over 256 threads (deterministic): a
// butterfly of lane exchanges within each wavefront (lane 0's total is the
// one used), then the four wavefront totals in a fixed order.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return r;
}

// Region v's area (Step 7: FP64 shoelace over its rings' vertex pairs in
// ring order), by one block of 256 threads; thread 0 stores it.
__device__ __forceinline__ void region_area(const InstG& I, int v, double* red) {
  const int t = threadIdx.x;
  double acc = 0.0;
  const int end = I.reg_pair_off[v];
  // four of the thread's edges per round: their loads are all in flight
  // before the first is used (the terms are added in the same order)
  constexpr int U = 4;
  typedef int i2 __attribute__((ext_vector_type(2)));
  for (int e0 = I.reg_pair_off[v - 1] + t; e0 < end; e0 += 256 * U) {
    i2 pr[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pr[u] = *(g_ptr<const i2>)(I.reg_pairs + min(e0 + 256 * u, end - 1));   // unconditional
    float2 a[U], b[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      a[u] = ld2(I.xy + pr[u].x);
      b[u] = ld2(I.xy + pr[u].y);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (e0 + 256 * u < end) acc += (double)a[u].x * (double)b[u].y - (double)b[u].x * (double)a[u].y;
  }
  acc = block_sum(acc, red);
  if (t == 0) I.areas[v] = 0.5 * acc;
}

// Step 7 for one instance, by one block of 256 threads: region weights
// w(v) = s(v) O / sum s, the mean and max area errors eps and xi, and in
// mode 0 the stopping rule (max error below tol, no new minimum within
// `patience` iterations, the iteration cap, or fixed_iters), written to
// the instance's state by thread 0; modes 2-4 score the warm start's
// trial steps.  Returns the stopping decision of mode 0 in thread 0 (0 in
// the other threads).
__device__ __forceinline__ int stopping_rule(const InstG& I, int mode, float alpha, double* red,
                                             bool flags_snapshot = false) {
  const int t = threadIdx.x, R = I.R;
  g_ptr<IterState> st = I.st;
  // the state the stopping rule reads (written only by the one block that
  // runs the rule for the instance), loaded while the sums run
  int32_t st_eval = 0, st_iter = 0, st_bestk = 0, st_flags = 0;
  double st_best = 0.0;
  if (t == 0 && mode == 0) {
    st_eval = st->evaluated;
    st_iter = st->iter;
    st_bestk = st->best_k;
    st_flags = flags_snapshot ? st->flags_rule : st->flags;
    st_best = st->best_xi;
  }
  double sa = 0.0, ss = 0.0, bad = 0.0;
  double A1 = 0.0;   // the thread's first region, kept for the second pass
  float s1 = 0.f;
  for (int v = 1 + t; v <= R; v += 256) {
    const float s = I.values[v - 1];
    const double A = I.areas[v];
    if (v == 1 + t) {
      A1 = A;
      s1 = s;
    }
    sa += A;
    ss += (double)s;
    bad = (s >= 0.f && s <= 3.4028235e38f) ? bad : 1.0;   // NaN, infinite or negative value
  }
  sa = block_sum(sa, red);
  ss = block_sum(ss, red);
  bad = block_max(bad, red);
  double se = 0.0, me = 0.0;
  for (int v = 1 + t; v <= R; v += 256) {
    const double A = v == 1 + t ? A1 : I.areas[v];
    const double w = (double)(v == 1 + t ? s1 : I.values[v - 1]) * sa / ss;
    const double m = fmax(A, w);
    const double e = m > 0.0 ? fabs(A - w) / m : 0.0;
    se += e;
    me = fmax(me, e);
  }
  se = block_sum(se, red);
  me = block_max(me, red);
  if (t != 0) return 0;
  const double xi = me, eps = R > 0 ? se / R : 0.0;
  I.areas[0] = 1.0 - sa;
  st->xi = xi;
  st->eps = eps;
  if (mode == 2) {
    st->xi0 = xi;
    st->ws_best = xi;
    st->ws_alpha = 0.f;
  }
  if (mode == 3 && I.init_field != nullptr) {
    // a trial step of the warm start: kept if the moved map did not fold
    // (no contested pixel, no overflowing crossing buffer) and its error is
    // the lowest so far, below the plain start's
    const int f = st->flags;
    if (!(f & CG_FLAG_OVERFLOW) && st->contested == 0 && xi < st->ws_best) {
      st->ws_best = xi;
      st->ws_alpha = alpha;
    }
    st->flags = f & ~CG_FLAG_OVERFLOW;
  }
  if (mode == 4 && I.init_field != nullptr && st->ws_alpha == 0.f) st->flags |= CG_FLAG_FALLBACK;
  if (mode != 0) return 0;
  int it, best_k = st_bestk;
  if (!st_eval) {
    st->evaluated = 1;
    it = 0;
    st->best_xi = xi;
    st->best_k = best_k = 0;
  } else {
    it = st_iter + 1;
    st->iter = it;
    if (xi < st_best) {
      st->best_xi = xi;
      st->best_k = best_k = it;
    }
  }
  int done = 0, status = CG_STATUS_MAXITER;
  if (bad > 0.0 || !(ss > 0.0)) {   // the values define no density: nothing is iterated
    g_atomic_or(&st->flags, (int32_t)CG_FLAG_BADVALUES);   // other blocks may set flags meanwhile
    done = 1;
    status = CG_STATUS_ERROR;
  } else if (st_flags & CG_FLAG_OVERFLOW) { done = 1; status = CG_STATUS_ERROR; }
  else if (I.fixed_iters > 0) { done = it >= I.fixed_iters; status = CG_STATUS_MAXITER; }
  else if (xi < (double)I.tol) { done = 1; status = CG_STATUS_CONVERGED; }
  else if (it - best_k >= I.patience) { done = 1; status = CG_STATUS_STALLED; }
  else if (it >= I.max_iters) { done = 1; status = CG_STATUS_MAXITER; }
  st->status = status;
  st->done = done;
  return done;
}

__device__ __forceinline__ int64_t floordiv(int64_t a, int64_t b) {  // b > 0
  int64_t q = a / b;
  return (q * b > a) ? q - 1 : q;
}
__device__ __forceinline__ int64_t ceildiv(int64_t a, int64_t b) { return -floordiv(-a, b); }

// ---------------------------------------------------------------------------
// accumulation precision

struct Comp {  // unevaluated sum hi + lo of two floats
  float hi, lo;
};

template <int P> struct PT;
template <> struct PT<CG_F32> { typedef float acc; typedef float carry; typedef float store; };
template <> struct PT<CG_COMP> { typedef Comp acc; typedef double carry; typedef float store; };
template <> struct PT<CG_F64> { typedef double acc; typedef double carry; typedef double store; };
template <> struct PT<CG_F64ACC> { typedef double acc; typedef double carry; typedef float store; };

__device__ __forceinline__ void acc_zero(float& a) { a = 0.f; }
__device__ __forceinline__ void acc_zero(double& a) { a = 0.0; }
__device__ __forceinline__ void acc_zero(Comp& a) { a.hi = 0.f; a.lo = 0.f; }

// add a density sample
__device__ __forceinline__ void acc_add(float& a, float x) { a += x; }
__device__ __forceinline__ void acc_add(double& a, float x) { a += (double)x; }
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  float bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}
__device__ __forceinline__ void acc_add(Comp& a, float x) {
  float s, e;
  two_sum(a.hi, x, s, e);
  a.hi = s;
  a.lo += e;
}
// add another accumulator
__device__ __forceinline__ void acc_addv(float& a, float b) { a += b; }
__device__ __forceinline__ void acc_addv(double& a, double b) { a += b; }
__device__ __forceinline__ void acc_addv(Comp& a, Comp b) {
  float s, e;
  two_sum(a.hi, b.hi, s, e);
  a.hi = s;
  a.lo += e + b.lo;
}
__device__ __forceinline__ float acc_sub(float a, float b) { return a - b; }
__device__ __forceinline__ double acc_sub(double a, double b) { return a - b; }
__device__ __forceinline__ Comp acc_sub(Comp a, Comp b) {
  Comp nb{-b.hi, -b.lo};
  acc_addv(a, nb);
  return a;
}
__device__ __forceinline__ float acc_half(float a) { return 0.5f * a; }
__device__ __forceinline__ double acc_half(double a) { return 0.5 * a; }
__device__ __forceinline__ Comp acc_half(Comp a) { return Comp{0.5f * a.hi, 0.5f * a.lo}; }

// conversions between accumulator, carry and storage types
__device__ __forceinline__ float to_carry(float a) { return a; }
__device__ __forceinline__ double to_carry(double a) { return a; }
__device__ __forceinline__ double to_carry(Comp a) { return (double)a.hi + (double)a.lo; }
__device__ __forceinline__ void from_carry(float& a, float c) { a = c; }
__device__ __forceinline__ void from_carry(double& a, double c) { a = c; }
__device__ __forceinline__ void from_carry(Comp& a, double c) {
  a.hi = (float)c;
  a.lo = (float)(c - (double)a.hi);
}
__device__ __forceinline__ float to_store(float a) { return a; }
__device__ __forceinline__ double to_store(double a) { return a; }
__device__ __forceinline__ float to_store(Comp a) { return (float)((double)a.hi + (double)a.lo); }

__device__ __forceinline__ float shfl_up_acc(float v, int d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ double shfl_up_acc(double v, int d) { return __shfl_up(v, d, 64); }
__device__ __forceinline__ Comp shfl_up_acc(Comp v, int d) {
  return Comp{__shfl_up(v.hi, d, 64), __shfl_up(v.lo, d, 64)};
}

__device__ __forceinline__ float shfl_acc(float v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ double shfl_acc(double v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ Comp shfl_acc(Comp v, int src) {
  return Comp{__shfl(v.hi, src, 64), __shfl(v.lo, src, 64)};
}

// Exclusive scan of one value per lane over a 64-wide wavefront (fixed order).
template <typename A>
__device__ __forceinline__ A wave_exclusive_scan(A v, int lane) {
  A x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    A t = shfl_up_acc(x, d);
    if (lane >= d) acc_addv(x, t);
  }
  A ex = shfl_up_acc(x, 1);
  if (lane == 0) acc_zero(ex);
  return ex;
}

// XCD-aware block order: consecutive logical tiles land on the same XCD
// (the hardware deals blocks round-robin over the 8 XCDs), so what
// neighbouring tiles share (adjacent segments of the same label rows, the
// line masses the writer reads from the tiles beside it) stays in one L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  constexpr int64_t X = 8;
  int64_t per = nblocks / X;
  if (per == 0 || b >= per * X) return b;
  return (b % X) * per + b / X;
}

// Integral-image tiling of one texture: tiles of TW columns x TH rows,
// padded extents NX = ntx*TW >= N, NY = nty*TH >= N; index ranges of the
// anti-diagonal (u = i+j-1 in [-1, NX+NY-1]) and diagonal (v = i-j in
// [-NY, NX]) carries.  Scratch arrays hold elements of the carry type.
struct SatLayout {
  int32_t ntx, nty, NX, NY, LA, LB;
  int32_t carry_ch;        // carry-pass chunks per index (a power of two <= 256)
  int64_t rowTot, RC, tileTot, prefTot, colsum, cdfA, cdfB, Cval, agg_elems;
  int64_t Stop, TAc, TBc, carry_elems;
};

__host__ __device__ inline SatLayout sat_layout(int N, int TW, int TH) {
  SatLayout L;
  L.ntx = (N + TW - 1) / TW;
  L.nty = (N + TH - 1) / TH;
  L.NX = L.ntx * TW;
  L.NY = L.nty * TH;
  L.LA = L.NX + L.NY + 1;
  L.LB = L.NX + L.NY + 1;
  L.carry_ch = 1;
  while (L.carry_ch * kCarryRows < L.nty) L.carry_ch *= 2;
  const int64_t ntx = L.ntx, nty = L.nty, D = TW + TH - 1;
  int64_t o = 0;
  L.rowTot = o; o += ntx * L.NY;
  L.RC = o; o += ntx * L.NY;
  L.tileTot = o; o += nty * ntx;
  L.prefTot = o; o += nty * (ntx + 1);
  L.colsum = o; o += nty * ntx * (TW + 1);
  L.cdfA = o; o += nty * ntx * D;
  L.cdfB = o; o += nty * ntx * D;
  L.Cval = o; o += 1;
  L.agg_elems = o;
  o = 0;
  L.Stop = o; o += nty * (int64_t)(L.NX + 1);
  L.TAc = o; o += (nty + 1) * (int64_t)L.LA;
  L.TBc = o; o += (nty + 1) * (int64_t)L.LB;
  L.carry_elems = o;
  return L;
}

}  // namespace cgk
