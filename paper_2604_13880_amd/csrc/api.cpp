// Host side of libcg: the C ABI declared in cg.h.
//
// A call builds a "plan": one device descriptor (cgk::Inst) per cartogram
// instance, per-kind block-offset tables and the instance scratch buffers,
// all carved from context-owned device buffers that only grow.  The same
// kernels run for one instance (the per-step calls) and for whole batches
// (cg_step_series), where the iteration body is captured once into a HIP
// graph and replayed, with a convergence poll between replays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <tuple>
#include <vector>

#include "cg.h"
#include "cg_dev.h"
#include "cg_net.h"
#include "host.h"

namespace cgk {
void launch_raster(const Batch& B, int ept, int64_t edge_blocks, int64_t row_blocks, hipStream_t s, StageHook h,
                   void* u, bool rule = false);
bool launch_sat(const Batch& B, int prec, int tw, int th, bool dense, bool il, int64_t tiles, int64_t c1,
                int64_t c2, hipStream_t s, StageHook h, void* u);
bool sat_shape_supported(int tw, int th);
void launch_density(const Batch& B, hipStream_t s);
void launch_map(const Batch& B, int prec, bool il, int64_t pt_blocks, hipStream_t s);
void launch_apply_field(const Batch& B, int64_t pt_blocks, float alpha, hipStream_t s);
void launch_restore(const Batch& B, int64_t pt_blocks, hipStream_t s);
void launch_log_density(const uint16_t* labels, const int64_t* counts, const float* values, int R, int N, float shape,
                        float* lut, float* out, hipStream_t s);
void launch_tracer_field(int G, const float* fin, float* out, hipStream_t s);
void launch_field_pool(int G, int f, const float* in, float* out, hipStream_t s);
void launch_areas(const Batch& B, int64_t region_blocks, hipStream_t s);
void launch_err(const Batch& B, int mode, hipStream_t s, float alpha = 0.f);
void launch_init(const Batch& B, int64_t pt_blocks, hipStream_t s);
void launch_export(const Batch& B, int64_t* contested, double* eps_xi, hipStream_t s);
void launch_frames(const float* a, const float* b, float* out, int64_t n, int K, hipStream_t s);
}  // namespace cgk

using cgk::Batch;
using cgk::Inst;
using cgk::IterState;
using cgk::SatLayout;

using namespace cgh;
using cgk::kFillRows;

namespace {

// Host -> device copy through a pinned staging buffer guarded by an event.
int upload(cg_ctx* c, void* dst, const void* src, size_t bytes, hipStream_t st) {
  if (c->pinned_pending) {
    HIP_OK(c, hipEventSynchronize(c->pinned_ev));
    c->pinned_pending = false;
  }
  if (c->pinned_n < bytes) {
    if (c->pinned) HIP_OK(c, hipHostFree(c->pinned));
    c->pinned = nullptr;
    size_t want = std::max(bytes, (size_t)65536);
    HIP_OK(c, hipHostMalloc((void**)&c->pinned, want, hipHostMallocDefault));
    c->pinned_n = want;
  }
  memcpy(c->pinned, src, bytes);
  HIP_OK(c, hipMemcpyAsync(dst, c->pinned, bytes, hipMemcpyHostToDevice, st));
  HIP_OK(c, hipEventRecord(c->pinned_ev, st));
  c->pinned_pending = true;
  return CG_OK;
}

size_t store_size(int prec) { return prec == CG_F64 ? 8 : 4; }
size_t carry_size(int prec) { return prec == CG_F32 ? 4 : 8; }  // COMP, F64, F64ACC carry in double

// ---------------------------------------------------------------------------
// plans

struct Spec {
  const cg_map* map = nullptr;
  int N = 0;
  float2* xy = nullptr;
  float2* extra = nullptr;
  int64_t n_extra = 0;
  const float2* src_xy = nullptr;
  const float2* src_extra = nullptr;
  const float* values = nullptr;
  // caller-provided buffers (null: scratch)
  uint16_t* labels = nullptr;
  int64_t* counts = nullptr;
  float* lut = nullptr;
  int32_t n_lut = 0;
  const float* density = nullptr;
  void *S = nullptr, *T = nullptr, *HA = nullptr, *HB = nullptr;
  int64_t pitch = 0;
  double* areas = nullptr;
  float shape = 1.f, tol = 0.01f;
  int32_t area_source = CG_AREA_PIXEL, patience = 32, max_iters = 512, fixed_iters = 0;
  const float* init_field = nullptr;
  int64_t init_G = 0;
  double bg_mass = -1.0;    // prescribed background mass (eq.(4)), < 0: shape * d0
};

struct Needs {
  bool raster = false, sat = false, areas = false;
};

struct Plan {
  Batch B{};
  int prec = CG_F32, tw = 128, th = 16;
  bool dense = false;
  bool il = false;          // S and T interleaved as (S, T) pairs (the plan owns both tables)
  int n = 0;
  int64_t edge_blocks = 0, row_blocks = 0, tiles = 0, c1 = 0, c2 = 0, pt_blocks = 0, reg_blocks = 0;
  IterState* d_state = nullptr;
  std::vector<Inst> inst;
  bool fuse_lut = false;    // Step 3 built by the integral-image reduce pass (see lut_fusable)
  int emit_ept = 1;         // edges per thread of the rasteriser's emit pass
};

// Step 3 inside the integral-image reduce pass (one launch fewer) when
// every LUT fits its LDS and the redundant per-block builds are cheap:
// tiles x LUT entries summed over the batch up to 2^20 (measured: a single
// 1024^2 cartogram gains 5 us per iteration, a 64 x 2048^2 batch would
// lose 24 us).
bool lut_fusable(const Plan& P) {
  bool fuse = !P.dense;
  int64_t work = 0;
  for (const Inst& I : P.inst) {
    fuse = fuse && I.n_lut == I.R + 1 && I.n_lut <= cgk::kLutLds;
    const cgk::SatLayout L = cgk::sat_layout(I.N, P.tw, P.th);
    work += (int64_t)L.ntx * L.nty * I.n_lut;
  }
  return fuse && work <= ((int64_t)1 << 20);
}

int64_t pitch_of(int N) { return (int64_t)((N + 1 + 63) / 64) * 64; }

// Caller-provided device memory for a plan (the allocation-free entry
// point): scratch and descriptors are carved from it instead of the
// context's grow-only buffers, and the descriptors are written by a kernel
// from its arguments instead of a pinned staging copy.
struct Arena {
  char* base = nullptr;
  size_t bytes = 0;
};

// Descriptor bytes written from kernel arguments (one block).
constexpr int kBlobWords = 256;
struct Blob {
  uint32_t w[kBlobWords];
};
__global__ __launch_bounds__(256) void k_put_blob(uint32_t* dst, Blob b, int nwords) {
  for (int i = threadIdx.x; i < nwords; i += 256) dst[i] = b.w[i];
}

int build_plan(cg_ctx* c, const std::vector<Spec>& specs, int prec, int tw, int th, bool dense,
               const Needs& nd, hipStream_t st, Plan& P, const char* tag, const Arena* arena = nullptr) {
  const int n = (int)specs.size();
  P.n = n;
  P.prec = prec;
  P.tw = tw;
  P.th = th;
  P.dense = dense;
  P.inst.assign(n, Inst{});
  // the integral-image writer fills whole tile rows: every texture holds a
  // whole number of them (powers of two, tiles capped by cap_shape)
  if (nd.sat)
    for (const Spec& s : specs)
      if (th <= 0 || s.N % th != 0 || tw > std::max(64, s.N) ||
          2 * store_size(prec) * (size_t)(s.N + 1) * pitch_of(s.N) >= ((size_t)1 << 31))
        return fail(c, CG_EINVAL, "tile shape does not fit a texture of the batch");
  P.il = nd.sat && !dense;
  for (const Spec& s : specs) P.il = P.il && !s.S && !s.T;
  // scratch layout
  struct Own {
    int64_t rowcnt = -1, xing = -1, labels = -1, counts = -1, lut = -1, S = -1, T = -1,
            HA = -1, HB = -1, agg = -1, carry = -1, areas = -1;
  };
  std::vector<Own> owns(n);
  std::vector<size_t> base(n);
  size_t total = 0;
  for (int k = 0; k < n; ++k) {
    const Spec& s = specs[k];
    const int N = s.N;
    const int R = s.map ? s.map->R : 0;
    base[k] = total;
    size_t o = 0;
    auto take = [&](size_t bytes) -> int64_t {
      size_t at = o;
      o += align_up(bytes);
      return (int64_t)at;
    };
    Inst& I = P.inst[k];
    I.N = N;
    I.R = R;
    I.n_vert = s.map ? s.map->n_vert : 0;
    I.n_pts = (int32_t)(I.n_vert + s.n_extra);
    I.n_edges = s.map ? s.map->n_edges : 0;
    I.n_rings = s.map ? s.map->n_rings : 0;
    I.n_lut = s.lut && s.n_lut ? s.n_lut : R + 1;
    I.tw = tw;
    I.th = th;
    SatLayout L = cgk::sat_layout(N, tw, th);
    I.ntx = L.ntx;
    I.nty = L.nty;
    I.area_source = s.area_source;
    I.patience = s.patience;
    I.max_iters = s.max_iters;
    I.fixed_iters = s.fixed_iters;
    I.shape = s.shape;
    I.tol = s.tol;
    I.bg_mass = s.bg_mass;
    I.pitch = s.pitch ? s.pitch : pitch_of(N);
    I.xy = s.xy;
    I.extra = s.extra;
    I.src_xy = s.src_xy;
    I.src_extra = s.src_extra;
    I.init_field = s.init_field;
    I.init_G = s.init_G;
    I.values = s.values;
    I.density = s.density;
    if (s.map) {
      I.edges = s.map->d_edges;
      I.reg_pair_off = s.map->d_reg_pair_off;
      I.reg_pairs = s.map->d_reg_pairs;
    }
    // scratch offsets relative to the instance base (-1: caller buffer or unused)
    Own& ow = owns[k];
    if (nd.raster) {
      ow.rowcnt = take(sizeof(uint32_t) * N);
      ow.xing = take(sizeof(uint64_t) * (size_t)N * cgk::kFillXing);   // a bucket per row
    }
    if ((nd.raster || nd.sat) && !dense && !s.labels) ow.labels = take(sizeof(uint16_t) * (size_t)N * N);
    if (nd.raster && !s.counts) ow.counts = take(sizeof(int64_t) * (R + 1));
    if (!dense && !s.lut) ow.lut = take(sizeof(float) * (R + 1));
    if (nd.sat) {
      const size_t tb = store_size(prec) * (size_t)(N + 1) * I.pitch;
      if (P.il) {
        ow.S = take(2 * tb);    // (S, T) pairs; T is the second element
      } else {
        if (!s.S) ow.S = take(tb);
        if (!s.T) ow.T = take(tb);
      }
      if (!s.HA) ow.HA = take(store_size(prec) * (2 * N + 1));
      if (!s.HB) ow.HB = take(store_size(prec) * (2 * N + 1));
      ow.agg = take(carry_size(prec) * L.agg_elems);
      ow.carry = take(carry_size(prec) * L.carry_elems);
    }
    if (nd.areas && !s.areas) ow.areas = take(sizeof(double) * (R + 1));
    total += o;
    I.labels = s.labels;
    I.counts = s.counts;
    I.lut = s.lut;
    I.S = s.S;
    I.T = s.T;
    I.HA = s.HA;
    I.HB = s.HB;
    I.areas = s.areas;
  }
  char* ws = nullptr;
  int rc = CG_OK;
  if (arena) {
    if (total > arena->bytes)
      return fail(c, CG_EINVAL, "scratch of " + std::to_string(total) + " bytes exceeds the " +
                                    std::to_string(arena->bytes) + "-byte static buffer");
    ws = arena->base;
  } else {
    rc = get_buf(c, (std::string(tag) + ":scratch").c_str(), std::max<size_t>(total, 256), st, &ws);
    if (rc) return rc;
  }
  for (int k = 0; k < n; ++k) {
    Inst& I = P.inst[k];
    const Own& ow = owns[k];
    char* b = ws + base[k];
    auto at = [&](int64_t off) -> char* { return off >= 0 ? b + off : nullptr; };
    I.row_cnt = (uint32_t*)at(ow.rowcnt);
    I.xing = (uint64_t*)at(ow.xing);
    if (ow.labels >= 0) I.labels = (uint16_t*)at(ow.labels);
    if (ow.counts >= 0) I.counts = (int64_t*)at(ow.counts);
    if (ow.lut >= 0) I.lut = (float*)at(ow.lut);
    if (ow.S >= 0) I.S = at(ow.S);
    if (ow.T >= 0) I.T = at(ow.T);
    if (P.il) I.T = at(ow.S) + store_size(prec);
    if (ow.HA >= 0) I.HA = at(ow.HA);
    if (ow.HB >= 0) I.HB = at(ow.HB);
    I.agg = at(ow.agg);
    I.carry = at(ow.carry);
    if (ow.areas >= 0) I.areas = (double*)at(ow.areas);
  }
  // descriptors, offsets and states in one device buffer
  std::vector<int64_t> offs(8 * (size_t)(n + 1), 0);
  auto kind = [&](int kd) { return offs.data() + (size_t)kd * (n + 1); };
  // edges per emit thread: several once a launch holds many rounds of
  // blocks (more than 8192 single-edge blocks, 2M edges; measured: emit of
  // 64 x 2048^2 125 -> 90 us with 4, while a 1024^2 cartogram's 196 blocks
  // take 8 -> 12 us)
  {
    int64_t blocks1 = 0;
    for (const Inst& I : P.inst) blocks1 += std::max<int64_t>(1, (I.n_edges + 255) / 256);
    P.emit_ept = blocks1 > 8192 ? cgk::kEmitEdges : 1;
  }
  const int64_t edges_per_block = 256 * (int64_t)P.emit_ept;
  for (int k = 0; k < n; ++k) {
    const Inst& I = P.inst[k];
    SatLayout L = cgk::sat_layout(I.N, tw, th);
    // every instance gets an edge block: its first one clears the totals
    // the rasteriser's fill accumulates; with single-edge blocks that is
    // a block of its own, followed by one block per region (the previous
    // iteration's areas, inside the iteration loop), and the fill has a
    // block more (that iteration's stopping rule)
    const bool one = P.emit_ept == 1;
    const int64_t cnt[8] = {
        one ? (I.n_edges + edges_per_block - 1) / edges_per_block + 1 + I.R
            : std::max<int64_t>(1, (I.n_edges + edges_per_block - 1) / edges_per_block),
        (I.N + kFillRows - 1) / kFillRows + (one ? 1 : 0),
        (int64_t)L.ntx * L.nty,
        (L.NY + L.nty + 1 + 255) / 256,
        (L.NX + 1 + (int64_t)L.LA + L.LB + (256 / L.carry_ch) - 1) / (256 / L.carry_ch),
        std::max<int64_t>(1, (I.n_pts + 255) / 256),
        I.R,
        1};
    for (int kd = 0; kd < 8; ++kd) kind(kd)[k + 1] = kind(kd)[k] + cnt[kd];
  }
  // per kind: a block's instance is block / stride when every instance has
  // `stride` blocks of the kind; otherwise a table holds (instance, its
  // first block) for every block of the kind
  int32_t stride[cgk::KD_COUNT];
  size_t tab_at[cgk::KD_COUNT];
  size_t tab_words = 0;
  for (int kd = 0; kd < cgk::KD_COUNT; ++kd) {
    if (kind(kd)[n] > (int64_t)UINT32_MAX) return fail(c, CG_EINVAL, "batch too large: more than 2^32 blocks of one kind");
    const int64_t s0 = kind(kd)[1] - kind(kd)[0];
    bool eq = s0 > 0 && s0 < INT32_MAX;
    for (int k = 1; eq && k < n; ++k) eq = kind(kd)[k + 1] - kind(kd)[k] == s0;
    stride[kd] = eq ? (int32_t)s0 : 0;
    tab_at[kd] = tab_words;
    if (!eq) tab_words += 2 * (size_t)kind(kd)[n];
  }
  const size_t inst_bytes = align_up(sizeof(Inst) * n);
  const size_t off_bytes = align_up(sizeof(int64_t) * offs.size());
  const size_t tab_bytes = align_up(sizeof(uint32_t) * tab_words);
  const size_t st_bytes = align_up(sizeof(IterState) * n);
  char* desc = nullptr;
  if (arena) {
    const size_t at = align_up(total);
    if (at + inst_bytes + off_bytes + tab_bytes + st_bytes > arena->bytes)
      return fail(c, CG_EINVAL, "scratch and descriptors of " +
                                    std::to_string(at + inst_bytes + off_bytes + tab_bytes + st_bytes) +
                                    " bytes exceed the " + std::to_string(arena->bytes) + "-byte static buffer");
    if (inst_bytes + off_bytes + tab_bytes > sizeof(Blob))
      return fail(c, CG_EINVAL, "descriptors too large for an allocation-free call");
    desc = arena->base + at;
  } else {
    rc = get_buf(c, (std::string(tag) + ":desc").c_str(), inst_bytes + off_bytes + tab_bytes + st_bytes, st, &desc);
    if (rc) return rc;
  }
  P.d_state = (IterState*)(desc + inst_bytes + off_bytes + tab_bytes);
  for (int k = 0; k < n; ++k) P.inst[k].st = P.d_state + k;
  std::vector<char> host(inst_bytes + off_bytes + tab_bytes, 0);
  memcpy(host.data(), P.inst.data(), sizeof(Inst) * n);
  memcpy(host.data() + inst_bytes, offs.data(), sizeof(int64_t) * offs.size());
  uint32_t* tab = (uint32_t*)(host.data() + inst_bytes + off_bytes);
  for (int kd = 0; kd < cgk::KD_COUNT; ++kd) {
    if (stride[kd]) continue;
    uint32_t* t = tab + tab_at[kd];
    for (int k = 0; k < n; ++k)
      for (int64_t b = kind(kd)[k]; b < kind(kd)[k + 1]; ++b) {
        t[2 * b] = (uint32_t)k;
        t[2 * b + 1] = (uint32_t)kind(kd)[k];
      }
  }
  if (arena) {
    Blob blob;
    memset(&blob, 0, sizeof(blob));
    memcpy(blob.w, host.data(), host.size());
    hipLaunchKernelGGL(k_put_blob, dim3(1), dim3(256), 0, st, (uint32_t*)desc, blob,
                       (int)((host.size() + 3) / 4));
  } else {
    rc = upload(c, desc, host.data(), host.size(), st);
    if (rc) return rc;
  }
  const int64_t* doff = (const int64_t*)(desc + inst_bytes);
  const uint32_t* dtab = (const uint32_t*)(desc + inst_bytes + off_bytes);
  Batch& B = P.B;
  B.inst = (const Inst*)desc;
  B.n = n;
  B.skip_done = 1;
  B.max_n = 0;
  for (int k = 0; k < n; ++k) B.max_n = std::max(B.max_n, (int32_t)P.inst[k].N);
  B.make_lut = 0;
  B.states = P.d_state;
  for (int kd = 0; kd < cgk::KD_COUNT; ++kd) {
    B.stride[kd] = stride[kd];
    B.where[kd] = stride[kd] ? nullptr : dtab + tab_at[kd];
  }
  B.off_edges = doff + 0 * (n + 1);
  B.off_rows = doff + 1 * (n + 1);
  B.off_tiles = doff + 2 * (n + 1);
  B.off_carry1 = doff + 3 * (n + 1);
  B.off_carry2 = doff + 4 * (n + 1);
  B.off_pts = doff + 5 * (n + 1);
  B.off_regions = doff + 6 * (n + 1);
  B.off_inst = doff + 7 * (n + 1);
  P.edge_blocks = kind(0)[n];
  P.row_blocks = kind(1)[n];
  P.tiles = kind(2)[n];
  P.c1 = kind(3)[n];
  P.c2 = kind(4)[n];
  P.pt_blocks = kind(5)[n];
  P.reg_blocks = kind(6)[n];
  return CG_OK;
}

int default_shape(int N, int64_t batch_px, int* tw, int* th) {
  (void)batch_px;
  if (N <= 128) { *tw = 64; *th = 16; }
  else if (N <= 1024) { *tw = 128; *th = 16; }
  else { *tw = 128; *th = 32; }
  return CG_OK;
}

void shape_for(const cg_ctx* c, int N, int prec, int64_t batch_px, int* tw, int* th) {
  auto it = c->tiles.find(std::make_tuple(N, prec, batch_px));
  if (it == c->tiles.end()) {
    // nearest autotuned batch size for this (N, prec)
    int64_t best = -1;
    for (auto& kv : c->tiles) {
      if (std::get<0>(kv.first) == N && std::get<1>(kv.first) == prec) {
        const int64_t bp = std::get<2>(kv.first);
        if (best < 0 || std::llabs(bp - batch_px) < std::llabs(best - batch_px)) {
          best = bp;
          *tw = kv.second.first;
          *th = kv.second.second;
        }
      }
    }
    if (best >= 0) return;
    default_shape(N, batch_px, tw, th);
    return;
  }
  *tw = it->second.first;
  *th = it->second.second;
}

// Tiles never wider than the narrowest texture of a launch (64 at least):
// then every tile column lies inside the table's pitch, and the integral-
// image writer stores whole tile rows without a per-column bound check
// (columns past N land in the row padding).
void cap_shape(int minN, int* tw, int* th) {
  const int cap = std::max(64, minN);
  if (*tw <= cap) return;
  *tw = cap;
  if (cap == 64) *th = 16;
  else if (*th > 32) *th = 32;
}

struct HookCtx {
  cg_ctx* c;
  int it;
};

void prof_hook(int stage, int after, void* user) {
  HookCtx* h = (HookCtx*)user;
  if (stage != h->c->prof_stage || h->it % h->c->prof_every != 0) return;
  hipEventRecord(h->c->prof_ev[2 * h->it + after], h->c->prof_stream);
  if (after) h->c->prof_rec[h->it] = 1;
}

void launch_iteration(const Plan& P, hipStream_t st, cg_ctx* c, int it) {
  HookCtx hc{c, it};
  const bool prof = c && c->prof_stage >= 0;
  cgk::StageHook h = prof ? prof_hook : nullptr;
  void* u = prof ? (void*)&hc : nullptr;
  auto hk = [&](int s, int after) { if (h) h(s, after, u); };
  // with single-edge emit blocks the previous iteration's areas are
  // computed in the emit pass and its stopping rule runs in the fill, and
  // the last iteration's follow the loop (launch_rule); else each
  // iteration ends with its own
  const bool fold = P.emit_ept == 1;
  cgk::launch_raster(P.B, P.emit_ept, P.edge_blocks, P.row_blocks, st, h, u, fold && it > 0);
  const bool fuse = P.fuse_lut;
  cgk::Batch Bl = P.B;
  if (fuse) {
    Bl.make_lut = 1;
  } else {
    hk(cgk::ST_DENSITY, 0);
    cgk::launch_density(P.B, st);
    hk(cgk::ST_DENSITY, 1);
  }
  cgk::launch_sat(Bl, P.prec, P.tw, P.th, false, P.il, P.tiles, P.c1, P.c2, st, h, u);
  hk(cgk::ST_MAP, 0);
  cgk::launch_map(P.B, P.prec, P.il, P.pt_blocks, st);
  hk(cgk::ST_MAP, 1);
  if (!fold) {
    hk(cgk::ST_AREAS, 0);
    cgk::launch_areas(P.B, P.reg_blocks, st);
    hk(cgk::ST_AREAS, 1);
    hk(cgk::ST_ERR, 0);
    cgk::launch_err(P.B, 0, st);
    hk(cgk::ST_ERR, 1);
  }
}

// The areas and the stopping rule after the last of a run of iterations
// whose earlier ones ran in the next iteration's emit pass and fill.
// Timed in the first iteration's event slots (the stages have no other
// launches to time).
void launch_rule(const Plan& P, hipStream_t st, cg_ctx* c) {
  if (P.emit_ept != 1) return;   // each iteration ended with its own
  HookCtx hc{c, 0};
  const bool prof = c && c->prof_stage >= 0;
  if (prof) prof_hook(cgk::ST_AREAS, 0, &hc);
  cgk::launch_areas(P.B, P.reg_blocks, st);
  if (prof) prof_hook(cgk::ST_AREAS, 1, &hc);
  if (prof) prof_hook(cgk::ST_ERR, 0, &hc);
  cgk::launch_err(P.B, 0, st);
  if (prof) prof_hook(cgk::ST_ERR, 1, &hc);
}

int check_launch(cg_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, CG_EDEVICE, std::string("kernel launch: ") + hipGetErrorString(e));
  return CG_OK;
}

}  // namespace

// ===========================================================================
// Static device scratch of the allocation-free entry point
// (cg_integral_image_noalloc).  Every GPU the library runs on holds its own
// copy until the process ends.  Host code never uses the array's name as a
// device address: cg_create looks up each device's copy once, with that
// device current, and every later use goes through that address.

constexpr size_t kNoAllocBytes = (size_t)24 << 20;
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// Called by cg_create with `device` current.
void scratch_lookup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess) g_scratch_ptr[device] = p;
  else (void)hipGetLastError();   // the entry point then reports CG_EDEVICE
}

void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

int inim_args(cg_ctx* c, int N, const uint16_t* labels, const float* lut, int32_t n_lut, const float* density,
              int precision, const cg_inim* out, const char* who) {
  const std::string w(who);
  if (!out || !out->S || !out->T || !out->HA || !out->HB) return fail(c, CG_EINVAL, w + ": output buffers missing");
  if (!pow2_ok(N)) return fail(c, CG_EINVAL, w + ": N must be a power of two in [16, 8192]");
  if (precision < CG_F32 || precision > CG_F64ACC) return fail(c, CG_EINVAL, w + ": bad precision");
  if (!density && (!labels || !lut || n_lut < 1 || n_lut > 65536))
    return fail(c, CG_EINVAL, w + ": need labels + lut (1 <= n_lut <= 65536) or a density texture");
  if (((uintptr_t)labels | (uintptr_t)density) & 15)
    return fail(c, CG_EINVAL, w + ": labels / density must be 16-byte aligned");
  return CG_OK;
}

// One integral-image call: plan (from the context's buffers, or from
// `arena`) and the launches of the three passes.
int inim_run(cg_ctx* c, int N, const uint16_t* labels, const float* lut, int32_t n_lut, const float* density,
             int precision, cg_inim* out, hipStream_t st, const Arena* arena) {
  int tw, th;
  shape_for(c, N, precision, (int64_t)N * N, &tw, &th);
  cap_shape(N, &tw, &th);
  Spec s;
  s.N = N;
  s.labels = (uint16_t*)labels;
  s.lut = (float*)lut;
  s.n_lut = n_lut;
  s.density = density;
  s.S = out->S;
  s.T = out->T;
  s.HA = out->HA;
  s.HB = out->HB;
  s.pitch = pitch_of(N);
  Needs nd;
  nd.sat = true;
  Plan P;
  int rc = build_plan(c, {s}, precision, tw, th, density != nullptr, nd, st, P, "call", arena);
  if (rc) return rc;
  P.B.skip_done = 0;
  if (!cgk::launch_sat(P.B, precision, tw, th, density != nullptr, P.il, P.tiles, P.c1, P.c2, st, nullptr, nullptr))
    return fail(c, CG_EUNSUPPORTED, "integral image: unsupported tile shape");
  out->N = N;
  out->precision = precision;
  out->pitch = s.pitch;
  return check_launch(c);
}

}  // namespace

// ===========================================================================
// C ABI

extern "C" {

int cg_create(int device, cg_ctx** out) {
  if (!out) return CG_EINVAL;
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) return CG_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return CG_EDEVICE;
  cg_ctx* c = new cg_ctx();
  c->device = device;
  scratch_lookup(device);
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->pinned_ev, hipEventDisableTiming) != hipSuccess) {
    delete c;
    return CG_EDEVICE;
  }
  *out = c;
  return CG_OK;
}

int cg_destroy(cg_ctx* c) {
  if (!c) return CG_EINVAL;
  hipSetDevice(c->device);
  hipDeviceSynchronize();
  for (auto& kv : c->bufs)
    if (kv.second.p) hipFree(kv.second.p);
  if (c->pinned) hipHostFree(c->pinned);
  if (c->pinned_ev) hipEventDestroy(c->pinned_ev);
  for (auto& e : c->graphs) hipGraphExecDestroy(e.exec);
  if (c->st_pinned) hipHostFree(c->st_pinned);
  if (c->stream) hipStreamDestroy(c->stream);
  delete c;
  return CG_OK;
}

const char* cg_last_error(const cg_ctx* c) { return c ? c->err.c_str() : "null context"; }

void* cg_stream(const cg_ctx* c) { return c ? (void*)c->stream : nullptr; }

int cg_map_build(cg_ctx* c, int32_t n_vertices, int32_t n_regions, int32_t n_rings,
                 const int32_t* ring_off, const int32_t* ring_idx, const int32_t* ring_reg,
                 cg_map** out) {
  if (!c || !out) return CG_EINVAL;
  *out = nullptr;
  if (n_vertices < 0 || n_regions < 0 || n_regions > 65534 || n_rings < 0 || !ring_off ||
      (n_rings > 0 && (!ring_idx || !ring_reg)))
    return fail(c, CG_EINVAL, "cg_map_build: bad sizes or null arrays");
  if (ring_off[0] != 0) return fail(c, CG_EINVAL, "cg_map_build: ring_off[0] must be 0");
  for (int r = 0; r < n_rings; ++r) {
    if (ring_off[r + 1] < ring_off[r] + 3) return fail(c, CG_EINVAL, "cg_map_build: a ring has fewer than 3 vertices");
    if (ring_reg[r] < 1 || ring_reg[r] > n_regions) return fail(c, CG_EINVAL, "cg_map_build: ring region out of range");
  }
  const int32_t total = ring_off[n_rings];
  for (int i = 0; i < total; ++i)
    if (ring_idx[i] < 0 || ring_idx[i] >= n_vertices) return fail(c, CG_EINVAL, "cg_map_build: vertex index out of range");
  // unique edges with the regions on both sides
  std::map<std::pair<int, int>, std::vector<int>> owner;
  for (int r = 0; r < n_rings; ++r) {
    const int b = ring_off[r], len = ring_off[r + 1] - b;
    for (int k = 0; k < len; ++k) {
      const int a = ring_idx[b + k], bb = ring_idx[b + (k + 1) % len];
      if (a == bb) continue;
      owner[{std::min(a, bb), std::max(a, bb)}].push_back(ring_reg[r]);
    }
  }
  std::vector<int4> edges;
  edges.reserve(owner.size());
  for (auto& kv : owner) {
    if (kv.second.size() > 2) return fail(c, CG_EINVAL, "cg_map_build: an edge is used by more than two rings");
    int ra = kv.second[0], rb = kv.second.size() > 1 ? kv.second[1] : 0;
    if (ra == rb) continue;  // both sides the same region: never changes membership
    edges.push_back(make_int4(kv.first.first, kv.first.second, ra, rb));
  }
  // region -> ring edges (a, b), the rings of a region in input order: the
  // shoelace sum of a region is one pass over a contiguous list
  std::vector<int32_t> reg_off(n_regions + 1, 0);
  for (int r = 0; r < n_rings; ++r) reg_off[ring_reg[r]] += ring_off[r + 1] - ring_off[r];
  for (int v = 1; v <= n_regions; ++v) reg_off[v] += reg_off[v - 1];
  std::vector<int2> reg_pairs((size_t)total);
  {
    std::vector<int32_t> pos(reg_off.begin(), reg_off.end() - 1);
    for (int r = 0; r < n_rings; ++r) {
      const int beg = ring_off[r], len = ring_off[r + 1] - beg;
      int32_t& p = pos[ring_reg[r] - 1];
      for (int e = 0; e < len; ++e) reg_pairs[p++] = make_int2(ring_idx[beg + e], ring_idx[beg + (e + 1 == len ? 0 : e + 1)]);
    }
  }
  cg_map* m = new cg_map();
  m->device = c->device;
  m->n_vert = n_vertices;
  m->R = n_regions;
  m->n_rings = n_rings;
  m->n_edges = (int32_t)edges.size();
  hipSetDevice(c->device);
  auto put = [&](void** dst, const void* src, size_t bytes) -> bool {
    if (hipMalloc(dst, std::max<size_t>(bytes, 16)) != hipSuccess) return false;
    if (bytes && hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) return false;
    return true;
  };
  bool ok = put((void**)&m->d_edges, edges.data(), sizeof(int4) * edges.size()) &&
            put((void**)&m->d_reg_pair_off, reg_off.data(), sizeof(int32_t) * reg_off.size()) &&
            put((void**)&m->d_reg_pairs, reg_pairs.data(), sizeof(int2) * reg_pairs.size());
  if (!ok) {
    cg_map_destroy(m);
    return fail(c, CG_ENOMEM, "cg_map_build: device allocation failed");
  }
  *out = m;
  return CG_OK;
}

int cg_map_destroy(cg_map* m) {
  if (!m) return CG_EINVAL;
  // the map owns its buffers and records its device: destroying it after
  // its context is fine
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  hipFree(m->d_edges);
  hipFree(m->d_reg_pair_off);
  hipFree(m->d_reg_pairs);
  delete m;
  return CG_OK;
}

int32_t cg_map_n_edges(const cg_map* m) { return m ? m->n_edges : -1; }

int cg_rasterize(cg_ctx* c, const cg_map* map, const float* xy, int N, uint16_t* labels,
                 int64_t* counts, int64_t* contested, void* stream) {
  if (!c) return CG_EINVAL;
  if (!map || !xy || !labels) return fail(c, CG_EINVAL, "cg_rasterize: null argument");
  if (!pow2_ok(N)) return fail(c, CG_EINVAL, "cg_rasterize: N must be a power of two in [16, 8192]");
  hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  Spec s;
  s.map = map;
  s.N = N;
  s.xy = (float2*)xy;
  s.labels = labels;
  s.counts = counts;
  Needs nd;
  nd.raster = true;
  Plan P;
  int rc = build_plan(c, {s}, CG_F32, 64, 16, false, nd, st, P, "call");
  if (rc) return rc;
  P.B.skip_done = 0;
  cgk::launch_init(P.B, P.pt_blocks, st);
  cgk::launch_raster(P.B, P.emit_ept, P.edge_blocks, P.row_blocks, st, nullptr, nullptr);
  if (contested) cgk::launch_export(P.B, contested, nullptr, st);
  return check_launch(c);
}

int cg_inim_size(int N, int precision, int64_t* pitch, size_t* table_bytes, size_t* marginal_bytes) {
  if (!pow2_ok(N) || precision < CG_F32 || precision > CG_F64ACC) return CG_EINVAL;
  const int64_t p = pitch_of(N);
  if (pitch) *pitch = p;
  if (table_bytes) *table_bytes = store_size(precision) * (size_t)(N + 1) * p;
  if (marginal_bytes) *marginal_bytes = store_size(precision) * (size_t)(2 * N + 1);
  return CG_OK;
}

int cg_integral_image(cg_ctx* c, int N, const uint16_t* labels, const float* lut, int32_t n_lut,
                      const float* density, int precision, cg_inim* out, void* stream) {
  if (!c) return CG_EINVAL;
  int rc = inim_args(c, N, labels, lut, n_lut, density, precision, out, "cg_integral_image");
  if (rc) return rc;
  hipSetDevice(c->device);
  return inim_run(c, N, labels, lut, n_lut, density, precision, out, pick_stream(c, stream), nullptr);
}

int cg_integral_image_noalloc(cg_ctx* c, int N, const uint16_t* labels, const float* lut, int32_t n_lut,
                              const float* density, int precision, cg_inim* out, void* stream) {
  if (!c) return CG_EINVAL;
  int rc = inim_args(c, N, labels, lut, n_lut, density, precision, out, "cg_integral_image_noalloc");
  if (rc) return rc;
  Arena a;
  a.base = (char*)scratch_ptr(c->device);
  a.bytes = kNoAllocBytes;
  if (!a.base) return fail(c, CG_EDEVICE, "cg_integral_image_noalloc: static scratch unavailable on this device");
  hipSetDevice(c->device);
  return inim_run(c, N, labels, lut, n_lut, density, precision, out, pick_stream(c, stream), &a);
}

int cg_map_points(cg_ctx* c, const cg_inim* im, const float* xy_in, float* xy_out, int64_t n_points,
                  void* stream) {
  if (!c) return CG_EINVAL;
  if (!im || !xy_in || !xy_out || n_points < 0) return fail(c, CG_EINVAL, "cg_map_points: bad arguments");
  if (!pow2_ok(im->N) || im->precision < CG_F32 || im->precision > CG_F64ACC || im->pitch < im->N + 1 ||
      !im->S || !im->T || !im->HA || !im->HB)
    return fail(c, CG_EINVAL, "cg_map_points: bad integral-image descriptor");
  if (n_points == 0) return CG_OK;
  if (n_points > INT32_MAX) return fail(c, CG_EINVAL, "cg_map_points: too many points");
  hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  Spec s;
  s.N = im->N;
  s.S = im->S;
  s.T = im->T;
  s.HA = im->HA;
  s.HB = im->HB;
  s.pitch = im->pitch;
  s.xy = (float2*)xy_out;
  s.src_xy = (const float2*)xy_in;
  Needs nd;
  Plan P;
  // a map-less instance: n_pts comes from n_extra with no vertices
  s.extra = (float2*)xy_out;
  s.src_extra = (const float2*)xy_in;
  s.n_extra = n_points;
  s.xy = nullptr;
  s.src_xy = nullptr;
  int rc = build_plan(c, {s}, im->precision, 64, 16, false, nd, st, P, "call");
  if (rc) return rc;
  P.B.skip_done = 0;
  cgk::launch_init(P.B, P.pt_blocks, st);
  cgk::launch_map(P.B, im->precision, P.il, P.pt_blocks, st);
  return check_launch(c);
}

int cg_region_areas(cg_ctx* c, const cg_map* map, const float* xy, const float* values, double* areas,
                    double* eps_xi, void* stream) {
  if (!c) return CG_EINVAL;
  if (!map || !xy || !areas) return fail(c, CG_EINVAL, "cg_region_areas: null argument");
  if (eps_xi && !values) return fail(c, CG_EINVAL, "cg_region_areas: eps_xi needs values");
  hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  Spec s;
  s.map = map;
  s.N = 16;
  s.xy = (float2*)xy;
  s.values = values;
  s.areas = areas;
  Needs nd;
  nd.areas = true;
  Plan P;
  int rc = build_plan(c, {s}, CG_F32, 64, 16, false, nd, st, P, "call");
  if (rc) return rc;
  P.B.skip_done = 0;
  cgk::launch_init(P.B, P.pt_blocks, st);
  cgk::launch_areas(P.B, P.reg_blocks, st);
  if (values) {
    cgk::launch_err(P.B, 1, st);
    if (eps_xi) cgk::launch_export(P.B, nullptr, eps_xi, st);
  }
  return check_launch(c);
}

static const int kShapes[][2] = {{64, 16}, {128, 16}, {128, 32}, {256, 32}, {256, 64}};

int cg_set_tile_shape(cg_ctx* c, int N, int precision, int64_t batch_pixels, int32_t tw, int32_t th) {
  if (!c) return CG_EINVAL;
  if (!pow2_ok(N) || precision < CG_F32 || precision > CG_F64ACC || batch_pixels < 0 ||
      !cgk::sat_shape_supported(tw, th))
    return fail(c, CG_EINVAL, "cg_set_tile_shape: bad arguments or unsupported shape");
  c->tiles[std::make_tuple(N, precision, batch_pixels)] = {tw, th};
  return CG_OK;
}

int cg_autotune(cg_ctx* c, int N, int precision, int32_t batch, const char* cache_path) {
  if (!c) return CG_EINVAL;
  if (!pow2_ok(N) || precision < CG_F32 || precision > CG_F64ACC || batch < 1 || batch > 4096)
    return fail(c, CG_EINVAL, "cg_autotune: bad arguments");
  const int64_t px = (int64_t)N * N * batch;
  hipDeviceProp_t prop;
  HIP_OK(c, hipGetDeviceProperties(&prop, c->device));
  const std::string arch = prop.gcnArchName;
  std::string key;
  {
    std::ostringstream os;
    os << arch.substr(0, arch.find(':')) << " " << N << " " << precision << " " << px;
    key = os.str();
  }
  if (cache_path) {  // "arch N precision batch_pixels tw th" per line
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream is(line);
      std::string a;
      int n, p, tw, th;
      int64_t b;
      if (is >> a >> n >> p >> b >> tw >> th) {
        std::ostringstream os;
        os << a << " " << n << " " << p << " " << b;
        if (os.str() == key && cgk::sat_shape_supported(tw, th)) {
          c->tiles[std::make_tuple(N, precision, px)] = {tw, th};
          return CG_OK;
        }
      }
    }
  }
  hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, nullptr);
  // synthetic batch: a label map with a few regions, one LUT
  char* lab = nullptr;
  int rc = get_buf(c, "tune:labels", sizeof(uint16_t) * (size_t)N * N, st, &lab);
  if (rc) return rc;
  char* lut = nullptr;
  if ((rc = get_buf(c, "tune:lut", sizeof(float) * 4, st, &lut))) return rc;
  const float lutv[4] = {1.0f, 3.0f, 0.25f, 7.0f};
  std::vector<uint16_t> hl((size_t)N * N);
  for (int q = 0; q < N; ++q)
    for (int p = 0; p < N; ++p) hl[(size_t)q * N + p] = (uint16_t)(((p * 7) / N + (q * 5) / N) & 3);
  HIP_OK(c, hipMemcpyAsync(lab, hl.data(), hl.size() * sizeof(uint16_t), hipMemcpyHostToDevice, st));
  HIP_OK(c, hipMemcpyAsync(lut, lutv, sizeof(lutv), hipMemcpyHostToDevice, st));
  HIP_OK(c, hipStreamSynchronize(st));
  hipEvent_t e0, e1;
  HIP_OK(c, hipEventCreate(&e0));
  HIP_OK(c, hipEventCreate(&e1));
  float best = 1e30f;
  int btw = 0, bth = 0;
  for (auto& sh : kShapes) {
    const int tw = sh[0], th = sh[1];
    if (tw > std::max(64, N)) continue;
    std::vector<Spec> specs(batch);
    for (auto& sp : specs) {
      sp.N = N;
      sp.labels = (uint16_t*)lab;
      sp.lut = (float*)lut;
      sp.n_lut = 4;
    }
    Needs nd;
    nd.sat = true;
    Plan P;
    if ((rc = build_plan(c, specs, precision, tw, th, false, nd, st, P, "tune"))) break;
    P.B.skip_done = 0;
    for (int w = 0; w < 2; ++w) cgk::launch_sat(P.B, precision, tw, th, false, P.il, P.tiles, P.c1, P.c2, st, nullptr, nullptr);
    const int reps = 5;
    hipEventRecord(e0, st);
    for (int r = 0; r < reps; ++r) cgk::launch_sat(P.B, precision, tw, th, false, P.il, P.tiles, P.c1, P.c2, st, nullptr, nullptr);
    hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) { rc = fail(c, CG_EDEVICE, "cg_autotune: device error"); break; }
    float ms = 0.f;
    hipEventElapsedTime(&ms, e0, e1);
    ms /= reps;
    if (ms < best) { best = ms; btw = tw; bth = th; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc) return rc;
  if ((rc = check_launch(c))) return rc;
  c->tiles[std::make_tuple(N, precision, px)] = {btw, bth};
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    out << key << " " << btw << " " << bth << "\n";
  }
  return CG_OK;
}

static const char* kStageNames[cgk::ST_COUNT] = {
    "raster_emit", "raster_fill", "density", "sat_reduce",
    "sat_carry1", "sat_carry2", "sat_final", "map_points", "areas", "err"};

int cg_profile_stage(cg_ctx* c, const char* stage, int32_t every) {
  if (!c) return CG_EINVAL;
  if (every < 1) return fail(c, CG_EINVAL, "cg_profile_stage: every must be >= 1");
  c->prof_every = every;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  c->prof_failed = 0;
  if (!stage || !*stage) {
    c->prof_stage = -1;
    return CG_OK;
  }
  for (int i = 0; i < cgk::ST_COUNT; ++i)
    if (strcmp(stage, kStageNames[i]) == 0) {
      c->prof_stage = i;
      return CG_OK;
    }
  return fail(c, CG_EINVAL, std::string("cg_profile_stage: unknown stage ") + stage);
}

int cg_profile_read(cg_ctx* c, double* total_ms, int64_t* launches) {
  if (!c) return CG_EINVAL;
  if (total_ms) *total_ms = c->prof_ms;
  if (launches) *launches = c->prof_launches;
  return CG_OK;
}

int cg_log_density(cg_ctx* c, int N, const uint16_t* labels, const int64_t* counts, const float* values,
                   int32_t n_regions, float shape, float* out, void* stream) {
  if (!c) return CG_EINVAL;
  if (!labels || !counts || !values || !out) return fail(c, CG_EINVAL, "cg_log_density: null argument");
  if (!pow2_ok(N)) return fail(c, CG_EINVAL, "cg_log_density: N must be a power of two in [16, 8192]");
  if (n_regions < 1 || n_regions > 65535 || !(shape >= 0))
    return fail(c, CG_EINVAL, "cg_log_density: need 1 <= n_regions <= 65535 and shape >= 0");
  (void)hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  char* lut = nullptr;
  int rc = get_buf(c, "log_lut", sizeof(float) * (size_t)(n_regions + 1), st, &lut);
  if (rc) return rc;
  cgk::launch_log_density(labels, counts, values, n_regions, N, shape, (float*)lut, out, st);
  return check_launch(c);
}

int cg_log_density_maps(cg_ctx* c, int32_t n, const cg_map* const* maps, const float* const* xy, int N,
                        const float* const* values, float shape, float* out, void* stream) {
  if (!c) return CG_EINVAL;
  if (n < 1 || !maps || !xy || !values || !out) return fail(c, CG_EINVAL, "cg_log_density_maps: null argument");
  if (!pow2_ok(N)) return fail(c, CG_EINVAL, "cg_log_density_maps: N must be a power of two in [16, 8192]");
  if (!(shape >= 0)) return fail(c, CG_EINVAL, "cg_log_density_maps: need shape >= 0");
  int32_t maxR = 0;
  std::vector<Spec> specs(n);
  for (int k = 0; k < n; ++k) {
    if (!maps[k] || !xy[k] || !values[k]) return fail(c, CG_EINVAL, "cg_log_density_maps: null map, positions or values");
    if (maps[k]->R < 1 || maps[k]->R > 65535) return fail(c, CG_EINVAL, "cg_log_density_maps: need 1 <= R <= 65535");
    maxR = std::max(maxR, maps[k]->R);
    specs[k].map = maps[k];
    specs[k].N = N;
    specs[k].xy = (float2*)xy[k];
  }
  (void)hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  Needs nd;
  nd.raster = true;
  Plan P;
  int rc = build_plan(c, specs, CG_F32, 64, 16, false, nd, st, P, "logd");
  if (rc) return rc;
  P.B.skip_done = 0;
  cgk::launch_init(P.B, P.pt_blocks, st);
  cgk::launch_raster(P.B, P.emit_ept, P.edge_blocks, P.row_blocks, st, nullptr, nullptr);
  char* lut = nullptr;
  if ((rc = get_buf(c, "log_lut", sizeof(float) * (size_t)(maxR + 1), st, &lut))) return rc;
  for (int k = 0; k < n; ++k)   // stream order: each launch has the LUT scratch to itself
    cgk::launch_log_density(P.inst[k].labels, P.inst[k].counts, values[k], maps[k]->R, N, shape, (float*)lut,
                            out + (size_t)k * N * N, st);
  return check_launch(c);
}

int cg_tracer_field(cg_ctx* c, int32_t G, const float* final_xy, float* out, void* stream) {
  if (!c) return CG_EINVAL;
  if (!out || G < 1 || G > 65536) return fail(c, CG_EINVAL, "cg_tracer_field: need out and 1 <= G <= 65536");
  (void)hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  cgk::launch_tracer_field(G, final_xy, out, st);
  return check_launch(c);
}

int cg_field_pool(cg_ctx* c, int32_t G, const float* in, int32_t factor, float* out, void* stream) {
  if (!c) return CG_EINVAL;
  if (!in || !out || G < 1 || factor < 1 || G % factor != 0)
    return fail(c, CG_EINVAL, "cg_field_pool: need in, out and a factor dividing G");
  (void)hipSetDevice(c->device);
  hipStream_t st = pick_stream(c, stream);
  cgk::launch_field_pool(G, factor, in, out, st);
  return check_launch(c);
}

int cg_tile_shape(const cg_ctx* c, int N, int precision, int64_t batch_pixels, int32_t* tw, int32_t* th) {
  if (!c || !tw || !th || !pow2_ok(N)) return CG_EINVAL;
  int a, b;
  shape_for(c, N, precision, batch_pixels, &a, &b);
  cap_shape(N, &a, &b);
  *tw = a;
  *th = b;
  return CG_OK;
}

}  // extern "C"

// ===========================================================================
// series driver

namespace {

// Where a cartogram's results go: time step `slot` >= 0, or value-
// interpolated frame f = -1 - slot (transition t-1 -> t, frame k:
// f = (t-1)(K-1) + k-1).
struct StepRef {
  int series, slot;
};

int run_batch(cg_ctx* c, const std::vector<Spec>& specs, const std::vector<StepRef>& refs,
              const cg_series_desc* desc, cg_series_out* out, int prec, int graph_iters, hipStream_t st) {
  if (specs.empty()) return CG_OK;
  int64_t px = 0;
  int maxN = 0;
  for (auto& s : specs) {
    px += (int64_t)s.N * s.N;
    maxN = std::max(maxN, s.N);
  }
  int tw, th;
  shape_for(c, maxN, prec, px, &tw, &th);
  int minN = maxN;
  for (auto& s : specs) minN = std::min(minN, s.N);
  cap_shape(minN, &tw, &th);
  Needs nd;
  nd.raster = nd.sat = nd.areas = true;
  Plan P;
  int rc = build_plan(c, specs, prec, tw, th, false, nd, st, P, "series");
  if (rc) return rc;
  P.fuse_lut = lut_fusable(P);
  const int n = P.n;
  cgk::launch_init(P.B, P.pt_blocks, st);
  bool warm = false;
  for (auto& s : specs) warm = warm || s.init_field != nullptr;
  if (warm) {
    // warm start: error of the plain start, then trial steps alpha * field
    // (each rasterised for the fold check and scored by its max area
    // error), then the best non-folding step, or the plain start
    static const float kAlphas[] = {1.0f, 0.75f, 0.5f, 0.25f};
    cgk::launch_areas(P.B, P.reg_blocks, st);
    cgk::launch_err(P.B, 2, st);
    for (float a : kAlphas) {
      cgk::launch_restore(P.B, P.pt_blocks, st);
      cgk::launch_apply_field(P.B, P.pt_blocks, a, st);
      cgk::launch_raster(P.B, P.emit_ept, P.edge_blocks, P.row_blocks, st, nullptr, nullptr);
      cgk::launch_areas(P.B, P.reg_blocks, st);
      cgk::launch_err(P.B, 3, st, a);
    }
    cgk::launch_restore(P.B, P.pt_blocks, st);
    cgk::launch_apply_field(P.B, P.pt_blocks, -1.f, st);
    cgk::launch_err(P.B, 4, st);
  }
  cgk::launch_areas(P.B, P.reg_blocks, st);
  cgk::launch_err(P.B, 0, st);
  if ((rc = check_launch(c))) return rc;
  // capture the iteration body once (graph_iters < 0: launch eagerly,
  // |graph_iters| iterations between convergence polls)
  const bool eager = graph_iters < 0;
  const int K = graph_iters > 0 ? graph_iters : (graph_iters < 0 ? -graph_iters : 8);
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const bool prof = c->prof_stage >= 0;
  if (prof) {
    while ((int)c->prof_ev.size() < 2 * K) {
      hipEvent_t e;
      HIP_OK(c, hipEventCreate(&e));
      c->prof_ev.push_back(e);
    }
    c->prof_k = K;
    c->prof_rec.assign(K, 0);
    c->prof_stream = st;
  }
  bool cached = false;   // exec belongs to the context's graph cache
  if (!eager) {
    // the captured iteration reads every per-call value (descriptors,
    // states) from device memory: a call with the same launches (same
    // batch descriptor, buffer addresses, grids, tile shape, chunk length,
    // stream) replays the graph instantiated for an earlier one
    GraphKey key;
    memset(&key, 0, sizeof(key));
    key.B = P.B;
    key.prec = P.prec;
    key.tw = P.tw;
    key.th = P.th;
    key.il = P.il ? 1 : 0;
    key.fuse = P.fuse_lut ? 1 : 0;
    key.K = K;
    key.ept = P.emit_ept;
    key.blocks[0] = P.edge_blocks;
    key.blocks[1] = P.row_blocks;
    key.blocks[2] = P.tiles;
    key.blocks[3] = P.c1;
    key.blocks[4] = P.c2;
    key.blocks[5] = P.pt_blocks;
    key.blocks[6] = P.reg_blocks;
    key.stream = st;
    if (!prof)
      for (auto& e : c->graphs)
        if (memcmp(&e.key, &key, sizeof(key)) == 0) {
          exec = e.exec;
          cached = true;
        }
    if (!exec) {
      HIP_OK(c, hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
      for (int it = 0; it < K; ++it) launch_iteration(P, st, c, it);
      launch_rule(P, st, c);
      HIP_OK(c, hipStreamEndCapture(st, &graph));
      HIP_OK(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
      if (!prof) {
        if (c->graphs.size() >= 8) {   // keep the most recent few
          (void)hipGraphExecDestroy(c->graphs.front().exec);
          c->graphs.erase(c->graphs.begin());
        }
        c->graphs.push_back(GraphEntry{key, exec});
        cached = true;
      }
    }
  }
  std::vector<IterState> hs(n);
  if (c->st_pinned_n < (size_t)n) {   // pinned state buffer of the convergence polls, kept by the context
    if (c->st_pinned) (void)hipHostFree(c->st_pinned);
    c->st_pinned = nullptr;
    c->st_pinned_n = 0;
    HIP_OK(c, hipHostMalloc(&c->st_pinned, sizeof(IterState) * n, hipHostMallocDefault));
    c->st_pinned_n = n;
  }
  IterState* pinned = (IterState*)c->st_pinned;
  int max_budget = 0;
  for (auto& s : specs) max_budget = std::max(max_budget, s.fixed_iters > 0 ? s.fixed_iters : s.max_iters);
  int launched = 0;
  rc = CG_OK;
  while (true) {
    if (hipMemcpyAsync(pinned, P.d_state, sizeof(IterState) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      rc = fail(c, CG_EDEVICE, "cg_step_series: device error while iterating");
      break;
    }
    if (prof && launched > 0) {
      for (int it = 0; it < K; it += c->prof_every) {
        if (!c->prof_rec[it]) continue;   // the stage was not launched (folded into another kernel)
        c->prof_rec[it] = 0;
        float ms = 0.f;
        hipError_t e = hipEventElapsedTime(&ms, c->prof_ev[2 * it], c->prof_ev[2 * it + 1]);
        if (e == hipSuccess) {
          c->prof_ms += ms;
          c->prof_launches += 1;
        } else {
          (void)hipGetLastError();  // timing unavailable for this replay; leave no sticky error
          c->prof_failed += 1;
        }
      }
    }
    bool all = true;
    for (int k = 0; k < n; ++k) all = all && pinned[k].done;
    if (all) break;
    if (launched > max_budget + 2 * K) {
      rc = fail(c, CG_EDEVICE, "cg_step_series: iteration budget exceeded without stopping");
      break;
    }
    if (eager) {
      for (int it = 0; it < K; ++it) launch_iteration(P, st, c, it);
      launch_rule(P, st, c);
      if ((rc = check_launch(c))) break;
    } else if (hipGraphLaunch(exec, st) != hipSuccess) {
      rc = fail(c, CG_EDEVICE, "cg_step_series: graph launch failed");
      break;
    }
    launched += K;
  }
  memcpy(hs.data(), pinned, sizeof(IterState) * n);
  if (exec && !cached) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (rc) return rc;
  for (int k = 0; k < n; ++k) {
    const StepRef& r = refs[k];
    cg_series_out& o = out[r.series];
    if (r.slot < 0) {
      const int f = -1 - r.slot;
      if (o.frame_iters) o.frame_iters[f] = hs[k].iter;
      if (o.frame_xi) o.frame_xi[f] = hs[k].xi;
      continue;
    }
    if (o.iters) o.iters[r.slot] = hs[k].iter;
    if (o.status) o.status[r.slot] = hs[k].status;
    if (o.flags) o.flags[r.slot] = hs[k].flags;
    if (o.eps) o.eps[r.slot] = hs[k].eps;
    if (o.xi) o.xi[r.slot] = hs[k].xi;
    if (o.warm_step) o.warm_step[r.slot] = hs[k].ws_alpha;
  }
  (void)desc;
  return CG_OK;
}

// One cartogram of a series in the order its chain runs: a time step, or
// (value-interpolated transitions) a frame between two steps.
struct Link {
  StepRef ref;
  float* xy;             // output positions
  float* extra;          // output tracer points or null
  const float* values;   // [R] device
  double bg_mass;        // eq.(4) background mass or -1
  int prev;              // chain predecessor (cumulative start) or -1
};

Spec spec_for(const cg_series_desc& d, const std::vector<Link>& ch, int e, bool cumulative) {
  Spec s;
  const Link& L = ch[e];
  const bool chained = cumulative && L.prev >= 0;
  s.map = d.map;
  s.N = d.N;
  s.xy = (float2*)L.xy;
  s.src_xy = chained ? (const float2*)ch[L.prev].xy : (const float2*)d.xy0;
  if (L.extra) {
    s.extra = (float2*)L.extra;
    s.n_extra = d.n_extra;
    s.src_extra = chained ? (const float2*)ch[L.prev].extra : (const float2*)d.extra;
  }
  s.values = L.values;
  s.bg_mass = L.bg_mass;
  s.shape = d.shape;
  s.tol = d.tol;
  s.area_source = d.area_source;
  s.patience = d.patience;
  s.max_iters = d.max_iters;
  s.fixed_iters = d.fixed_iters;
  if (d.init_field && (!cumulative || e == 0)) {
    s.init_field = d.init_field;
    s.init_G = d.init_G;
  }
  return s;
}

bool area_mode(const cg_series_desc& d) { return d.area_min != 0.f || d.area_max != 0.f; }
bool value_frames(const cg_series_desc& d) { return d.frames >= 2 && d.frame_mode == CG_FRAMES_VALUES; }

// The chain of cartograms of series d: its steps, with the value frames
// between them when asked for (their values interpolated on the host into
// `vbuf`, rows in chain order), and each one's background mass.
int chain_for(cg_ctx* c, const cg_series_desc& d, const cg_series_out& o, int series, float* vbuf,
              hipStream_t st, std::vector<Link>& ch) {
  const int T = d.n_steps, R = d.map->R, K = d.frames;
  const bool vf = value_frames(d);
  const int64_t n = d.map->n_vert;
  std::vector<float> hv;
  std::vector<double> tot;
  if (vf || area_mode(d)) {
    hv.resize((size_t)T * R);
    HIP_OK(c, hipMemcpyAsync(hv.data(), d.values, sizeof(float) * hv.size(), hipMemcpyDeviceToHost, st));
    HIP_OK(c, hipStreamSynchronize(st));
  }
  // chain order: step 0, (frames of transition 0 -> 1), step 1, ...
  std::vector<float> ev;   // expanded values of the value frames, chain order
  ch.clear();
  for (int t = 0; t < T; ++t) {
    if (vf && t > 0)
      for (int k = 1; k < K; ++k) {
        const int f = (t - 1) * (K - 1) + (k - 1);
        Link L{{series, -1 - f}, o.frames + (size_t)f * n * 2, nullptr, nullptr, -1.0, (int)ch.size() - 1};
        const double a = (double)k / K;
        for (int v = 0; v < R; ++v)
          ev.push_back((float)((1.0 - a) * hv[(size_t)(t - 1) * R + v] + a * hv[(size_t)t * R + v]));
        L.values = vbuf + (ev.size() / R - 1) * R;
        ch.push_back(L);
      }
    Link L{{series, t}, o.xy + (size_t)t * n * 2,
           (d.extra && d.n_extra > 0 && o.extra_xy) ? o.extra_xy + (size_t)t * d.n_extra * 2 : nullptr,
           d.values + (size_t)t * R, -1.0, (int)ch.size() - 1};
    ch.push_back(L);
  }
  if (!ev.empty()) HIP_OK(c, hipMemcpyAsync(vbuf, ev.data(), sizeof(float) * ev.size(), hipMemcpyHostToDevice, st));
  if (area_mode(d)) {
    // eq.(4): map totals of the steps, their extremes over mass_t0..mass_t1
    std::vector<double> M(T, 0.0);
    for (int t = 0; t < T; ++t)
      for (int v = 0; v < R; ++v) M[t] += (double)hv[(size_t)t * R + v];
    const int t0 = d.mass_t1 >= d.mass_t0 ? d.mass_t0 : 0, t1 = d.mass_t1 >= d.mass_t0 ? d.mass_t1 : T - 1;
    double lo = M[t0], hi = M[t0];
    for (int t = t0; t <= t1; ++t) {
      lo = std::min(lo, M[t]);
      hi = std::max(hi, M[t]);
    }
    size_t fr = 0;
    for (Link& L : ch) {
      double Mi = 0.0;
      if (L.ref.slot >= 0) {
        Mi = M[L.ref.slot];
      } else {
        for (int v = 0; v < R; ++v) Mi += (double)ev[fr * R + v];
        ++fr;
      }
      const double w = hi == lo ? 1.0 : std::min(1.0, std::max(0.0, (Mi - lo) / (hi - lo)));
      const double A = (1.0 - w) * d.area_min + w * d.area_max;
      L.bg_mass = Mi * (1.0 - A) / A;
    }
  }
  if (!ev.empty()) HIP_OK(c, hipStreamSynchronize(st));   // ev is read by the copy above
  return CG_OK;
}

}  // namespace

extern "C" int cg_step_series(cg_ctx* c, const cg_series_desc* desc, int n_series, cg_series_out* out,
                              int32_t graph_iters, void* stream) {
  if (!c) return CG_EINVAL;
  if (!desc || !out || n_series < 0) return fail(c, CG_EINVAL, "cg_step_series: bad arguments");
  size_t vframes = 0;
  for (int i = 0; i < n_series; ++i) {
    const cg_series_desc& d = desc[i];
    if (!d.map || !d.xy0 || !d.values || !out[i].xy) return fail(c, CG_EINVAL, "cg_step_series: null map/xy0/values/out.xy");
    if (!pow2_ok(d.N)) return fail(c, CG_EINVAL, "cg_step_series: N must be a power of two in [16, 8192]");
    if (d.n_steps < 1 || d.map->R < 1) return fail(c, CG_EINVAL, "cg_step_series: need n_steps >= 1 and R >= 1");
    if (d.mode != CG_DIRECT && d.mode != CG_CUMULATIVE) return fail(c, CG_EINVAL, "cg_step_series: bad mode");
    if (d.precision < CG_F32 || d.precision > CG_F64ACC) return fail(c, CG_EINVAL, "cg_step_series: bad precision");
    if (d.area_source != CG_AREA_PIXEL && d.area_source != CG_AREA_POLYGON) return fail(c, CG_EINVAL, "cg_step_series: bad area source");
    if (!(d.tol > 0) || d.patience < 0 || d.max_iters < 0 || d.fixed_iters < 0 || !(d.shape >= 0))
      return fail(c, CG_EINVAL, "cg_step_series: bad stopping parameters");
    if (d.frames >= 2 && !out[i].frames) return fail(c, CG_EINVAL, "cg_step_series: frames requested without a buffer");
    if (d.init_field && d.init_G < 1) return fail(c, CG_EINVAL, "cg_step_series: init_field needs init_G >= 1");
    if ((int64_t)d.map->n_vert + d.n_extra > INT32_MAX) return fail(c, CG_EINVAL, "cg_step_series: too many points");
    if (d.frame_mode != CG_FRAMES_POSITIONS && d.frame_mode != CG_FRAMES_VALUES)
      return fail(c, CG_EINVAL, "cg_step_series: bad frame mode");
    if (value_frames(d) && d.extra && d.n_extra > 0)
      return fail(c, CG_EUNSUPPORTED, "cg_step_series: value-interpolated frames with tracer points");
    if (area_mode(d) && !(d.area_min > 0.f && d.area_min <= d.area_max && d.area_max < 1.f))
      return fail(c, CG_EINVAL, "cg_step_series: need 0 < area_min <= area_max < 1");
    if (area_mode(d) && d.mass_t1 >= d.mass_t0 && (d.mass_t0 < 0 || d.mass_t1 >= d.n_steps))
      return fail(c, CG_EINVAL, "cg_step_series: mass_t0..mass_t1 outside the steps");
    if (value_frames(d)) vframes += (size_t)(d.n_steps - 1) * (d.frames - 1) * d.map->R;
  }
  hipSetDevice(c->device);
  // order after the caller's stream, then run on the private (capturable) stream
  hipStream_t caller = pick_stream(c, stream);
  hipStream_t st = c->stream;
  {
    hipEvent_t ev;
    HIP_OK(c, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIP_OK(c, hipEventRecord(ev, caller));
    HIP_OK(c, hipStreamWaitEvent(st, ev, 0));
    HIP_OK(c, hipEventDestroy(ev));
  }
  c->last = st;
  // value rows of the interpolated frames of every series
  char* vb = nullptr;
  if (vframes) {
    int rc = get_buf(c, "series:frame_values", sizeof(float) * vframes, st, &vb);
    if (rc) return rc;
  }
  std::vector<std::vector<Link>> chains(n_series);
  {
    size_t at = 0;
    for (int i = 0; i < n_series; ++i) {
      int rc = chain_for(c, desc[i], out[i], i, (float*)vb + at, st, chains[i]);
      if (rc) return rc;
      if (value_frames(desc[i])) at += (size_t)(desc[i].n_steps - 1) * (desc[i].frames - 1) * desc[i].map->R;
    }
  }
  for (int prec = CG_F32; prec <= CG_F64ACC; ++prec) {
    // direct cartograms of every series with this precision: one batch
    std::vector<Spec> specs;
    std::vector<StepRef> refs;
    size_t max_e = 0;
    for (int i = 0; i < n_series; ++i) {
      if (desc[i].precision != prec) continue;
      if (desc[i].mode == CG_DIRECT) {
        for (size_t e = 0; e < chains[i].size(); ++e) {
          specs.push_back(spec_for(desc[i], chains[i], (int)e, false));
          refs.push_back(chains[i][e].ref);
        }
      } else {
        max_e = std::max(max_e, chains[i].size());
      }
    }
    int rc = run_batch(c, specs, refs, desc, out, prec, graph_iters, st);
    if (rc) return rc;
    // cumulative series: link e of all of them together, in chain order
    for (size_t e = 0; e < max_e; ++e) {
      specs.clear();
      refs.clear();
      for (int i = 0; i < n_series; ++i) {
        if (desc[i].precision != prec || desc[i].mode != CG_CUMULATIVE || e >= chains[i].size()) continue;
        specs.push_back(spec_for(desc[i], chains[i], (int)e, true));
        refs.push_back(chains[i][e].ref);
      }
      rc = run_batch(c, specs, refs, desc, out, prec, graph_iters, st);
      if (rc) return rc;
    }
  }
  for (int i = 0; i < n_series; ++i) {
    const cg_series_desc& d = desc[i];
    if (d.frames < 2 || value_frames(d)) continue;
    const int64_t n = d.map->n_vert;
    for (int t = 1; t < d.n_steps; ++t)
      cgk::launch_frames(out[i].xy + (size_t)(t - 1) * n * 2, out[i].xy + (size_t)t * n * 2,
                         out[i].frames + (size_t)(t - 1) * (d.frames - 1) * n * 2, n, d.frames, st);
  }
  HIP_OK(c, hipStreamSynchronize(st));
  return check_launch(c);
}
