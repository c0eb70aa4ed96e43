// Host-side state shared by the C ABI translation units of libcg.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "cg.h"
#include "cg_dev.h"

namespace cgh {

struct DevBuf {
  char* p = nullptr;
  size_t n = 0;
};

constexpr size_t kAlign = 256;

inline size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

}  // namespace cgh

struct cg_map {
  int device = 0;            // HIP device holding the map (the map may outlive its context)
  int32_t n_vert = 0, R = 0, n_rings = 0, n_edges = 0;
  int4* d_edges = nullptr;
  int32_t* d_reg_pair_off = nullptr;   // [R+1] region -> its ring edges
  int2* d_reg_pairs = nullptr;         // ring edges (a, b) grouped by region
};

// Launch parameters of a captured iteration graph (compared bytewise).
struct GraphKey {
  cgk::Batch B;
  int32_t prec, tw, th, il, fuse, K, ept, pad;
  int64_t blocks[7];
  hipStream_t stream;
};
struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
};

struct cg_ctx {
  int device = 0;
  hipStream_t stream = nullptr;  // private stream of the series driver (graph capture)
  hipStream_t last = nullptr;
  bool last_set = false;
  std::string err;
  std::map<std::string, cgh::DevBuf> bufs;
  char* pinned = nullptr;
  size_t pinned_n = 0;
  hipEvent_t pinned_ev = nullptr;
  bool pinned_pending = false;
  std::map<std::tuple<int, int, int64_t>, std::pair<int, int>> tiles;  // (N, prec, batch px) -> shape
  // per-stage timing of series iterations
  int prof_stage = -1;
  int prof_every = 1;        // time one launch in every prof_every iterations
  std::vector<hipEvent_t> prof_ev;
  std::vector<char> prof_rec;   // the event pair of an iteration was recorded in this launch sequence
  int prof_k = 0;            // iterations recorded per graph replay
  double prof_ms = 0.0;
  int64_t prof_launches = 0;
  int64_t prof_failed = 0;
  hipStream_t prof_stream = nullptr;
  // series driver: instantiated iteration graphs, pinned state buffer
  std::vector<GraphEntry> graphs;
  void* st_pinned = nullptr;
  size_t st_pinned_n = 0;
};

namespace cgh {

inline int fail(cg_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_OK(ctx, expr)                                                               \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return cgh::fail(ctx, CG_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// The stream a call runs on: the caller's (NULL is the HIP null stream).
// Scratch buffers are shared between calls, so switching streams first
// drains the previous one.
inline hipStream_t pick_stream(cg_ctx* c, void* s) {
  hipStream_t st = (hipStream_t)s;
  if (c->last_set && c->last != st) (void)hipStreamSynchronize(c->last);
  c->last = st;
  c->last_set = true;
  return st;
}

// Grow-only named device buffers (stream-ordered reuse).
inline int get_buf(cg_ctx* c, const char* name, size_t bytes, hipStream_t st, char** out) {
  DevBuf& b = c->bufs[name];
  if (b.n < bytes) {
    if (b.p) {
      HIP_OK(c, hipStreamSynchronize(st));
      HIP_OK(c, hipFree(b.p));
      b.p = nullptr;
      b.n = 0;
    }
    size_t want = std::max(bytes, (size_t)4096);
    want = want + want / 4;
    HIP_OK(c, hipMalloc(&b.p, want));
    b.n = want;
  }
  *out = b.p;
  return CG_OK;
}

inline bool pow2_ok(int N) { return N >= 16 && N <= 8192 && (N & (N - 1)) == 0; }

}  // namespace cgh
