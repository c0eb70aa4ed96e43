/*
 * cg.h -- C ABI of the MI355X integral-image cartogram library (libcg.so).
 *
 * The library computes contiguous cartograms by the iterative
 * density-equalising transformation (DET) built on integral images:
 * every iteration rasterises the region polygons into a density texture
 * (value over current area, background density = shape parameter times
 * the mean density), computes the axis-aligned and 45-degree tilted
 * integral images, moves every vertex by the bilinearly interpolated
 * eight-anchor displacement and recomputes the region areas
 * (paper: Method, "Construction of Static Cartograms", Steps 0-7;
 * Background, eqs. (1)-(3)).
 *
 * Conventions shared by every call:
 *   - Texture side N is a power of two, 16 <= N <= 8192 (Background,
 *     remark after eq.(1)).  Pixel (p, q) covers [p, p+1] x [q, q+1] in
 *     pixel units, p = column (x), q = row (y); the y axis points down.
 *     Node (i, j), 0 <= i, j <= N, sits at (x, y) = (i/N, j/N).
 *   - Positions are float32 pairs (x, y) in the unit square, array
 *     [n][2].  Region ids are 1..R; id 0 is the background.
 *   - Every array argument is DEVICE memory unless its comment says
 *     host.  The library never frees caller memory.
 *   - `stream` is a hipStream_t (NULL = the HIP null stream).  All calls
 *     are asynchronous on `stream` unless stated otherwise.
 *   - Every call returns CG_OK or a negative CG_E* code; invalid
 *     arguments are rejected before anything is launched, and
 *     cg_last_error() then describes the problem.  One context per host
 *     thread; calls on one context must not run concurrently.
 */
#ifndef CG_H_
#define CG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CG_OK 0
#define CG_EINVAL (-1)
#define CG_ENOMEM (-2)
#define CG_EDEVICE (-3)
#define CG_EUNSUPPORTED (-4)

/* Accumulation precision of the integral images (tables stored as float
 * for F32/COMP/F64ACC, double for F64). */
#define CG_F32 0    /* float accumulation */
#define CG_COMP 1   /* compensated float (TwoSum) accumulation, float carries in double */
#define CG_F64 2    /* double accumulation and storage */
#define CG_F64ACC 3 /* double accumulation, float storage */

#define CG_DIRECT 0     /* every time step deforms the original map */
#define CG_CUMULATIVE 1 /* every time step starts from the previous cartogram */

#define CG_AREA_PIXEL 0   /* density = value / pixel count (Step 2) */
#define CG_AREA_POLYGON 1 /* density = value / shoelace area */

/* Per-step outcome of the stopping rule (Method, end of the static
 * construction): max area error below tol, no new minimum within
 * `patience` iterations, iteration cap, or an internal error. */
#define CG_STATUS_CONVERGED 0
#define CG_STATUS_STALLED 1
#define CG_STATUS_MAXITER 2
#define CG_STATUS_ERROR 3

/* Flags raised during a run (OR-ed). */
#define CG_FLAG_CONTESTED 1 /* a pixel centre was claimed by two regions: the map folded */
#define CG_FLAG_OVERFLOW 2  /* a crossing buffer overflowed: results invalid */
#define CG_FLAG_FALLBACK 4  /* a warm start was rejected and the plain start used */
#define CG_FLAG_BADVALUES 8 /* a value is negative, infinite or NaN, or all are 0: the step is not
                               iterated and ends with CG_STATUS_ERROR */

typedef struct cg_ctx cg_ctx;
typedef struct cg_map cg_map;

/* Context: owns scratch workspaces, the tile-shape table and a private
 * stream on which cg_step_series captures and replays its graphs (after
 * the caller's stream).  `device` is the HIP device ordinal. */
int cg_create(int device, cg_ctx** out);
int cg_destroy(cg_ctx* ctx);
/* Text of the last error on this context (never NULL; owned by ctx). */
const char* cg_last_error(const cg_ctx* ctx);
/* The context's stream (a hipStream_t). */
void* cg_stream(const cg_ctx* ctx);

/* Map topology (Method, Step 0: regions given as polygons with shared
 * boundaries).  Host arrays: rings in CSR form, ring_off [n_rings+1],
 * ring_idx [ring_off[n_rings]] vertex ids in 0..n_vertices-1 (each ring
 * listed once, not closed), ring_reg [n_rings] region id in 1..n_regions.
 * Rings must have positive signed area 0.5*sum(x_k y_{k+1} - x_{k+1} y_k)
 * (a region may own several rings; holes are not supported).  The call
 * builds the unique edge table (each edge with the regions on its two
 * sides, 0 outside the map) and uploads it.  CG_EINVAL when an edge is
 * used by more than two rings or indices are out of range.  Vertex
 * positions are not part of the map: they are caller-owned device
 * arrays.  Blocking (uploads finish before return). */
int cg_map_build(cg_ctx* ctx, int32_t n_vertices, int32_t n_regions, int32_t n_rings,
                 const int32_t* ring_off, const int32_t* ring_idx, const int32_t* ring_reg,
                 cg_map** out);
/* Frees the map's device buffers; the map may outlive the context that
 * built it (destroying it after cg_destroy is fine). */
int cg_map_destroy(cg_map* map);
int32_t cg_map_n_edges(const cg_map* map);

/* Step 2 (region area by pixel counting): label map of the map at
 * positions xy [n_vertices][2].  labels: uint16 [N][N], row = y, value =
 * region whose polygon contains the pixel centre under the exact rule:
 * coordinates snapped to X = rint(x*256N), a row is crossed by an edge
 * when exactly one endpoint has Y <= 256q+128, a centre on an edge
 * belongs to the region on its +x side; a centre claimed by several
 * regions (folded map) gets the highest claiming id.  counts: int64
 * [R+1] pixel counts o(v) (index 0 = background), or NULL.  contested:
 * int64 [1] number of contested pixels, or NULL. */
int cg_rasterize(cg_ctx* ctx, const cg_map* map, const float* xy, int N, uint16_t* labels,
                 int64_t* counts, int64_t* contested, void* stream);

/* Node integral images of one texture (Background, "Integral Images",
 * eq.(1)).  Element type: double for CG_F64, float otherwise.
 *   S  [(N+1)][pitch]: S[j][i] = integral of d over [0,i] x [0,j]
 *   T  [(N+1)][pitch]: integral of d over the top wedge of node (i,j),
 *                      { (x',y') : y' <= j - |x' - i| }
 *   HA [2N+1]: HA[s] = integral over x'+y' <= s
 *   HB [2N+1]: HB[r+N] = integral over y'-x' <= r
 * All eight integral images of a node are O(1) combinations of these
 * (alpha = S, beta = S(i,N)-S, delta = S(N,j)-S, gamma = C-S(i,N)-S(N,j)+S,
 *  alpha_t = T, beta_t = HA-T, delta_t = HB-T, gamma_t = C-HA-HB+T). */
typedef struct {
  int32_t N;
  int32_t precision;
  int64_t pitch; /* elements per node-table row, >= N+1 */
  void* S;
  void* T;
  void* HA;
  void* HB;
} cg_inim;

/* Sizes the caller allocates for cg_integral_image (any argument may be NULL). */
int cg_inim_size(int N, int precision, int64_t* pitch, size_t* table_bytes, size_t* marginal_bytes);

/* Step 4: integral images of the density texture.  Either labels (uint16
 * [N][N]) with lut (float [n_lut] density per label; every label must be
 * < n_lut), or, when `density` is not NULL, a dense float [N][N]
 * texture (labels/lut ignored); labels / density must be 16-byte
 * aligned.  out->S, T, HA, HB are caller buffers of cg_inim_size's sizes;
 * out->N/precision/pitch are filled in. */
int cg_integral_image(cg_ctx* ctx, int N, const uint16_t* labels, const float* lut, int32_t n_lut,
                      const float* density, int precision, cg_inim* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * same operation as cg_integral_image, same arguments and results (bit
 * for bit), but every temporary (tile aggregates, carries, the launch
 * descriptors) lives in a static device buffer of 24 MiB that the library
 * holds on each GPU until the process ends; the call itself allocates
 * nothing and writes its descriptors with a kernel, not a host copy.  The
 * buffer holds any N <= 2048 (at most 19 MB of scratch with the smallest
 * tiles) and larger N with large enough tiles; a call whose scratch does
 * not fit returns CG_EINVAL with the sizes in cg_last_error().  Every
 * call on one GPU shares that buffer: calls that overlap on one GPU (on
 * different streams, or from different contexts or threads without
 * ordering) race and give undefined results.  CG_EDEVICE if the buffer's
 * address could not be obtained when the context was created. */
int cg_integral_image_noalloc(cg_ctx* ctx, int N, const uint16_t* labels, const float* lut, int32_t n_lut,
                              const float* density, int precision, cg_inim* out, void* stream);

/* Steps 5-6: move n_points points by the DET displacement
 * D = t(.; d) - t(.; d0) of eqs.(2)-(3), evaluated at the four corner
 * nodes of each point from `inim` and interpolated bilinearly, then
 * clamped to [0,1]^2.  xy_out may alias xy_in. */
int cg_map_points(cg_ctx* ctx, const cg_inim* inim, const float* xy_in, float* xy_out,
                  int64_t n_points, void* stream);

/* Region areas by the shoelace formula and the cartographic errors
 * (Background, "Quality Measures").  areas: double [R+1]; areas[v] =
 * sum of v's ring areas, areas[0] = 1 - sum (the background).  When
 * values (float [R]) and eps_xi (double [2]) are given, eps_xi receives
 * the mean and max of |A-w|/max(A,w), w(v) = s(v) * sum_u A(u) / sum_u s(u).
 * Deterministic: fixed-order FP64 reductions, no atomics. */
int cg_region_areas(cg_ctx* ctx, const cg_map* map, const float* xy, const float* values,
                    double* areas, double* eps_xi, void* stream);

/* Geographic-distortion measures of a cartogram against its original map
 * (Background, "Quality Measures"), from the label maps of the map and of
 * the cartogram at the same texture size N (cg_rasterize, uint16 [N][N],
 * 16-byte aligned) and the two position sets (float [n_vertices][2]):
 *   adjacency: int64 [3]  |E_m|, |E_c|, |E_c n E_m|, where two regions are
 *              neighbours when pixels of both share a pixel side (the
 *              background, label 0, is no region);
 *   overlap:   int64 [R+1] for every region v the largest |P_m n (P_c + t)|
 *              over all translations t by whole pixels, P_m and P_c the
 *              pixel sets of v in the two label maps ([0] = 0);
 *   pixels:    int64 [2][R+1] |P_m|, then |P_c|, per region;
 *   shape:     double [R+1] shape distortion of v: the symmetric
 *              difference of P_m and the best-translated P_c over their
 *              union, (|P_m| + |P_c| - 2 overlap) / (|P_m| + |P_c| - overlap)
 *              (0 when both sets are empty, 1 when only one is; [0] = 0);
 *   bary:      double [2][R+1][2] region barycentres (area centroids of
 *              all of a region's rings) in the map, then in the cartogram,
 *              or NULL;
 *   summary:   double [4] topology distortion tau = 1 - |E_c n E_m| /
 *              |E_c u E_m| (0 when both are empty), the mean and the max of
 *              the shape distortion over regions 1..R, and the relative
 *              position error R = sum over ordered pairs u != v of
 *              |angle(b_c(u,v), b_m(u,v))| / (pi |V| (|V| - 1)), b(u,v) the
 *              vector from u's barycentre to v's.
 * Integer results are exact; the doubles are FP64 sums in a fixed order.
 * 1 <= R <= 4095 (CG_EUNSUPPORTED otherwise); CG_EINVAL when a label map
 * holds a label above R.  Blocking: returns when the results are written. */
typedef struct {
  int64_t* adjacency;
  int64_t* overlap;
  int64_t* pixels;
  double* shape;
  double* bary;
  double* summary;
} cg_quality_out;

int cg_quality(cg_ctx* ctx, const cg_map* map, int N, const uint16_t* labels_map, const uint16_t* labels_cart,
               const float* xy_map, const float* xy_cart, cg_quality_out* out, void* stream);

/* Whole cartograms for time series (Method, Steps 0-7 iterated with the
 * stopping rule; "Coherence of Dynamic Cartograms" for the direct and
 * cumulative strategies).  One descriptor per series; every series has
 * n_steps value vectors.  Direct steps of all series run together in one
 * batch; cumulative steps run in order, all series together. */
typedef struct {
  const cg_map* map;
  const float* xy0;     /* [n_vertices][2] original map */
  int32_t N;            /* texture side */
  int32_t n_steps;      /* T >= 1 */
  const float* values;  /* [T][R] */
  int32_t mode;         /* CG_DIRECT / CG_CUMULATIVE */
  float shape;          /* b: background density = b * d0 (1 = the paper's default) */
  int32_t area_source;  /* CG_AREA_PIXEL (default) / CG_AREA_POLYGON */
  float tol;            /* stop when max area error < tol (0.01) */
  int32_t patience;     /* stop when no new minimum for this many iterations (32) */
  int32_t max_iters;    /* iteration cap (512) */
  int32_t fixed_iters;  /* > 0: run exactly this many iterations, no stopping rule */
  int32_t precision;    /* CG_F32 / CG_COMP / CG_F64 */
  int32_t frames;       /* K >= 2: K-1 interpolated frames per transition; 0: none */
  const float* extra;   /* [n_extra][2] tracer points moved along, or NULL */
  int64_t n_extra;
  const float* init_field; /* warm start: float [G][G][2] displacement (dx, dy) at the pixel centres
                              ((i + 1/2)/G, (j + 1/2)/G) of a G x G grid, or NULL; see below */
  int32_t init_G;
  /* Background mass from the map total (Method, "Interactive Steering",
   * eq.(4)): with 0 < area_min <= area_max < 1, step t's background holds
   * M_b(t) = M_i(t) (1 - A_i(t)) / A_i(t), M_i(t) the sum of its values,
   * A_i(t) = (1 - w) area_min + w area_max, w = (M_i(t) - M_min) /
   * (M_max - M_min) clamped to [0, 1] (1 when M_max = M_min), the extremes
   * taken over steps mass_t0..mass_t1 (all steps when mass_t1 < mass_t0);
   * the background density is shape * M_b / (background pixels).
   * area_min = area_max = 0: off (background density shape * d0). */
  float area_min;
  float area_max;
  int32_t mass_t0;
  int32_t mass_t1;
  int32_t frame_mode;   /* CG_FRAMES_POSITIONS / CG_FRAMES_VALUES, used when frames >= 2 */
} cg_series_desc;

/* In-between frames of a transition t-1 -> t (k = 1..K-1): */
#define CG_FRAMES_POSITIONS 0 /* linear interpolation of the two steps' vertex positions */
#define CG_FRAMES_VALUES 1    /* a cartogram of the values (1-k/K) s_{t-1} + (k/K) s_t, from the original
                                 map (direct) or from the previous frame (cumulative: the chain runs step,
                                 frames, next step); not with tracer points */

typedef struct {
  float* xy;        /* device [T][n_vertices][2] */
  float* extra_xy;  /* device [T][n_extra][2] or NULL */
  float* frames;    /* device [T-1][K-1][n_vertices][2] or NULL */
  int32_t* iters;   /* HOST [T] iterations done */
  int32_t* status;  /* HOST [T] CG_STATUS_* */
  int32_t* flags;   /* HOST [T] CG_FLAG_*, over the run's rasterisations (in launches of up to 2M
                       edges these include one of the final positions, made before the stopping
                       rule ends the run; a flag from that one does not change the status) */
  double* eps;      /* HOST [T] final mean area error */
  double* xi;       /* HOST [T] final max area error */
  float* warm_step; /* HOST [T] warm-start step taken (0: plain start), or NULL */
  int32_t* frame_iters; /* HOST [T-1][K-1] iterations of each CG_FRAMES_VALUES frame, or NULL */
  double* frame_xi;     /* HOST [T-1][K-1] final max area error of each such frame, or NULL */
} cg_series_out;

/* Runs every series in desc[0..n_series); out[k] receives series k.
 * Warm start: with init_field, the starting positions (of the first step
 * in cumulative mode, of every step in direct mode) are moved by alpha
 * times the field (bilinear between the grid's pixel centres, constant
 * beyond the outermost ones, clamped to the unit square) for the trial
 * steps alpha = 1, 3/4, 1/2, 1/4.  Each moved map is rasterised and its max
 * area error computed; a step whose map folded (a pixel centre claimed by
 * two regions) is rejected.  The run starts from the non-folding step
 * with the lowest error if that error is below the plain start's, else
 * from the plain start, with CG_FLAG_FALLBACK set for that step.  The
 * plain iteration then runs as usual.
 * Blocking: starts after the work already queued on `stream` and
 * returns when all steps have stopped.  Iterations are issued
 * as captured HIP graphs of `graph_iters` iterations (0: default 8; a
 * negative value launches -graph_iters iterations eagerly, without a graph),
 * with a convergence poll between replays. */
int cg_step_series(cg_ctx* ctx, const cg_series_desc* desc, int n_series, cg_series_out* out,
                   int32_t graph_iters, void* stream);

/* Integral-image tile shape (TW columns x TH rows per tile) used for a
 * launch whose largest texture side is N and whose textures hold
 * batch_pixels pixels in total.  The table is per context: cg_autotune
 * times every supported shape on a synthetic batch of `batch` label maps
 * of side N (blocking) and records the fastest, reading and appending
 * "arch N precision batch_pixels tw th" lines in cache_path when it is
 * not NULL; cg_set_tile_shape records a shape directly; other launches
 * use the nearest recorded batch size for (N, precision), else a
 * default.  Supported shapes: 64x16, 128x16, 128x32, 256x32, 256x64. */
int cg_tile_shape(const cg_ctx* ctx, int N, int precision, int64_t batch_pixels, int32_t* tw, int32_t* th);
int cg_set_tile_shape(cg_ctx* ctx, int N, int precision, int64_t batch_pixels, int32_t tw, int32_t th);
int cg_autotune(cg_ctx* ctx, int N, int precision, int32_t batch, const char* cache_path);

/* Timing of one pipeline stage inside cg_step_series (profiling aid).
 * cg_profile_stage selects the stage ("raster_emit", "raster_fill",
 * "density", "sat_reduce", "sat_carry1", "sat_carry2", "sat_final",
 * "map_points", "areas", "err"; NULL or "" to stop) and resets the
 * totals.  "density" and "sat_carry1" are separate launches only for
 * batches where folding them into the integral-image passes does not pay
 * (large LUT work, tables too large for LDS); otherwise they report no
 * launches.  While selected, the launch of that kernel
 * in one of every `every` iterations is bracketed by HIP events recorded
 * on the launch stream, and cg_profile_read returns the summed
 * milliseconds and the number of launches timed so far.  Events are only
 * recorded when the series runs eagerly (graph_iters < 0): HIP does not
 * time event records captured into graphs. */
int cg_profile_stage(cg_ctx* ctx, const char* stage, int32_t every);
int cg_profile_read(cg_ctx* ctx, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* CG_H_ */
