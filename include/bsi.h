/*
 * bsi.h -- B-spline interpolation of periodic spectral fields on MI355X (gfx950).
 *
 * The method is the one of van Hinsberg, ten Thije Boonkkamp, Toschi and
 * Clercx, "On the efficiency and accuracy of interpolation methods for
 * spectral codes" (SIAM J. Sci. Comput. 2012):
 *
 *   prefilter  (Section 7)  multiply every Fourier mode of the field by
 *              c(kx) c(ky) c(kz) and apply one inverse 3D real FFT, giving the
 *              B-spline coefficient grid u_B;
 *   evaluation (Sections 2, 3, 5; Table 1)  for every particle, pick the N^3
 *              nearest grid points, form the 1D weights M tbar and M^(1) tbar
 *              per axis, and contract them with the local coefficients to get
 *              u and all first derivatives.
 *
 * Everything is a plain C ABI: device or host pointers and sizes, no
 * framework types.  All functions return a bsi_status and never throw.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Spectrum   uhat[c][k0][k1][k2], c < ncomp, k0 < n0, k1 < n1, k2 <= n2/2:
 *            Fourier-series coefficients of a real field on the box
 *            [0,L0)x[0,L1)x[0,L2), u(x) = sum_k uhat_k exp(2 pi i sum_d k_d x_d / L_d),
 *            in the real-FFT half-spectrum layout (index k >= n/2+1 of axes
 *            0 and 1 is the negative wave number k - n).  complex128 or
 *            complex64, interleaved (re, im).  As for any inverse real FFT,
 *            only the real parts of the k2 = 0 and k2 = n2/2 entries of the
 *            transformed lines are used; a Hermitian spectrum is unaffected.
 * Positions  pos[p][d], FP64, any finite value (wrapped periodically).
 *            A particle with a non-finite coordinate gets NaN outputs and is
 *            counted (bsi_field_stats).
 * Outputs    u[p][c] and grad[p][c][d] = d u_c / d x_d in physical units,
 *            FP64 for a BSI_F64 coefficient grid, FP32 otherwise.
 * Streams    every call is asynchronous on the given HIP stream (NULL = the
 *            context's stream).  Buffers passed in belong to the caller and
 *            must stay valid until the stream reaches the call's work.
 *            Faults surface at the next synchronising call as BSI_E_DEVICE.
 * Threads    a context and its fields are used from one host thread at a time;
 *            distinct contexts may be used concurrently.
 * Errors     on failure a thread-local message is available from
 *            bsi_last_error().
 */
#ifndef BSI_H
#define BSI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bsi_status {
    BSI_OK = 0,
    BSI_E_INVAL = 1,        /* bad argument (pointer, size, descriptor)              */
    BSI_E_NOMEM = 2,        /* device or host allocation failed / over budget        */
    BSI_E_UNSUPPORTED = 3,  /* valid but not implemented (e.g. odd order, n=5*k)     */
    BSI_E_DEVICE = 4,       /* HIP runtime error or device fault                     */
    BSI_E_BUSY = 5,         /* server queue full                                     */
    BSI_E_CANCELLED = 6     /* server request cancelled                              */
} bsi_status;

/* Storage type of the coefficient grid (and of spectra: F64 = complex128,
 * F32 = complex64).  BF16 is storage only: evaluation accumulates in FP32. */
typedef enum bsi_dtype { BSI_F64 = 0, BSI_F32 = 1, BSI_BF16 = 2 } bsi_dtype;

/* Choice of c(k), Section 7.  L2OPT: c = F[B](kappa) / sum_i F[B](kappa+i)^2,
 * the L2-optimal constants the paper proposes.  INTERP: c = 1 / F_D[B_D](k),
 * the straightforward inverse of the sampled spline (exact at grid nodes).
 * NONE: c = 1, the grid holds the field's own values (the data of the
 * Lagrange, linear and Hermite comparison methods, Section 8). */
typedef enum bsi_prefilter {
    BSI_PREFILTER_L2OPT = 0, BSI_PREFILTER_INTERP = 1, BSI_PREFILTER_NONE = 2
} bsi_prefilter;

/* Interpolation method (Section 2: u~ = f[u]^T M xbar on a cell; Section 8
 * compares these).  BSPLINE: M_(N) of Section 7 on the prefiltered coefficient
 * grid, orders 2 (linear), 4, 6.  LAGRANGE: the polynomial of degree N-1
 * through the N nearest grid values (Section 5 stencil), orders 2 (linear), 4,
 * 6; prefilter must be NONE.  HERMITE: cubic Hermite (order 4, Section 2 matrix)
 * on the value and the derivatives of the field at the 2^3 corners of the cell
 * (Section 3 tensor B; the 8 derivative fields per component come from 8
 * inverse FFTs, Table 2); prefilter must be NONE. */
typedef enum bsi_basis { BSI_BASIS_BSPLINE = 0, BSI_BASIS_LAGRANGE = 1, BSI_BASIS_HERMITE = 2 } bsi_basis;

typedef struct bsi_field_desc {
    int32_t n[3];        /* grid points per axis, each 2^a 3^b, max(2*order, 8) <= n <= 1024 */
    int32_t ncomp;       /* 1 (scalar) or 3 (vector field, Section 3 last paragraph)   */
    int32_t order;       /* N (degree N-1): 2, 4 or 6; 4 for BSI_BASIS_HERMITE          */
    int32_t coef;        /* bsi_dtype of the coefficient grid                          */
    int32_t prefilter;   /* bsi_prefilter                                              */
    int32_t basis;       /* bsi_basis (0 = B-spline, the paper's method)               */
    double length[3];    /* box lengths L_d; 0 means 2*pi                              */
} bsi_field_desc;

/* Evaluation tuning knobs (results never depend on them). */
typedef struct bsi_eval_config {
    int32_t sort_tile;   /* cells per Morton tile edge for particle binning; 0 = no binning */
    int32_t block;       /* threads per workgroup of the gather kernel (64..1024, multiple of 64) */
    int32_t xcd_remap;   /* 1 = map consecutive binned particle blocks onto one XCD (tiled
                            gather: each XCD's workgroups start on their own range of tiles)   */
    int32_t variant;     /* 0 = LDS-tiled gather when sort_tile > 0 and the tile fits (sizes 4, 6,
                            8, 12, 16 whose block is at most 64 KB of LDS and whose origin is
                            16-byte aligned); otherwise, and for 1, one thread per particle
                            reading the grid directly */
    int32_t tiles_per_group; /* read by no kernel now (the tiled gather takes work items, the
                                batch's tile kernels one tile at a time); kept so that tuning
                                records and callers' structs keep their layout; any value */
    int32_t tile_block;      /* threads per workgroup of the tiled gather with 8^3-cell tiles:
                                0 or 64 = one wavefront per tile, 256 = four wavefronts share a
                                tile (dense tiles); other tile sizes have a fixed block */
    int32_t item_rounds;     /* tiled gather: a crowded tile is cut into work items of at most
                                item_rounds x (threads per workgroup) particles, shared out
                                among the workgroups (0 = 4) */
    int32_t reserved[1];     /* must be 0 */
} bsi_eval_config;

typedef struct bsi_ctx bsi_ctx;
typedef struct bsi_field bsi_field;
typedef struct bsi_server bsi_server;
typedef struct bsi_eval_plan bsi_eval_plan;

/* ---- context ------------------------------------------------------------ */

/* Create a context on HIP device `device`.  `hip_stream` (a hipStream_t or
 * NULL) becomes the context's default stream; NULL means the device's null
 * stream.  The context owns FFT twiddle tables, prefilter tables and scratch. */
bsi_status bsi_ctx_create(int device, void* hip_stream, bsi_ctx** out);
/* Destroy a context.  All its fields must have been destroyed. */
void bsi_ctx_destroy(bsi_ctx* ctx);
/* Message of the last failure on this host thread ("" if none). */
const char* bsi_last_error(void);
/* Library version string. */
const char* bsi_version(void);

/* ---- fields ------------------------------------------------------------- */

/* Validate `desc` and allocate the field's coefficient grid on the device.
 * BSI_E_INVAL for bad sizes/ncomp/dtype/lengths/basis or a basis whose
 * prefilter must be NONE, BSI_E_UNSUPPORTED for another order or an n that is
 * not 2^a 3^b, BSI_E_NOMEM if the grid does not fit.  The grid is
 * (n0+N-1)(n1+N-1)(n2+N-1)*ncomp elements: the periodic grid plus N-1 ghost
 * planes per axis, components interleaved.  A Hermite field stores its 8
 * derivative fields interleaved on a doubled grid: entry 2g+a of each axis
 * holds the a-th (0 or 1) derivative along that axis, in grid units (spacing
 * one), at grid point g; (2n0+2)(2n1+2)(2n2+2)*ncomp elements with 2 ghost
 * entries per axis, 8 times the memory of one grid (Table 2's (N/2)^3 fields). */
bsi_status bsi_field_create(bsi_ctx* ctx, const bsi_field_desc* desc, bsi_field** out);
void bsi_field_destroy(bsi_field* field);
/* Device bytes held by the field (grid and counters). */
size_t bsi_field_bytes(const bsi_field* field);

/* Prefilter (Section 7): uhat_dev is the device spectrum described above,
 * complex128 if uhat_prec == BSI_F64 or complex64 if BSI_F32.  The symbol
 * product is formed and applied in FP64, then one inverse 3D real FFT runs in
 * FP64 (BSI_F64 grid) or FP32 (BSI_F32 / BSI_BF16 grid; BF16 is a
 * round-to-nearest-even cast of the FP32 result).  uhat is only read.  With
 * prefilter NONE the grid is the field's values; for a Hermite field the call
 * runs 8 inverse FFTs, one per derivative field, the spectrum multiplied by
 * prod_d (i 2 pi k'_d / n_d)^(a_d) in FP64 (zero at the Nyquist index of a
 * differentiated axis). */
bsi_status bsi_field_set_spectrum(bsi_field* field, const void* uhat_dev,
                                  int32_t uhat_prec, void* hip_stream);

/* Load the coefficient grid directly: grid_dev is FP64 [ncomp][n0][n1][n2]
 * (component-major, no ghosts; [ncomp][2n0][2n1][2n2] in the interleaved
 * layout above for a Hermite field), cast to the field's storage type.  Lets
 * the evaluation be checked on a grid computed elsewhere. */
bsi_status bsi_field_set_coefficients(bsi_field* field, const double* grid_dev,
                                      void* hip_stream);
/* Read the coefficient grid back as FP64 [ncomp][n0][n1][n2] (widened from
 * the storage type; the interleaved [ncomp][2n0][2n1][2n2] for Hermite). */
bsi_status bsi_field_get_coefficients(const bsi_field* field, double* grid_dev,
                                      void* hip_stream);

/* ---- evaluation (Sections 2, 3, 5; Table 1) ----------------------------- */

/* Interpolate u (and grad u if grad_dev != NULL) at P particle positions
 * with the field's method (B-spline, Lagrange, linear or Hermite: same stencil
 * rule and contraction, Sections 2, 3, 5; Hermite fields are evaluated one
 * lane per binned particle, never from LDS tiles).
 * pos_dev: FP64 [P][3]; u_dev: [P][ncomp]; grad_dev: [P][ncomp][3]; device
 * pointers, 8-byte aligned.  0 <= P < 2^31; P == 0 does nothing. */
bsi_status bsi_eval(bsi_field* field, const double* pos_dev, int64_t P,
                    void* u_dev, void* grad_dev, void* hip_stream);
/* Same with explicit tuning knobs (NULL = the context's tuned configuration
 * for this field and particle count, see bsi_ctx_lookup_config). */
bsi_status bsi_eval_ex(bsi_field* field, const double* pos_dev, int64_t P,
                       void* u_dev, void* grad_dev, const bsi_eval_config* cfg,
                       void* hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as bsi_eval_ex, bitwise, with the same arguments, but the
 * binning workspace is a fixed device array of 128 MiB per GPU, part of the
 * library's code object (each GPU the library runs on holds it until the
 * process ends; its address is looked up once per device by bsi_ctx_create).
 * The call allocates nothing and creates no events (the context's stage
 * timing does not record it).  BSI_E_INVAL, with the bytes needed in
 * bsi_last_error(), when the call's workspace (about 70 bytes per particle
 * plus 8 per Morton tile of the field, for binned configurations) exceeds the
 * array; use fewer particles per call or bsi_eval_ex then.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (other streams or
 * host threads) race and must not be issued; consecutive calls on one stream
 * are ordered and safe.  Nothing in the array needs clearing between calls. */
bsi_status bsi_eval_static(bsi_field* field, const double* pos_dev, int64_t P,
                           void* u_dev, void* grad_dev, const bsi_eval_config* cfg,
                           void* hip_stream);

/* An evaluation in two halves (the same work and results as bsi_eval_ex, bitwise):
 * bsi_eval_plan_bin does everything that depends on the positions only (cell,
 * Morton binning, work items: Section 5's stencil rule), bsi_eval_plan_run the
 * gather and contraction from that binning and the field's grid as it is when
 * the run executes.  The binning can thus run on another stream while the
 * field's prefilter (bsi_field_set_spectrum) runs, and one binning serves
 * several runs (the field's grid may change in between).
 *
 * bsi_eval_plan_create: a plan for `field` and up to max_particles positions,
 * with its own device workspace (allocated here, freed by destroy) and the
 * configuration *cfg (NULL: the context's tuned one for max_particles).
 * bsi_eval_plan_bin: bins P <= max_particles positions pos_dev [P][3] FP64 on
 * the stream; pos_dev belongs to the caller and must stay unchanged until the
 * last run that uses this binning has completed.  BSI_E_INVAL if P exceeds the
 * plan's capacity.
 * bsi_eval_plan_run: u_dev [P][ncomp], grad_dev [P][ncomp][3] or NULL, as
 * bsi_eval; BSI_E_INVAL before the first bin.  The caller orders a run after
 * its bin (same stream, or an event) and after the field's prefilter; calls on
 * one plan that overlap race.
 * A plan must be destroyed before its field. */
bsi_status bsi_eval_plan_create(bsi_field* field, int64_t max_particles, const bsi_eval_config* cfg,
                                bsi_eval_plan** out);
bsi_status bsi_eval_plan_bin(bsi_eval_plan* plan, const double* pos_dev, int64_t P, void* hip_stream);
bsi_status bsi_eval_plan_run(bsi_eval_plan* plan, void* u_dev, void* grad_dev, void* hip_stream);
void bsi_eval_plan_destroy(bsi_eval_plan* plan);

/* (B-spline fields of orders 4 and 6; BSI_E_UNSUPPORTED for other fields.)
 * u, grad u and the second derivatives at P particles (Section 2: the l-th
 * derivative of the interpolant uses M^(l) = M D^l, here l = 2; Section 3 for
 * the tensor product).  u_dev [P][ncomp], grad_dev [P][ncomp][3] (NULL = not
 * computed), hess_dev [P][ncomp][6] with hess[p][c][m] = d2 u_c / dx_i dx_j for
 * (i, j) = (0,0), (0,1), (0,2), (1,1), (1,2), (2,2); physical units (each
 * derivative carries n/L of its axis).  Element type as for bsi_eval; same
 * validation, non-finite handling and asynchrony.  The particles are binned
 * with the context's evaluation workspace of the stream. */
bsi_status bsi_eval_hessian(bsi_field* field, const double* pos_dev, int64_t P, void* u_dev,
                            void* grad_dev, void* hess_dev, void* hip_stream);

/* Cell index and offset of each particle per axis, exactly as the evaluation
 * computes them (Section 5 stencil rule): s = x * (n/L) (one FP64 product),
 * f = floor(s), t = s - f, cell = f mod n in [0, n).  cell_dev: int32 [P][3],
 * t_dev: FP64 [P][3].  Non-finite coordinates give cell -1, t NaN. */
bsi_status bsi_debug_cells(bsi_field* field, const double* pos_dev, int64_t P,
                           int32_t* cell_dev, double* t_dev, void* hip_stream);

/* The binning of the evaluation path, for tests (not part of the method: a
 * locality device).  Buckets are Morton tiles of `tile` cells per edge (tile
 * >= 1 and >= ceil(max(n) / 256), else BSI_E_INVAL): bucket b < nbuckets - 1
 * holds the particles whose cell (bsi_debug_cells) lies in the tile with
 * coordinates (cell_d / tile) whose bits interleave into b, axis 0 highest of
 * each triple; the last bucket holds the particles without a cell.  Always sets
 * *nbuckets (> 0).  With hist_dev == NULL nothing else is done; otherwise
 * hist_dev and offs_dev (device uint32 [nbuckets]) receive each bucket's
 * particle count and first binned slot (the exclusive prefix sum of the
 * counts), perm_dev (device uint32 [P]) the particle index held by every binned
 * slot and pos_sorted_dev (device FP64 [P][3]) its position.  The order of the
 * particles inside a bucket is unspecified.  Uses the context's evaluation
 * workspace of the stream. */
bsi_status bsi_debug_bins(bsi_field* field, const double* pos_dev, int64_t P, int32_t tile,
                          uint32_t* hist_dev, uint32_t* offs_dev, uint32_t* perm_dev,
                          double* pos_sorted_dev, int64_t* nbuckets, void* hip_stream);

/* Number of non-finite positions seen by evaluations of this field so far
 * (synchronises the field's last stream). */
bsi_status bsi_field_stats(bsi_field* field, int64_t* nonfinite_positions);

/* ---- batching: many fields in one graph of a few launches ---------------- */

/* One evaluation inside a batch: the arguments of bsi_eval for one field. */
typedef struct bsi_eval_item {
    bsi_field* field;
    const double* pos;   /* device, FP64 [P][3]                        */
    int64_t P;           /* 0 <= P < 2^31; an item with P == 0 is skipped */
    void* u;             /* device, [P][ncomp]                         */
    void* grad;          /* device, [P][ncomp][3], or NULL (checked on items with P > 0) */
} bsi_eval_item;

typedef struct bsi_batch bsi_batch;

/* (Items must be B-spline fields of orders 4 and 6; BSI_E_UNSUPPORTED otherwise.)
 * Plan the evaluation of `count` items (1..65535) as one unit of work: every
 * item's particles are binned by the Morton tile of its own sort granularity
 * (one set of binning launches for all items), and per (order, components)
 * class present one persistent kernel walks the class's non-empty tiles of the
 * items gathered from LDS tiles (8^3 cells) and one kernel takes the class's
 * groups of 64 binned particles of the items gathered one lane per particle,
 * so that large and small items share the GPU without a launch per item.  cfgs (count
 * entries) gives each item's configuration, or NULL for the tuned ones
 * (bsi_ctx_lookup_config); a tiled configuration is run with 8^3-cell tiles
 * (one lane per particle if the class has no such tile).  Results are bitwise those of
 * bsi_eval_ex with the item's planned configuration (bsi_batch_item_config).
 * All items belong to `ctx`, share the coefficient type, and give grad for
 * all items or for none (BSI_E_INVAL otherwise).  The batch owns a device
 * workspace sized for the items; the item pointers are fixed at creation (new
 * particles are evaluated by writing them into the same buffers).
 * BSI_E_NOMEM if the workspace does not fit. */
bsi_status bsi_batch_create(bsi_ctx* ctx, const bsi_eval_item* items, int32_t count,
                            const bsi_eval_config* cfgs, bsi_batch** out);
/* Run the batch on `hip_stream`.  use_graph = 0 enqueues the kernels
 * directly; use_graph = 1 captures them into a HIP graph on the first call
 * (no memset nodes: counters are cleared by a kernel) and launches that graph
 * on every call. */
bsi_status bsi_batch_run(bsi_batch* batch, int32_t use_graph, void* hip_stream);
/* The configuration item `item` is evaluated with (variant 0 = tiled with
 * sort_tile 8, variant 1 = one lane per particle binned by sort_tile). */
bsi_status bsi_batch_item_config(const bsi_batch* batch, int32_t item, bsi_eval_config* cfg);
/* Device bytes of the batch workspace. */
size_t bsi_batch_bytes(const bsi_batch* batch);
/* Wait for the device, then free the batch and its graph. */
void bsi_batch_destroy(bsi_batch* batch);
/* One-shot: create, run without a graph, synchronise `hip_stream`, destroy. */
bsi_status bsi_eval_batch(bsi_ctx* ctx, const bsi_eval_item* items, int32_t count, void* hip_stream);

/* ---- serving: resident fields, continuous batching of particle queries --- */

typedef struct bsi_server_config {
    size_t hbm_budget;       /* device bytes for requests in flight (positions, outputs and
                                binning scratch), allocated once at creation             */
    int32_t max_slots;       /* requests on the GPU at once, one HIP stream each (1..64) */
    int32_t queue_capacity;  /* waiting requests before bsi_server_submit says BSI_E_BUSY */
    int32_t reserved[4];     /* must be 0 */
} bsi_server_config;

typedef struct bsi_server_report {
    int64_t completed;       /* requests finished successfully since the last reset      */
    int64_t failed;          /* requests that ended with an error                        */
    double p50_ns, p99_ns;   /* latency from submit to outputs in host memory            */
    double device_p50_ns, device_p99_ns;  /* first copy in to last copy out, on the GPU  */
    int64_t points;          /* particles of the completed requests                      */
    double points_per_s;     /* points / (last completion - first submit)                */
    int64_t max_inflight;    /* most requests on the GPU at once                         */
    size_t peak_arena_bytes; /* most arena bytes held at once                            */
} bsi_server_report;

/* Start a server on `ctx`: a device arena of cfg->hbm_budget bytes, max_slots
 * HIP streams (default priority) and one scheduler thread that owns all of
 * the server's GPU work.  Requests are admitted in arrival order as soon as a
 * slot is free and the arena holds the request's buffers; each admitted
 * request copies its positions in, runs the binned gather of its field (the
 * configuration bsi_ctx_lookup_config gives for its size) and copies u (and
 * grad) out on its slot's stream, so requests overlap on the device and a
 * request's result is bitwise the result of bsi_eval_ex on the same field
 * with that configuration, whatever else runs.  While a server runs, use its
 * context from other threads only after bsi_server_drain.  BSI_E_NOMEM if the
 * arena does not fit. */
bsi_status bsi_server_create(bsi_ctx* ctx, const bsi_server_config* cfg, bsi_server** out);
/* Make `field` (a field of the server's context, prefiltered by the caller)
 * servable under `field_id`.  The field must outlive the server. */
bsi_status bsi_server_add_field(bsi_server* server, int32_t field_id, bsi_field* field);
/* Queue a request: P (1 <= P < 2^31) positions pos_host [P][3] FP64, outputs
 * u_host [P][ncomp] and grad_host [P][ncomp][3] (or NULL) in host memory, in
 * the field's output type.  Host buffers should be pinned (hipHostMalloc) so
 * that copies overlap; they belong to the caller and must stay valid until
 * the request completes.  Returns a ticket.  BSI_E_NOMEM if the request alone
 * needs more than the arena, BSI_E_BUSY if the queue is full, BSI_E_INVAL for
 * an unknown field id. */
bsi_status bsi_server_submit(bsi_server* server, int32_t field_id, const double* pos_host, int64_t P,
                             void* u_host, void* grad_host, uint64_t* ticket);
/* *done = 1 once the request has completed (its outputs are in host memory);
 * the return value is then the request's own status.  latency_ns may be NULL.
 * A completed request's record is released once it has been collected: when
 * bsi_server_poll reports it done or bsi_server_wait returns it; a later poll
 * or wait of that ticket returns BSI_E_INVAL.  The server keeps the records
 * of requests completed and not yet collected, so callers collect every
 * ticket. */
bsi_status bsi_server_poll(bsi_server* server, uint64_t ticket, int32_t* done, int64_t* latency_ns);
/* Block until the request completes; returns its status (and collects it). */
bsi_status bsi_server_wait(bsi_server* server, uint64_t ticket, int64_t* latency_ns);
/* Block until every submitted request has completed. */
bsi_status bsi_server_drain(bsi_server* server);
/* Latency percentiles and throughput of the requests completed since the last
 * reset (percentiles over at most 2^20 requests: a uniform sample of them
 * when more have completed). */
bsi_status bsi_server_stats(bsi_server* server, bsi_server_report* out);
bsi_status bsi_server_reset_stats(bsi_server* server);
/* Finish every submitted request, stop the scheduler and free the server. */
void bsi_server_destroy(bsi_server* server);

/* ---- autotuning ------------------------------------------------------------- */

/* Time the candidate configurations of the evaluation (LDS-tiled gather with
 * sort tiles 4, 6, 8, 12, 16 and work items of 2, 4, 8 rounds; one lane per
 * particle binned by 4, 8, 16, 32) on P uniform positions generated on the
 * device from `seed`, and keep the fastest in the context's table under
 * (order, coefficient type, ncomp, density class round(log2(P / n0 n1 n2))).
 * When db_path is not NULL the entry is appended to that JSON-lines file.
 * best / best_us (may be NULL) receive the winner and its median time in
 * microseconds.  Allocates and frees its own buffers; synchronises. */
bsi_status bsi_tune(bsi_field* field, int64_t P, uint64_t seed, const char* db_path,
                    bsi_eval_config* best, double* best_us);
/* Add the entries of a JSON-lines file written by bsi_tune to the context's
 * table (later entries replace earlier ones with the same key).  BSI_E_INVAL
 * for an unreadable file or a malformed entry (nothing is added then). */
bsi_status bsi_ctx_load_tuning(bsi_ctx* ctx, const char* db_path);
/* The configuration bsi_eval and the batch planner use for `field` and P
 * particles: the table entry of the same key, else the nearest density class
 * (at most two away) of the same order/type/ncomp, else the built-in default
 * (tiled with 8^3-cell tiles from 1/64 particles per cell up, one lane per
 * particle below). */
bsi_status bsi_ctx_lookup_config(bsi_ctx* ctx, const bsi_field* field, int64_t P, bsi_eval_config* out);
/* Write P uniform positions in [0,L0)x[0,L1)x[0,L2) (length[3]) to pos_dev
 * [P][3]: coordinate d of particle p is L_d * u(3p + d), u(i) the top 53 bits
 * of SplitMix64 output i of `seed` (Steele, Lea and Flood 2014) over 2^53.
 * Used for tuning and for load generation. */
bsi_status bsi_fill_uniform_positions(bsi_ctx* ctx, uint64_t seed, int64_t P, const double* length,
                                      double* pos_dev, void* hip_stream);

/* ---- synthetic workloads and memory ---------------------------------------- */

/* Write a synthetic Kolmogorov-spectrum field (not part of the method; a
 * workload generator for benchmarks and serving loads) into uhat_dev
 * [ncomp][n][n][n/2+1], complex128 (prec = BSI_F64) or complex64 (BSI_F32):
 * amplitude |k|^(-11/6) for 0 < |k| <= n/3 and zero elsewhere, phase 2 pi u
 * with u from SplitMix64 (Steele, Lea and Flood 2014) output `counter` of
 * stream c = component, the stream starting at mix((seed * 0x9E3779B97F4A7C15)
 * xor c) and `counter` the flat half-spectrum index of the canonical member of
 * a Hermitian pair (the other member of a k2 = 0 pair is its conjugate);
 * divergence_free projects three components onto k-perpendicular per mode;
 * one global factor sets the mean over components of sum_k |uhat_k|^2 over the
 * full spectrum to 1.  n even, 2 <= n <= 4096.  Synchronises the stream. */
bsi_status bsi_synth_kolmogorov(bsi_ctx* ctx, int32_t n, int32_t ncomp, uint64_t seed,
                                int32_t divergence_free, int32_t prec, void* uhat_dev, void* hip_stream);
/* Wait for the device and free the context's cached FFT and evaluation
 * workspaces (they are allocated again on demand). */
bsi_status bsi_ctx_trim(bsi_ctx* ctx);

/* ---- stage timing -------------------------------------------------------- */

/* Enable (1) or disable (0) per-stage timing on a context.  While enabled, the
 * library brackets each of its kernel launches with HIP events recorded on the
 * launch stream, so durations are those of the kernels themselves.  Stages:
 * "fft_axis0", "fft_axis1", "fft_c2r", "bin_count", "bin_scan", "bin_scatter",
 * "gather"; batches: "batch_bin", "batch_gather" (direct runs) and
 * "batch_graph" (graph launches).  Nothing is timed inside a stream capture. */
bsi_status bsi_ctx_set_timing(bsi_ctx* ctx, int32_t enabled);
/* Total milliseconds and number of launches recorded for `stage` since the
 * last reset (waits for the recorded events). */
bsi_status bsi_ctx_read_timing(bsi_ctx* ctx, const char* stage, double* total_ms, int64_t* launches);
/* Forget all recorded timings. */
bsi_status bsi_ctx_reset_timing(bsi_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BSI_H */
