/*
 * sip.h — C ABI of the MI355X (gfx950) PARSDMM library (libsip.so).
 *
 * PARSDMM (Peters & Herrmann, arXiv:1902.09699) projects a model m on a 2D or
 * 3D regular grid onto the intersection of p sets V_i = {x | A_i x in C_i}
 * (Sec. "PARSDMM: Exploiting similarity between constraint sets", eq.
 * proj_intersect_indicator).  The library adds the identity block
 * A_{p+1} = I with the squared-distance prox (eqs. PARSDMM_2, prox_sq_dist)
 * and runs the iteration of eq. SDMM_adaptive / the PARSDMM listing:
 * a warm-started CG x-update on C = sum_i rho_i A_i^T A_i + rho_{p+1} I
 * (eqs. sys_mat, cg_stop), the per-set relaxation, projection and multiplier
 * update, the adapt-rho-gamma listing every adapt_every iterations and,
 * optionally, the stopping test of eqs. feas_stop / obj_stop.
 *
 * Conventions
 *  - Grids are C-ordered: axis 0 is z (vertical, slowest), the last axis is
 *    x (contiguous).  2D: n = {nz, nx}; 3D: n = {nz, ny, nx}.
 *  - D_a is the forward difference of eq. FD_mat along axis a, scaled by
 *    1/h[a]; its output lives on the grid with the last layer along a unused.
 *  - Every device pointer is HIP device memory of the plan's field type
 *    (float or double), C-ordered, N = prod(n) elements, 256-byte alignment
 *    not required.  The caller owns m and x.  Streams are hipStream_t passed
 *    as void*; NULL means the default stream.
 *  - Functions return sip_status (0 on success).  No exception crosses the
 *    ABI.  Plans and batches are not thread-safe; different plans on
 *    different streams are.
 *  - Results are bit-reproducible for float fields: the per-instance work
 *    decomposition and every reduction order depend only on the instance
 *    itself, not on the other instances sharing a batch.
 */
#ifndef SIP_H
#define SIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIP_MAX_SETS 16   /* the paper works with up to about 16 sets */

typedef enum {
  SIP_OK = 0,
  SIP_EINVAL = -1,       /* bad shape, set parameter, option or argument */
  SIP_ENOMEM = -2,       /* device or host allocation failed */
  SIP_EHIP = -3,         /* a HIP runtime call failed */
  SIP_ENUMERIC = -4,     /* non-finite input/iterate or CG breakdown (p^T C p <= 0) */
  SIP_EUNSUPPORTED = -5, /* combination the library does not implement */
  SIP_EBUDGET = -6,      /* batch: no free slot or not enough arena memory; plan: workspace too small */
  SIP_ETOOLARGE = -7     /* sip_project_noalloc: the instance needs more than its fixed device array */
} sip_status;

typedef enum { SIP_F32 = 0, SIP_F64 = 1 } sip_dtype;

/* Linear operators A_i (Sec. "Notation", eq. FD_mat; Table set-overview). */
typedef enum {
  SIP_OP_I = 0,    /* identity */
  SIP_OP_DZ = 1,   /* D_z (x) I: vertical difference */
  SIP_OP_DY = 2,   /* 3D only */
  SIP_OP_DX = 3,   /* I (x) D_x: horizontal difference */
  SIP_OP_GRAD = 4, /* [D_z; (D_y;) D_x] stacked: anisotropic total variation */
  SIP_OP_LAT = 5   /* [(D_y;) D_x] stacked: lateral differences */
} sip_op;

/* Simple sets C_i (Table set-overview). */
typedef enum {
  SIP_SET_BOUNDS = 0, /* lo <= (A x)[j] <= hi, +-INFINITY allowed; or per-row bound vectors */
  SIP_SET_L1 = 1,     /* ||A x||_1 <= tau */
  SIP_SET_CARD = 2,   /* card(A x) <= k: keep the k largest |.|, ties to the lower index */
  SIP_SET_L2 = 3,     /* ||A x||_2 <= tau */
  SIP_SET_ANNULUS = 4 /* lo <= ||A x||_2 <= hi (not convex for lo > 0): radial projection;
                         at A x = 0 the projection is lo times the first row's unit vector */
} sip_set_kind;

/* Line-wise sets (the paper's constraints on every row, column or fiber of
 * the model, section "Software and numerical examples" and the
 * full-waveform example): the set's projection acts on every line of A x on
 * its own; the operator is unchanged.  A line is a run of entries of one
 * component block of A x (an image of the grid, one layer shorter along the
 * component's difference axis) that differ only in the coordinate along the
 * line axis: 2D SIP_LINE_X is a row X[i, :], SIP_LINE_Z a column X[:, j].
 * L1, CARD (k per line), L2 and ANNULUS (at a zero line: lo on its first
 * entry) sets only; lines hold at most 4096 (float) or 2048 (double)
 * entries (SIP_EUNSUPPORTED beyond); not supported by sip_project_multilevel. */
typedef enum {
  SIP_LINE_NONE = 0, /* the set acts on the whole vector A x */
  SIP_LINE_Z = 1,
  SIP_LINE_Y = 2,    /* 3D only */
  SIP_LINE_X = 3
} sip_line;

typedef struct {
  int32_t ndim;   /* 2 or 3 */
  int32_t reserved;
  int64_t n[3];   /* sizes, axis 0 first; every size >= 1, N < 2^31 */
  double h[3];    /* grid spacings (> 0) used by the difference operators */
} sip_grid;

typedef struct {
  int32_t kind;   /* sip_set_kind */
  int32_t op;     /* sip_op; the operator's axes need at least 2 points */
  double lo, hi;  /* BOUNDS: lo <= hi; ANNULUS: radii, 0 <= lo <= hi */
  double tau;     /* L1, L2: tau >= 0 */
  int64_t k;      /* CARD: 1 <= k <= rows of A (line-wise: k >= 1 per line) */
  /* BOUNDS only, per-pixel bounds l[j] <= (A x)[j] <= u[j] (NULL: the scalar
   * lo / hi): device arrays of the field type, one block of N elements per
   * component of A in the grid's C order (the row of grid point P of
   * component c at c*N + P; entries of the unused last layer along the
   * component's axis are ignored).  Copied into the workspace when the
   * instance is admitted; the caller may free them afterwards.  Not
   * supported by sip_project_multilevel. */
  const void* lo_vec;
  const void* hi_vec;
  int32_t line;   /* sip_line */
  int32_t reserved_;
} sip_set;

typedef struct {
  int32_t max_iter;     /* PARSDMM iterations (cap when stopping is on); default 200 */
  int32_t cg_max;       /* CG steps per x-update (cap); default 10 */
  int32_t cg_fixed;     /* 1: exactly cg_max steps unless the residual is exactly 0 */
  int32_t adapt_every;  /* adapt-rho-gamma when k mod adapt_every == 1; 0 = off; default 2 */
  int32_t stop_every;   /* stopping test when k mod stop_every == 0; 0 = off (default) */
  int32_t evol_hist;    /* history length s of r_evol; default 5, at most 8 */
  double rho0, gamma0;  /* initial penalty and relaxation; default 1, 1 */
  double eps_corr;      /* correlation threshold of adapt-rho-gamma; default 0.3 */
  double rho_ratio_max; /* rho_i kept within [rho_{p+1}/R, R rho_{p+1}]; default 100 */
  double gamma_max;     /* relaxation cap below 2; default 1.999 */
  double eps_evol;      /* default 1e-2 */
  double eps_feas;      /* default 1e-3 */
  double cg_rel;        /* CG stops when ||r|| < cg_rel ||r_0||; default 0.1 */
  int32_t field;        /* sip_dtype of m, x and every field */
  int32_t reduce;       /* sip_dtype of every reduction (CG inner products, residual and stopping
                           norms, adapt dots, l1 bucket and prefix sums): SIP_F64 (default), or
                           SIP_F32 with field SIP_F32 (the pure-FP32 precision ablation) */
  int32_t log_schedule; /* 1: record (rho, gamma) of every iteration (sip_batch_schedule) */
  int32_t sel_fresh;    /* 1: every threshold selection reads all of w in its refine passes; 0
                           (default): the w pass also gathers the entries of the previous
                           iteration's first-digit bucket, and a selection whose first digit falls in
                           that bucket refines over them alone.  The same results either way. */
} sip_opts;

typedef struct {
  int32_t status;     /* sip_status of this instance */
  int32_t iters;      /* iterations run */
  int32_t cg_steps;   /* CG steps run, summed over iterations */
  int32_t converged;  /* 1 when the stopping test passed */
  int32_t nsets;
  int32_t sel_reused; /* threshold selections (pipelines x iterations) that refined over the
                         entries the w pass gathered (see sip_opts.sel_fresh) */
  double r_evol;                    /* last evaluated r_evol (eq. obj_stop), or -1 */
  double r_feas[SIP_MAX_SETS];      /* last evaluated r_feas_i (eq. feas_stop), or -1 */
  double rho[SIP_MAX_SETS + 1];     /* final rho_i, index nsets is rho_{p+1} */
  double gamma[SIP_MAX_SETS + 1];   /* final gamma_i */
} sip_result;

typedef struct sip_batch sip_batch;

/* Readable name of a status code (static storage). */
const char* sip_strerror(int32_t status);

/* Fill *o with the defaults listed in sip_opts. */
int32_t sip_opts_default(sip_opts* o);

/* Rows M_i of A_i on the grid (e.g. (nz-1) nx for D_z on nz x nx), or -1. */
int64_t sip_set_rows(const sip_grid* g, const sip_set* s);

/* Check a grid + set list + options; SIP_OK or SIP_EINVAL / SIP_EUNSUPPORTED. */
int32_t sip_validate(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o);

/* Exact device bytes one instance occupies in a batch arena (state vectors,
 * adapt snapshots, selection scratch, scalars), rounded to 256 bytes. */
int64_t sip_workspace_bytes(const sip_grid* g, const sip_set* sets, int32_t nsets,
                            const sip_opts* o);

/* One blocking projection (the PARSDMM listing): x <- P_{cap V_i}(m).
 * m_dev and x_dev are device arrays of N field elements; x_dev may equal
 * m_dev.  Allocates the instance workspace, runs up to max_iter iterations on
 * `stream`, waits, fills *res (may be NULL) and frees the workspace.
 * Returns the instance status. */
int32_t sip_project(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                    const void* m_dev, void* x_dev, sip_result* res, void* stream);

/* B independent projections of uneven size in one batch: instance b has grid
 * grids[b], sets sets_flat[off_b .. off_b + nsets[b]) (off_b = sum of earlier
 * nsets) and device arrays m_dev[b], x_dev[b].  Every phase of an iteration
 * is one launch over a work table of all instances' tiles, and `graph_iters`
 * iterations are replayed as one captured HIP graph.  Blocks until every
 * instance stopped; res (array of B, may be NULL) gets the per-instance
 * results.  Returns SIP_OK or the first failing instance's status. */
int32_t sip_project_batched(int32_t B, const sip_grid* grids, const sip_set* sets_flat,
                            const int32_t* nsets, const sip_opts* o,
                            const void* const* m_dev, void* const* x_dev,
                            sip_result* res, int32_t graph_iters, void* stream);

/* ---- resident batches (the served form and step-level control) ---------- */

/* A batch holds up to max_slots instances whose state stays on the device in
 * an arena of arena_bytes (one allocation made here, from which admission
 * carves every instance's state).  The work tables and per-item partial-sum
 * buffers are sized to the admitted instances: the first sip_batch_run after
 * an admission or removal that outgrows their capacity (capacities double)
 * reallocates them, after waiting for the stream.  All instances share the
 * options and field type. */
int32_t sip_batch_create(sip_batch** out, int32_t max_slots, int64_t arena_bytes,
                         const sip_opts* o);
int32_t sip_batch_destroy(sip_batch* b);

/* Admit one instance: carve its workspace from the arena and enqueue its
 * initialisation (x = m, y_i = A_i m, v_i = 0, rho_i = rho0, gamma_i = gamma0,
 * k = 1) on `stream`.  m_dev must stay valid until the initialisation ran;
 * x_dev receives the iterate in place until the slot is removed.
 * SIP_EBUDGET when no slot is free or the arena has no room. */
int32_t sip_batch_add(sip_batch* b, const sip_grid* g, const sip_set* sets, int32_t nsets,
                      const void* m_dev, void* x_dev, int32_t* slot, void* stream);

/* Enqueue `iters` iterations for every active, unfinished instance on
 * `stream` (a captured graph replayed; instances that finish stop early). */
int32_t sip_batch_run(sip_batch* b, int32_t iters, void* stream);

/* Wait for `stream`, then report per slot whether the instance finished
 * (done[s] = 1, stopped or reached max_iter or failed), was running (0) or
 * the slot is free (-1).  done has max_slots entries. */
int32_t sip_batch_poll(sip_batch* b, int32_t* done, void* stream);

/* Wait for `stream`, copy the slot's result and release its workspace. */
int32_t sip_batch_remove(sip_batch* b, int32_t slot, sip_result* res, void* stream);

/* Wait for `stream` and copy the slot's current result without removing it. */
int32_t sip_batch_result(sip_batch* b, int32_t slot, sip_result* res, void* stream);

/* Device arrays of a slot's state for export/import by the caller (same
 * stream ordering rules as any device memory).  which: 0 y_i, 1 v_i,
 * 2 vhat snapshot, 3 v snapshot, 4 y snapshot (i = nsets means the identity
 * block p+1); 5 r (the CG residual buffer; with cg_form 1 or 2 it holds the
 * warm-start residual or that of an even step), 6 x-snapshot buffer 0,
 * 7 x-snapshot buffer 1.  Set
 * arrays hold one block per operator component (z, y, x order), block c
 * starting at element c * comp_stride (comp_stride >= N, 256-byte aligned);
 * the first N entries of a block are the grid points, the unused last layer
 * along the component's axis and the tail padding are kept at zero.  count
 * is the number of elements of the whole array. */
int32_t sip_batch_field(sip_batch* b, int32_t slot, int32_t which, int32_t set,
                        void** dev_ptr, int64_t* count, int64_t* comp_stride);

/* Read / overwrite a slot's scalars: rho and gamma (nsets+1 each), the
 * iteration counter k and whether adapt-rho-gamma holds a snapshot. */
int32_t sip_batch_get_params(sip_batch* b, int32_t slot, double* rho, double* gamma,
                             int32_t* k, int32_t* have_snapshot, void* stream);
int32_t sip_batch_set_params(sip_batch* b, int32_t slot, const double* rho, const double* gamma,
                             int32_t k, int32_t have_snapshot, void* stream);

/* With opts.log_schedule: copy (rho, gamma) used in iterations 1..n
 * (n = min(iters run, max_n)) as n rows of nsets+1 values each. */
int32_t sip_batch_schedule(sip_batch* b, int32_t slot, double* rho, double* gamma,
                           int32_t max_n, int32_t* n, void* stream);

/* Work decomposition: grid points per item of the point kernels (RHS, CG,
 * projection) and of the threshold-set kernels, each a multiple of 256, and
 * grown when an instance would need more than max_items items; pt_threads
 * (256 or 512) is the block size of the RHS and CG kernels.  cg_form picks
 * the arrangement of the CG steps of the x-minimization (section "Solving the
 * linear system"): 0 the textbook form, two launches and two inner-product
 * reductions per step; 1 Chronopoulos and Gear's one-reduction form, one
 * launch per step (the same iterates in exact arithmetic, different
 * rounding; 10 instead of 8 vectors of traffic per step, fewer launches: it
 * pays on grids too small to keep the GPU busy); 2 one launch per step that
 * stages p of each item with one row before and two after, and r of the
 * item and the row after, in LDS, forms C p and the next residual there and
 * stores x, r, p only (6 vectors), with p^T C p from its expansion in the
 * previous step's sums (the textbook iterates' expressions; only that
 * double is summed another way), plus one r_0^T C r_0 pass per
 * x-minimization — for the instances without a y axis whose staged rows
 * fit 60 KiB of LDS (the batch's other instances run form 0 steps beside
 * them).
 * Results are bit-identical
 * for any batch composition at fixed tile settings.  Applies from the next
 * sip_batch_run.  Defaults 2048/512, 2048/512, 512 threads, form 0.
 * SIP_EINVAL for sizes that are not multiples of 256, max_items < 1, another
 * thread count or another form. */
int32_t sip_batch_set_tiles(sip_batch* b, int32_t pt_points, int32_t pt_max_items, int32_t thr_points,
                            int32_t thr_max_items, int32_t pt_threads, int32_t cg_form);

/* Re-initialise a slot's state from a new m of the same grid (x = m,
 * y_i = A_i m, v_i = 0, rho0/gamma0, k = 1) without touching the work tables
 * or captured graphs. */
int32_t sip_batch_reset(sip_batch* b, int32_t slot, const void* m_dev, void* stream);

/* Kernels that sip_batch_time_kernel can time in isolation. */
typedef enum {
  SIP_K_RHS = 0,       /* RHS + residual + r^T r */
  SIP_K_CG_DIR = 1,    /* CG direction update + p^T C p (step 1) */
  SIP_K_CG_UPD = 2,    /* CG x / r update + r^T r (step 1) */
  SIP_K_PROJ = 3,      /* bounds sets + identity block: relax, project, dual update */
  SIP_K_THR_W = 4,     /* threshold sets: w and the first radix histogram */
  SIP_K_THR_APPLY = 5, /* threshold sets: apply threshold + dual update */
  SIP_K_CG1_STEP = 6,  /* one-reduction CG step (step 1; run a cg_form 1 iteration first) */
  SIP_K_CG1_W0 = 7,    /* one-reduction CG: w_0 = C r_0 + r_0^T w_0 */
  SIP_K_LINE = 8,      /* line-wise sets: relax, project every line, dual update */
  SIP_K_CG2_STEP = 9,  /* LDS-staged CG step (step 1; only where the batch runs cg_form 2) */
  SIP_K_CG2_D0 = 10    /* LDS-staged CG: r_0^T C r_0 */
} sip_kernel_id;

/* Launch one kernel of the iteration `reps` times on `stream` over the
 * batch's current work tables, bracketed by HIP events, and return the mean
 * duration per launch in *avg_ms.  The kernel really runs: the slot states
 * change (time only after the results you need were read). */
int32_t sip_batch_time_kernel(sip_batch* b, int32_t kernel, int32_t reps, void* stream, double* avg_ms);

/* Plain device copy of `bytes` (a multiple of 16) from src to dst on
 * `stream`: the reference kernel for achievable HBM bandwidth and for
 * calibrating the FETCH_SIZE / WRITE_SIZE counters. */
int32_t sip_stream_copy(void* dst, const void* src, int64_t bytes, void* stream);

/* Per-kernel launch statistics of the last sip_batch_run: number of work
 * items of each phase (rhs/CG, threshold, selection, instance). */
int32_t sip_batch_items(sip_batch* b, int32_t* n_point_items, int32_t* n_thr_items,
                        int32_t* n_pipelines, int32_t* n_instances);

/* ---- Multilevel PARSDMM (section "Multilevel PARSDMM", ML-PARSDMM listing).
 * Coarse-to-fine continuation: level l (0 = the given grid) has ceil(n / 2)
 * points per axis of level l - 1 (samples 0, 2, 4, ...), spacing h * 2^l;
 * PARSDMM runs on the coarsest level from the usual start (x = m_l,
 * y_i = A_i m_l, v_i = 0), then x, y_i and v_i (i = 1..p+1) are interpolated
 * as images to the next finer grid and used as its initial guess, up to
 * level 0.  (rho, gamma) restart from (rho0, gamma0) on every level, or
 * continue from the coarser level's final values (carry_params = 1). */

/* Grid and set list of level `level`: bounds unchanged; an l1 tau and a
 * cardinality k scaled by rows of A at that level / rows at level 0
 * (k = floor(k * ratio + 1/2) within [1, rows]).  sets_out holds nsets
 * entries.  SIP_EINVAL on bad arguments; does not validate the level's
 * sets (an axis may become too short for a difference operator). */
int32_t sip_level(const sip_grid* g, const sip_set* sets, int32_t nsets, int32_t level,
                  sip_grid* g_out, sip_set* sets_out);

/* The coarse model of the next level: the binomial [1, 2, 1] / 4 filter
 * along every axis (edges replicated) followed by every other sample from 0.
 * src_dev: N elements of type dtype on grid g; dst_dev: the coarse grid's
 * elements (sip_level(g, ..., 1, ...)).  Enqueued on `stream`. */
int32_t sip_restrict(const sip_grid* g, int32_t dtype, const void* src_dev, void* dst_dev, void* stream);

/* Multilevel projection of m_dev onto the intersection, with nlevels levels
 * (1 = plain PARSDMM) and level_iters[l] the iteration cap of level l
 * (0 = the given grid; stopping rule per level as in opts); carry_params:
 * 0 = every level starts from (rho0, gamma0), 1 = from the coarser level's
 * final (rho, gamma).  Interpolation
 * is linear along each axis at the geometric position of every fine sample
 * (points at i / 2; rows of a difference along an axis at (i + 1/2) / 2 - 1/2
 * on that axis), clamped to the coarse image.  Allocates the coarse models
 * and iterates and each level's workspace, blocks until done, frees them.
 * *res (may be NULL): the result on the given grid; level_iters_run (nlevels
 * entries, may be NULL): iterations each level ran.  SIP_EINVAL when a level
 * is invalid (e.g. an axis of a difference operator shorter than 2 points),
 * otherwise as sip_project. */
int32_t sip_project_multilevel(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                               int32_t nlevels, const int32_t* level_iters, int32_t carry_params,
                               const void* m_dev, void* x_dev, sip_result* res, int32_t* level_iters_run,
                               void* stream);

/* ---------------------------------------------------------------- parallel Dykstra
 * The paper's baseline for its PARSDMM comparison (Appendix A, the
 * Parallel-DYKSTRA listing): x^0 = m, v_i^0 = m; each iteration projects
 * every v_i onto V_i = {x | A_i x in C_i} (independently: the single-set
 * PARSDMM instances of one batch, the paper's inner adaptive ADMM), then
 * x = sum_i w_i y_i and v_i = x + v_i - y_i.  This call does the last two
 * steps on the device: y[i], v[i] (i < p) and x are device arrays of n
 * elements of the field type (float for SIP_F32, double for SIP_F64),
 * caller-owned; w holds p host weights (the listing asks for sum 1; not
 * enforced).  x must not alias any y[i] or v[i].  Asynchronous on `stream`.
 * SIP_EINVAL for p outside [1, SIP_MAX_SETS], a null pointer, n < 0 or
 * another field. */
int32_t sip_dykstra_update(int32_t p, const void* const* y, void* const* v, const double* w, void* x, int64_t n,
                           int32_t field, void* stream);

/* ------------------------------------------------------------------ plans
 * The paper's set-up-once / project-many sequence (section "Software and
 * numerical examples": the constraint set-up and precomputation are done
 * once and reused) for one grid and set list: a plan precomputes the
 * operator descriptors, the state layout and the work tables at creation,
 * captures the iteration graphs at its first run and reuses all of them for
 * every later model m.  Not thread-safe; one plan per stream at a time. */

typedef struct sip_plan sip_plan;

/* Work decomposition of a plan (the tiles of sip_batch_set_tiles). */
typedef struct {
  int32_t pt_points, pt_max_items;   /* grid points per item of the RHS, CG and projection kernels; item cap */
  int32_t thr_points, thr_max_items; /* the same for the threshold-set kernels */
  int32_t pt_threads;                /* 256 or 512 */
  int32_t cg_form;                   /* 0 textbook CG, 1 one-reduction CG, 2 LDS-staged one-launch CG */
} sip_tiles;

/* Fill *t with the default tiles (2048/512, 2048/512, 512 threads, form 0). */
int32_t sip_tiles_default(sip_tiles* t);

/* Exact device bytes a plan needs for (grid, sets, options, tiles) when it
 * takes its memory from a caller workspace: descriptor, scalars, the
 * instance's state and the work tables; tiles NULL = defaults.  -1 when the
 * arguments are invalid. */
int64_t sip_plan_bytes(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                       const sip_tiles* tiles);

/* Create a plan.  workspace NULL: the library allocates its device memory;
 * otherwise every device buffer of the plan is carved from the caller's
 * block [workspace, workspace + workspace_bytes) (256-byte aligned, at
 * least sip_plan_bytes, owned by the caller and left alone until
 * sip_plan_destroy).  Per-row bound vectors of the sets are copied into the
 * plan here.  SIP_EINVAL for bad arguments or an unaligned workspace,
 * SIP_EBUDGET for a workspace smaller than sip_plan_bytes. */
int32_t sip_plan_create(sip_plan** out, const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                        const sip_tiles* tiles, void* workspace, int64_t workspace_bytes, void* stream);
int32_t sip_plan_destroy(sip_plan* p);

/* One blocking projection of m_dev with the plan (the PARSDMM listing, as
 * sip_project): x_dev (N field elements, may equal m_dev) receives the
 * result; *res (may be NULL) the result record.  Returns the status. */
int32_t sip_plan_project(sip_plan* p, const void* m_dev, void* x_dev, sip_result* res, void* stream);

/* Step-level control: sip_plan_start restarts the plan's state from m_dev
 * (x = m, y_i = A_i m, v_i = 0, rho0, gamma0, k = 1; waits for the stream)
 * with the iterate kept in x_dev; sip_plan_iterate enqueues up to `iters`
 * more iterations (fewer when the stopping test or max_iter ends the run);
 * sip_plan_result waits for the stream and reads the result record. */
int32_t sip_plan_start(sip_plan* p, const void* m_dev, void* x_dev, void* stream);
int32_t sip_plan_iterate(sip_plan* p, int32_t iters, void* stream);
int32_t sip_plan_result(sip_plan* p, sip_result* res, void* stream);

/* The whole iteration state of a started plan, for the listing's optional
 * initial guess of x, y_i and v_i (PARSDMM listing, input line): the
 * iterate x, every y_i and v_i (identity block included), rho_i, gamma_i,
 * the iteration counter, the adapt-rho-gamma snapshots, the x history of
 * the stopping test, the selection state and the schedule log, behind a
 * header naming the layout.  sip_state_bytes: size of the blob;
 * sip_state_export copies it into dst_dev (device memory of that size;
 * waits for the stream); sip_state_import overwrites the plan's state from
 * a blob exported by a plan of the same grid, set kinds and operators and
 * options (SIP_EINVAL otherwise, or before sip_plan_start), asynchronously
 * on `stream`.  Iterating after an import continues exactly as the
 * exporting plan would have. */
int64_t sip_state_bytes(const sip_plan* p);
int32_t sip_state_export(sip_plan* p, void* dst_dev, void* stream);
int32_t sip_state_import(sip_plan* p, const void* src_dev, void* stream);

/* ------------------------------------------------------ allocation-free form
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * projection of sip_project with the default tiles, whose every device
 * buffer (descriptor, scalars, instance state, work tables, partial sums,
 * selection histograms) is carved from a fixed 128 MiB device array of the
 * library (one per GPU, held until the process ends).  It makes no HIP
 * allocation (no hipMalloc, hipHostMalloc, hipFree, stream or graph
 * creation) and launches the iterations directly on `stream`; host-side
 * bookkeeping uses ordinary heap memory.  SIP_ETOOLARGE when the instance
 * needs more than the array (sip_plan_bytes with default tiles above
 * 128 MiB; e.g. a 341 x 1361 grid with four sets needs about 70 MiB).
 * Blocking.  Every call on a GPU reuses that GPU's array, so calls that
 * overlap on one GPU (other threads, other streams) race: serialise them. */
int32_t sip_project_noalloc(const sip_grid* g, const sip_set* sets, int32_t nsets, const sip_opts* o,
                            const void* m_dev, void* x_dev, sip_result* res, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* SIP_H */
