/*
 * gbem.h -- C ABI of the MI355X (gfx950) Galerkin boundary element
 * capacitance extractor.
 *
 * Method: arXiv 2203.11733 ("GBEM"), single-dielectric case, section 3.
 * The boundary of the conductors (and of an optional grounded enclosure) is
 * split into axis-aligned rectangles I_j; with piecewise constant charge the
 * Galerkin system is A X = B with
 *     A_ij = 1/(4 pi |I_i||I_j|) Int_{I_i} Int_{I_j} 1/|x-y|     (section 3.1, eq. "matrix")
 *     B_ik = 1 if I_i lies on conductor k, else 0               (eq. "lineareq1", one
 *                                                                right-hand side per main net)
 * A is symmetric positive definite (section 3.2, Theorem 1) and is factored by
 * Cholesky; the Maxwell capacitance matrix is
 *     C_kl = eps_r * eps0 * l * sum_{i on conductor k} X_il      (eq. "electriccharge";
 *                                                                C_1n = Q_n, section 3.2)
 * with eps0 = 8.8541878128e-12 F/m and l the length of one coordinate unit in
 * metres.  Self and near pairs are integrated in closed form (section 3.4),
 * far pairs by a p x p tensor Gauss-Legendre rule per panel.
 *
 * Conventions for every entry point:
 *  - Return codes only: nothing aborts or throws across the ABI.  On failure
 *    gbem_last_error() returns a message for the calling thread.
 *  - Host input arrays are read during the call (or copied before a
 *    non-blocking call returns); the caller keeps ownership.
 *  - Outputs are written only when GBEM_OK is returned.
 *  - "device" pointers are HIP device allocations on the context's device;
 *    "stream" arguments are hipStream_t passed as void* (NULL = the
 *    context's own stream).
 *  - A context is bound to one device.  Calls on one context are serialised
 *    internally, except gbem_submit/gbem_poll/gbem_wait which are thread-safe
 *    and overlap with other jobs.
 */
#ifndef GBEM_H
#define GBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gbem_ctx gbem_ctx;   /* opaque: device context, workspaces, serving loop */
typedef struct gbem_job gbem_job;   /* opaque: one submitted extraction */

typedef enum {
    GBEM_OK = 0,
    GBEM_EINVAL = 1,    /* invalid argument or mesh */
    GBEM_ENOMEM = 2,    /* device memory or the HBM budget cannot hold the job */
    GBEM_EDEVICE = 3,   /* a HIP call failed */
    GBEM_ENOTPD = 4,    /* Cholesky met a non-positive pivot */
    GBEM_ENOCONV = 5,   /* iterative refinement did not reach the tolerance (kept for the ABI: a
                         * stalled refinement now retries with a stronger factor instead) */
    GBEM_EBUSY = 6,     /* job still running (gbem_poll) */
    GBEM_ETIMEOUT = 7   /* gbem_wait timed out */
} gbem_status;

typedef enum {
    GBEM_F64 = 0,
    GBEM_F32 = 1,
    GBEM_F16 = 2,       /* factor stored FP32, trailing updates on FP16 MFMA, FP32 accumulate */
    GBEM_BF16 = 3       /* factor stored FP32, trailing updates on BF16 MFMA, FP32 accumulate */
} gbem_dtype;

/* Basis of the surface charge.  The method uses a piecewise constant density,
 * one unknown per panel (section 3.1: q_j constant on I_j); it is the only
 * basis, and the field exists so a mesh states it. */
typedef enum {
    GBEM_BASIS_P0 = 0
} gbem_basis;

/* A mesh: n_panels axis-aligned rectangles.  Panel i is the box lo[3i..3i+2] ..
 * hi[3i..3i+2] with exactly one axis where lo == hi (its normal axis) and
 * lo < hi on the other two.  conductor[i] is in [-1, n_conductors); -1 marks
 * a grounded panel (e.g. the paper's Dirichlet outer boundary, section 3.1)
 * that takes part in the system but has no right-hand side and is not reported. */
typedef struct {
    int32_t n_panels;
    int32_t n_conductors;
    const double *lo;           /* [3 * n_panels] */
    const double *hi;           /* [3 * n_panels] */
    const int32_t *conductor;   /* [n_panels] */
    double eps_r;               /* relative permittivity of the uniform dielectric, > 0 */
    double length_unit_m;       /* metres per coordinate unit (1e-6 for micrometres), > 0 */
    int32_t basis;              /* gbem_basis; must be GBEM_BASIS_P0 (zero-initialised structs are) */
} gbem_mesh;

typedef struct {
    int32_t far_order;          /* p: Gauss points per panel direction for far pairs, 1..8 (default 3) */
    double near_eta;            /* near iff dist^2 < eta^2 * max(diam_i^2, diam_j^2) (default 2, at least
                                 * 1e-6 so that pairs at zero distance, each panel with itself
                                 * included, are near: GBEM_EINVAL below);
                                 * near pairs get the exact integral, far pairs p x p Gauss.  A value
                                 * above every separation/diameter ratio of the mesh (e.g. 1e6) puts
                                 * every pair on the exact path: the exact reference mode (all
                                 * N(N+1)/2 pairs in the near list, about 1.5 s at N = 21,420) */
    int32_t far_dtype;          /* gbem_dtype of the far-pair arithmetic: GBEM_F64 or GBEM_F32 */
    int32_t factor_dtype;       /* gbem_dtype of the factorisation (GBEM_F64: no refinement) */
    double refine_tol;          /* refinement stops when max_k |b_k - A x_k|_2 / |b_k|_2 <= tol */
    int32_t max_refine;         /* refinement iteration cap (default 30) */
    int32_t profile;            /* bit c set: time the launches of kernel class c (gbem_kernel_class) with
                                   HIP events on their streams (gbem_report.prof_*); 0: no events */
    int32_t graph;              /* 1: replay the launches between the near-list readback and the first
                                   refinement readback (FP64: the end of the solve) as one hipGraph,
                                   captured per job and applied to the worker's cached executable of
                                   the same launch topology (hipGraphExecUpdate; instantiated when none
                                   matches); same kernels and results as 0.  Ignored with profile != 0;
                                   refused by gbem_extract_device_noalloc (instantiation allocates).
                                   Report times with 1: assemble = panels, near test and far field,
                                   factor = the graph, solve = the rest. */
} gbem_opts;

/* Kernel classes of gbem_report.prof_* (see the design notes for their work units). */
enum {
    GBEM_K_FAR = 0,         /* far-field Gauss tiles */
    GBEM_K_NEAR_LIST = 1,   /* near/far classification and CSR */
    GBEM_K_NEAR_EVAL = 2,   /* closed-form near entries */
    GBEM_K_DIAG = 3,        /* 128 x 128 diagonal-block Cholesky + inverse */
    GBEM_K_TRSM = 4,        /* panel solve (GEMM with the block inverse) + copy */
    GBEM_K_SYRK = 5,        /* trailing update of the matrix beyond the next panel (MFMA) */
    GBEM_K_SOLVE = 6,       /* triangular solves */
    GBEM_K_RESIDUAL = 7,    /* FP64 residual of the refinement */
    GBEM_K_PANEL = 8,       /* updates inside and of the next outer panel (look-ahead path) */
    GBEM_K_OTHER = 9,
    GBEM_K_COUNT = 10
};

typedef struct {
    double t_assemble_ms;       /* panel table + near list + far + near kernels */
    double t_factor_ms;         /* scaling/conversion + Cholesky */
    double t_solve_ms;          /* triangular solves + refinement + charge sums */
    double t_total_ms;
    double residual;            /* max_k |b_k - A x_k| / |b_k| (FP64 A), computed in the mixed modes */
    double asym;                /* max |C - C^T| / max |C| */
    int32_t refine_iters;
    int32_t factor_used;        /* gbem_dtype actually used (after any fallback) */
    int64_t n_near;             /* near pairs j <= i, diagonal included */
    int64_t n_panels;
    /* with opts.profile: per kernel class, summed over the extraction */
    double prof_ms[GBEM_K_COUNT];        /* GPU time between events around the launches */
    int64_t prof_launches[GBEM_K_COUNT];
    double prof_flops[GBEM_K_COUNT];     /* algorithmic floating-point operations */
    double prof_bytes[GBEM_K_COUNT];     /* algorithmic HBM bytes (compulsory reads + writes) */
    int32_t outer_width;        /* tile shapes the factorisation used (see gbem_tuning) */
    int32_t super_panels;
    int32_t graph_used;         /* opts.graph: 1 when the captured segment ran as a graph */
    int32_t graph_instantiated; /* 1: no cached executable matched, the graph was instantiated */
} gbem_report;

/* Tile shapes of the Cholesky factorisation (schedule only: results do not
 * depend on them beyond rounding order).  outer_width: columns per outer
 * panel, 256 or 512.  super_panels: outer panels per trailing update of the
 * 16-bit factors, 1, 2 or 4 (K = super_panels * outer_width).  The library picks
 * them per padded matrix order and factor dtype from a cache written by the
 * project's autotuner (paper_2203_11733_amd/autotune.py, which times every
 * candidate on the GPU): tune_gfx950.json next to the library, or the file
 * named by GBEM_TUNE_FILE, read when the first context is created; without
 * a cache, built-in defaults apply. */
typedef struct {
    int32_t outer_width;
    int32_t super_panels;
} gbem_tuning;
/* Replace the shape cache with the file at path (process-wide; NULL: back to
 * the built-in defaults).  GBEM_EINVAL when the file is missing or malformed
 * (the previous cache stays). */
gbem_status gbem_load_tuning(const char *path);
/* Force shapes for every later factorisation in the process (fields 0: from
 * the cache); t = NULL clears the override.  Used by the autotuner. */
gbem_status gbem_set_tuning_override(const gbem_tuning *t);
/* Where the current shapes come from (a path or "built-in defaults"). */
const char *gbem_tuning_source(void);

/* Version string of the library. */
const char *gbem_version(void);
/* Static text for a status code. */
const char *gbem_status_str(gbem_status s);
/* Message of the last failure on the calling thread ("" if none). */
const char *gbem_last_error(void);
/* Fill *o with the defaults: p = 3, eta = 2, far FP64, factor FP64, tol 1e-6, 30 iterations,
 * profiling off. */
void gbem_default_opts(gbem_opts *o);

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the device
 * memory the serving loop admits jobs into (0 = 90 % of the free memory). */
gbem_status gbem_create(int device, size_t hbm_budget_bytes, gbem_ctx **out);
/* Wait for outstanding jobs, free every resource of the context. */
gbem_status gbem_destroy(gbem_ctx *ctx);

/* Whole extraction, synchronous: host mesh in, host C_out (n_conductors^2
 * doubles, row-major, Farads) out.  rep may be NULL. */
gbem_status gbem_extract(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                         double *C_out, gbem_report *rep);

/* Same with a device-resident mesh (mesh->lo/hi/conductor are device pointers)
 * and a device-resident C_out; work is queued on `stream` and the call returns
 * when C_out is final on that stream. */
gbem_status gbem_extract_device(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                double *C_out_device, void *stream, gbem_report *rep);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * extraction as gbem_extract_device (same kernels, same launches, same
 * results), except that the call allocates nothing: no hipMalloc, hipFree or
 * other allocating routine.  Every intermediate (panel table, near list, A,
 * the scaled FP32 copy, the factor's workspaces, right-hand sides and
 * residuals) is carved from one static device array of 256 MiB per GPU,
 * which the first gbem_create on that GPU sets up and which stays held until
 * the process ends; the events, side stream and pinned readback words of
 * the call are made at that set-up too.  The caller passes the device mesh,
 * the device C_out and the stream as for gbem_extract_device.
 * Limits: padded order <= 5,632 (meshes up to about 5,600 panels with an FP64
 * factor, about 4,000 with a low-precision factor, whose scaled copy and
 * refinement buffers need room too).  A larger mesh, or a near list that
 * does not fit what is left of the array, returns GBEM_ENOMEM with the size in
 * gbem_last_error() before or instead of any result.  opts->profile must be 0
 * (GBEM_EINVAL).  The array keeps the last call's contents; every call
 * re-zeroes what must start at zero.  All calls on one GPU share the array:
 * the library makes them take turns (a per-GPU lock held until the call's
 * last kernel has finished), since overlapping calls would race on it. */
gbem_status gbem_extract_device_noalloc(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                        double *C_out_device, void *stream, gbem_report *rep);

/* Serving loop (continuous batching): submit copies the mesh and returns at
 * once; jobs are admitted as their HBM footprint fits the budget and run
 * concurrently on their own streams. */
gbem_status gbem_submit(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, gbem_job **out);
/* GBEM_OK when finished, GBEM_EBUSY while queued or running, else the job's error. */
gbem_status gbem_poll(gbem_job *job);
/* Block until the job finishes or timeout_s passes (< 0: no limit).  On
 * GBEM_OK writes C_out (host, n_conductors^2, row-major) and *rep (may be NULL). */
gbem_status gbem_wait(gbem_job *job, double timeout_s, double *C_out, gbem_report *rep);
/* Release a finished job (waits for it if it is still running). */
void gbem_job_free(gbem_job *job);
/* Serving statistics (each output may be NULL): jobs finished; the largest
 * sum of admitted footprints (the scheduler's estimates); the largest sum of
 * the device bytes the workers' workspaces really held, taken at the end of
 * each job.  Both peaks stay within the context's HBM budget. */
gbem_status gbem_server_stats(gbem_ctx *ctx, int64_t *jobs_done, size_t *peak_reserved_bytes,
                              size_t *peak_held_bytes);

/* Mesher.  Boxes -> rectangles with a deterministic order (boxes as given;
 * faces -x,+x,-y,+y,-z,+z; lower in-plane axis outer).  Edge rules:
 *   kind 0 (uniform): n = max(1, ceil(L/h - 1e-9)) cells, edges lo + ((hi-lo)*k)/n
 *   kind 1 (graded):  cells h_min, h_min*growth, ... from both ends while the
 *                     cell is <= h_max and the run stays <= L/2; the middle is
 *                     split uniformly into max(1, ceil(rem/h_max - 1e-9)) cells.
 * Rejects boxes with non-positive extent and box surfaces that intersect. */
typedef struct {
    int32_t kind;               /* 0 uniform, 1 edge-graded */
    double h;                   /* uniform cell size */
    double h_min, growth, h_max;
} gbem_mesh_rule;
typedef struct {
    int32_t n_panels;
    double *lo, *hi;            /* library-allocated [3 * n_panels] */
    int32_t *conductor;         /* library-allocated [n_panels] */
} gbem_mesh_buf;
gbem_status gbem_mesh_boxes(const double *box_lo, const double *box_hi, const int32_t *box_cond,
                            int32_t n_boxes, const gbem_mesh_rule *rule, gbem_mesh_buf *out);
/* Free the arrays of a gbem_mesh_buf filled by gbem_mesh_boxes or
 * gbem_mesh_partition. */
void gbem_mesh_buf_free(gbem_mesh_buf *buf);

/* Partition rule of section 3.3 (error estimate of Proposition 2: element
 * area times the field derivative, the derivative taken as falling with the
 * cube of the distance to the main net, eq. "electric_derivative").  For one
 * main net, every box face is split into rectangles I with
 *   |I| <= p4                       where the distance d(I, main net) <= p5,
 *   |I| <= p4 * p3 * (d / p5)^3     beyond,
 * p4 = p1 on faces that face the main net and p1 * p2 on faces turned away
 * from it (field shielding, p2 usually > 1).  Readings where the paper is
 * silent: d is the Euclidean distance from I to the nearest box of the main
 * net; the faces of the main net and of any box enclosing it face it, any
 * other face faces it when some box of the main net reaches beyond the face's
 * plane on its outer side; a rectangle over its bound is halved across its
 * longer side (lower in-plane axis on a tie) at lo + (hi - lo) * 0.5, depth
 * first, lower half first, all in plain FP64.  Output order: boxes as given,
 * faces -x, +x, -y, +y, -z, +z.  Boxes with conductor -1 (a grounded
 * enclosure) are meshed like conductors. */
typedef struct {
    double p1;   /* area bound (length unit^2) near the main net, facing side */
    double p2;   /* >= 1: factor of p1 on faces turned away from the main net */
    double p3;   /* > 0: factor of the far bound */
    double p5;   /* > 0: distance (length unit) where the far bound starts */
} gbem_partition;
/* main_net value for one mesh refined around every conductor: the union of
 * all boxes with a conductor id >= 0 acts as the main net (distance to the
 * nearest of them, faces of any conductor facing), so one mesh and one
 * system serve every column of C and C is symmetric by construction.  This
 * is the reading under which the paper's Table 2 (section 5) prints
 * C12 = C21 at every mesh size. */
#define GBEM_ALL_NETS (-2)
/* Mesh for main net main_net (a conductor id of box_cond, or GBEM_ALL_NETS);
 * arrays as for gbem_mesh_boxes (library-allocated, free with
 * gbem_mesh_buf_free).  GBEM_EINVAL: invalid rule, no box on main_net,
 * intersecting boxes, or a rule that asks for more than 2^29 panels or
 * pieces below 1e-12 of a face. */
gbem_status gbem_mesh_partition(const double *box_lo, const double *box_hi, const int32_t *box_cond,
                                int32_t n_boxes, int32_t main_net, const gbem_partition *rule,
                                gbem_mesh_buf *out);
/* The paper's extraction with per-main-net meshes (section 3.2: the main net
 * at potential 1, all other boundaries at 0, C_1 = Q_1 and C_n = Q_n): for
 * each conductor k = 0 .. n_conductors-1, mesh with gbem_mesh_partition(k),
 * extract, and keep column k of that extraction's Maxwell matrix (the charges
 * on every net with net k at potential 1).  The n_conductors extractions are
 * independent and run through the serving loop (several at once on their own
 * streams, queued behind jobs already submitted); the same HBM budget
 * applies.  C_out: host, n_conductors^2,
 * row-major, C_out[n * n_conductors + k] = charge on net n per volt on net k.
 * panels_out (optional, host, n_conductors): panel count of mesh k.  rep
 * (optional): GPU times and panel counts summed over the meshes, largest
 * residual and refinement count, asym of the assembled C (it measures how
 * much the per-net meshes disagree). */
gbem_status gbem_extract_partitioned(gbem_ctx *ctx, const double *box_lo, const double *box_hi,
                                     const int32_t *box_cond, int32_t n_boxes, int32_t n_conductors,
                                     double eps_r, double length_unit_m, const gbem_partition *rule,
                                     const gbem_opts *opts, double *C_out, int32_t *panels_out,
                                     gbem_report *rep);

/* ---- several dielectrics (section 4) ---------------------------------------
 * In each dielectric region the potential solves Laplace's equation; on the
 * boundary of a region, Green's identity ties the potential u and its normal
 * derivative q (along the region's outward normal) through the single-layer
 * integrals G and the double-layer integrals Q of section 4.2.  With u and q
 * constant per panel the Galerkin form has one equation per (region, panel
 * on its boundary) (section 4.1):
 *     1/2 |I_i| u_i + sum_k Q_ik u_k = sum_j G_ij q_j.
 * Unknowns: q on conductor and Dirichlet panels, u on Neumann panels, u and
 * q on interface panels (the neighbour region's q follows from
 * eps_a q_a = -eps_b q_b, section 2.1); u = 1 on the main net, 0 on the other
 * nets and on Dirichlet panels. */
typedef enum {
    GBEM_PANEL_CONDUCTOR = 0,   /* on net `conductor` (u known), one region side */
    GBEM_PANEL_DIRICHLET = 1,   /* grounded outer boundary (u = 0), one region side */
    GBEM_PANEL_NEUMANN = 2,     /* outer boundary with du/dn = 0, one region side */
    GBEM_PANEL_INTERFACE = 3    /* between two different regions */
} gbem_panel_kind;

/* A multi-dielectric mesh.  Panels are axis-aligned rectangles as in
 * gbem_mesh (lo, hi: [3 * n_panels]); region_plus[i] / region_minus[i] name
 * the region on the + / - side of panel i along its normal axis, in
 * [0, n_regions), or -1 where there is none (inside a conductor, outside the
 * domain); eps_r[n_regions] > 0.  conductor[i] is read for conductor panels
 * only (in [0, n_conductors), every net with at least one panel). */
typedef struct {
    int32_t n_panels;
    int32_t n_conductors;       /* 1..64 */
    int32_t n_regions;
    const double *lo;
    const double *hi;
    const int32_t *kind;        /* gbem_panel_kind per panel */
    const int32_t *conductor;
    const int32_t *region_plus;
    const int32_t *region_minus;
    const double *eps_r;
    double length_unit_m;       /* metres per coordinate unit, > 0 */
} gbem_dmesh;

/* Maxwell capacitance matrix of a multi-dielectric mesh (host arrays in and
 * out): C_out[n * n_conductors + k] = charge on net n (eps0 * sum over its
 * panels of eps_r q |I|) per volt on net k.  The single-layer entries use
 * opts->far_order and opts->near_eta in FP64 (far_dtype and factor_dtype are
 * not read); the double-layer entries split near and far at eta = 2 whatever
 * near_eta is (as gbem_assemble_double_layer with near_eta = 2); the system is not symmetric, so it is solved through its normal
 * equations M^T M x = M^T b by the FP64 Cholesky factorisation and refined
 * against the residual of M itself until max_k |b_k - M x_k| / |b_k| <=
 * 1e-13 (at most six sweeps; rep->residual reports it).  GBEM_EINVAL on an
 * inconsistent mesh (a panel kind with the wrong number of regions, a
 * conductor id out of range, a net without panels), GBEM_ENOTPD when the
 * normal equations are singular. */
gbem_status gbem_extract_dielectric(gbem_ctx *ctx, const gbem_dmesh *mesh, const gbem_opts *opts, double *C_out,
                                    gbem_report *rep);

/* A layered dielectric layout: a box domain cut along z into n_layers
 * dielectric layers (z_layer[0] = domain_lo[2] < ... < z_layer[n_layers] =
 * domain_hi[2], permittivity eps_r[a] in layer a), conductor boxes each
 * strictly inside one layer (net box_net[b] in [0, n_conductors)), the
 * bottom, top and side faces of the domain GBEM_PANEL_DIRICHLET or
 * GBEM_PANEL_NEUMANN (the paper's experiment with several dielectrics:
 * grounded top and bottom, Neumann elsewhere). Host arrays. */
typedef struct {
    int32_t n_boxes;
    const double *box_lo;       /* [3 * n_boxes] */
    const double *box_hi;
    const int32_t *box_net;     /* [n_boxes] */
    int32_t n_conductors;
    double domain_lo[3], domain_hi[3];
    int32_t n_layers;
    const double *z_layer;      /* [n_layers + 1] */
    const double *eps_r;        /* [n_layers] */
    int32_t bottom_kind, top_kind, side_kind;
    double length_unit_m;
} gbem_dlayout;

/* Panels of a multi-dielectric mesh (malloc'ed; free with gbem_dmesh_buf_free). */
typedef struct {
    int32_t n_panels;
    double *lo, *hi;            /* [3 * n_panels] */
    int32_t *kind, *conductor, *region_plus, *region_minus;
} gbem_dmesh_buf;
void gbem_dmesh_buf_free(gbem_dmesh_buf *buf);

/* Mesh of a layered layout for main net main_net by the paper's rules:
 * conductor faces and the domain boundary by the section 3.3 rule (as
 * gbem_mesh_partition: |I| <= p4 within p5 of the main net, p4 p3 (d/p5)^3
 * beyond, p4 = p1 on faces that face the main net and on the domain
 * boundary, p1 p2 on the others), the interfaces between layers by the
 * section 4.1 rule, |I| <= p1 within p5 and p1 p3 (d/p5)^2 beyond (the
 * printed length l read as p5, as in section 3.3). Panel order: conductor
 * boxes (faces -x, +x, -y, +y, -z, +z), bottom, top, side walls layer by
 * layer (-x, +x, -y, +y), interfaces bottom to top; each face by bisection
 * of its longer side, lower half first. */
gbem_status gbem_mesh_dielectric_partition(const gbem_dlayout *layout, int32_t main_net, const gbem_partition *rule,
                                           gbem_dmesh_buf *out);

/* Capacitance matrix of a layered layout with one mesh per main net (the
 * paper's method for several dielectrics, section 4 with section 3.3):
 * column k of C_out (row-major, C_out[n * n_conductors + k]) from the mesh of
 * main net k by gbem_mesh_dielectric_partition, extracted by
 * gbem_extract_dielectric; the n_conductors extractions run on up to four
 * lanes at once (a workspace and a stream each, kept by the context), each
 * column from one lane's kernels, so C equals that of the extractions run one
 * by one. panels_out (optional, host, n_conductors): panel count of mesh k.
 * rep (optional): times and panels summed over the meshes, largest residual,
 * asym of the assembled C. */
gbem_status gbem_extract_dielectric_partitioned(gbem_ctx *ctx, const gbem_dlayout *layout, const gbem_partition *rule,
                                                const gbem_opts *opts, double *C_out, int32_t *panels_out,
                                                gbem_report *rep);

/* ---- stage entry points (same kernels as gbem_extract; for parity tests) ---- */

/* Near-pair list of the mesh (host arrays in/out): row_ptr[n+1], col[nnz] with
 * j <= i ascending per row.  Call with col == NULL to get *nnz only. */
gbem_status gbem_near_list(gbem_ctx *ctx, const gbem_mesh *mesh, double near_eta,
                           int64_t *row_ptr, int32_t *col, int64_t col_capacity, int64_t *nnz);
/* Assemble A and copy it to host A_out (n x n, row-major; A is symmetric). */
gbem_status gbem_assemble(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts, double *A_out);
/* Assemble A with the same launches as gbem_extract and return m sampled
 * entries out[k] = A[ii[k], jj[k]] (host arrays). */
gbem_status gbem_assemble_sample(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                 int64_t m, const int32_t *ii, const int32_t *jj, double *out);
/* Input of a low-precision factorisation (the Cholesky factorisation of
 * section 3.2, applied to the Jacobi-scaled system): F = S A S in FP32 with
 * S = diag(A)^(-1/2), which the far and near assembly passes write beside A.
 * Assembles with the same launches as gbem_extract and returns m sampled
 * entries out[k] = F[ii[k], jj[k]] (host arrays; F holds the lower triangle,
 * so 0 <= jj[k] <= ii[k] < n_panels).  GBEM_EINVAL when opts->factor_dtype
 * is GBEM_F64 (no scaled copy is made) or an index is out of range. */
gbem_status gbem_assemble_scaled_sample(gbem_ctx *ctx, const gbem_mesh *mesh, const gbem_opts *opts,
                                        int64_t m, const int32_t *ii, const int32_t *jj, float *out);
/* Double-layer integrals of section 4.2 (host arrays): Q_out[i * n + k] =
 * Int_{I_i} Int_{I_k} <x - y, n_k> / (4 pi |x - y|^3) with n_k the unit
 * vector along + the normal axis of panel k; 0 for coplanar pairs.  Pairs of
 * the near list of near_eta (as in gbem_opts) are integrated in closed form
 * over both panels; the others take the closed-form integral over I_k (its
 * solid angle at x over 4 pi) under n x n Gauss points on I_i, n from 6 at
 * the near threshold down to 2 at 40 diameters (within about 1e-13 |I_i|). */
gbem_status gbem_assemble_double_layer(gbem_ctx *ctx, int32_t n_panels, const double *lo, const double *hi,
                                       double near_eta, double *Q_out);
/* In-place Cholesky A = L L^T of a device matrix (column-major, lower
 * triangle referenced, leading dimension lda >= n).  dtype GBEM_F64 takes
 * double*, GBEM_F32/F16/BF16 take float* (F16/BF16 = FP32 storage with 16-bit
 * MFMA trailing updates).  On GBEM_ENOTPD *info = 1 + index of the first bad pivot. */
gbem_status gbem_cholesky_device(gbem_ctx *ctx, int32_t n, int32_t dtype, void *A, int64_t lda,
                                 int32_t *info, void *stream);
/* Solve L L^T X = B in place on device (B: n x nrhs, column-major, ldb),
 * L from gbem_cholesky_device with the same dtype. */
gbem_status gbem_cholesky_solve_device(gbem_ctx *ctx, int32_t n, int32_t dtype, const void *L,
                                       int64_t lda, int32_t nrhs, void *B, int64_t ldb, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GBEM_H */
