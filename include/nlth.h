/*
 * nlth -- MI355X-native ensemble solver for nonlinear time-history analysis of
 * 3D seismic ground response with a multi-spring hysteretic law.
 *
 * Method: Ichimura, Fujita, Ito, Hori, Lalith, "Accelerating Nonlinear
 * Time-History Analysis with Complex Constitutive Laws via Heterogeneous
 * Memory Management" (arXiv 2604.02755).  Each time step solves the
 * Newmark-beta incremental system of Section 2.1, Eq. 1 by preconditioned CG
 * with an element-by-element (matrix-free) operator (Section 2.2, Algorithm 4),
 * then updates the multi-spring law at the four integration points of every
 * quadratic tetrahedron (Section 2.1, Eq. 2), paging the per-spring history
 * between pinned host memory and HBM when it does not fit (Section 2.2,
 * Algorithm 3).
 *
 * Conventions for every call:
 *  - SI units, z up; the free surface is the top, absorbing faces are given
 *    explicitly (base faces also carry the incident wave).
 *  - Return value: NLTH_OK (0) or a negative NLTH_E* code; nlth_last_error()
 *    then holds a message.
 *  - Input arrays are owned by the caller and copied (host pointers) during
 *    the call unless stated otherwise.
 *  - Output buffers are owned by the caller (host pointers).
 *  - Handles are owned by the library and released by their *_destroy call.
 *  - One context per device; calls on one context are serialised internally.
 */
#ifndef NLTH_H
#define NLTH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NLTH_VERSION 10000 /* 1.0.0 */

/* status codes */
#define NLTH_OK 0
#define NLTH_EINVAL -1          /* invalid argument, mesh or problem */
#define NLTH_EDEVICE -2         /* HIP runtime failure, or a host-only context */
#define NLTH_ENOMEM_DEVICE -3   /* does not fit the HBM budget even with paging */
#define NLTH_ENOMEM_HOST -4     /* pinned host budget exceeded */
#define NLTH_ENOCONV -5         /* a member's CG hit cg_maxit */
#define NLTH_EBUSY -6           /* request can never fit the budgets / handle in use */
#define NLTH_ECANCELED -7       /* request was cancelled */
#define NLTH_ETIMEDOUT -8       /* nlth_wait timed out */
#define NLTH_ENOTFOUND -9       /* unknown ticket */

/* damping modes: Rayleigh damping from the law's h (Section 2.1), constant h0, none */
#define NLTH_DAMPING_LAW 0
#define NLTH_DAMPING_CONST 1
#define NLTH_DAMPING_NONE 2

/* precision: all-FP64 block-Jacobi PCG, or FP64 flexible CG whose
 * preconditioner is an FP32 block-Jacobi PCG (Section 2.3: only the
 * preconditioner runs in single precision) */
#define NLTH_FP64 0
#define NLTH_MIXED 1

/* storage of D for the inner FP32 operator of NLTH_MIXED: bfloat16 (half the
 * bytes; the outer FP64 iteration keeps the solution at FP64 tolerance) or FP32 */
#define NLTH_INNER_BF16 0
#define NLTH_INNER_FP32 1
#define NLTH_INNER_BF16_MEAN 2

/* operator selector for nlth_apply_operator */
#define NLTH_OP_A 0 /* 4/dt^2 M + 2/dt C + K (Eq. 1 left-hand side) */
#define NLTH_OP_K 1 /* K */
#define NLTH_OP_M 2 /* M */
#define NLTH_OP_DIAG 3 /* the 3x3 diagonal blocks of A (the block-Jacobi preconditioner's) */

#define NLTH_DEVICE_NONE (-1) /* host-only context: validation and mesh analysis */

typedef struct nlth_ctx nlth_ctx;
typedef struct nlth_mesh nlth_mesh;
typedef struct nlth_ens nlth_ens;

typedef struct {
    int64_t hbm_budget;   /* device bytes the library may allocate; 0 = 90 % of free */
    int64_t host_budget;  /* host bytes the library may hold: pinned law state of paged
                             ensembles, and the serving loop's input copies of queued
                             requests and of its batches; 0 = 64 GiB */
    void* stream;         /* optional hipStream_t for compute (e.g. torch's); NULL = own */
    int32_t log_level;    /* 0 silent, 1 per solve, 2 per step */
    int32_t max_batch;    /* serving: most members per batch (0 = 64); a batch is sized,
                             in powers of two, for the members waiting when it forms */
    int32_t paging_sets;  /* an ensemble whose law state does not fit the device budget:
                             0 or 2 = two member sets, the solve of one running while the
                             other's law state streams over the host link (the chunk
                             pipeline of Section 2.2, Alg. 3, hides the transfers behind
                             the law kernels only); 1 = one set (its law phase waits for
                             the link);
                             other values: NLTH_EINVAL */
} nlth_ctx_opts;

/* Create a context on HIP device `device` (or NLTH_DEVICE_NONE).  `opts` may
 * be NULL.  Errors: NLTH_EDEVICE if the device cannot be used. */
int nlth_ctx_create(int device, const nlth_ctx_opts* opts, nlth_ctx** out);
/* Destroy; fails with NLTH_EBUSY while requests or meshes are alive. */
int nlth_ctx_destroy(nlth_ctx* ctx);
/* Message of the last error on this context (context-owned, NUL-terminated,
 * valid until the next call on the context).  ctx may be NULL (global). */
const char* nlth_last_error(const nlth_ctx* ctx);
int nlth_version(void);

/*
 * Mesh: quadratic (10-node) tetrahedra, Section 2.1.  Node order per tet is
 * VTK's: vertices v0..v3 then the midpoints of edges 01, 12, 20, 03, 13, 23.
 * Tets must be straight-sided (mid-nodes at edge midpoints) with a positive
 * Jacobian.  Boundary faces are 6-node triangles (3 vertices, then midpoints
 * of ab, bc, ca); kind 0 = base (absorbing dashpot + incident wave input),
 * kind 1 = side (absorbing dashpot).  Receivers are node ids whose velocity is
 * recorded every step.  All arrays are copied.
 * Errors: NLTH_EINVAL naming the first offending element/face/node.
 */
typedef struct {
    int32_t n_nodes;
    const double* xyz;         /* [n_nodes*3] */
    int32_t n_tets;
    const int32_t* tet10;      /* [n_tets*10] */
    const int32_t* layer;      /* [n_tets] layer id, 0 <= id < n_layers of the problem */
    int32_t n_bfaces;
    const int32_t* bface6;     /* [n_bfaces*6] */
    const uint8_t* bface_kind; /* [n_bfaces] */
    int32_t n_recv;
    const int32_t* recv;       /* [n_recv] */
} nlth_mesh_desc;

int nlth_mesh_create(nlth_ctx* ctx, const nlth_mesh_desc* d, nlth_mesh** out);
int nlth_mesh_destroy(nlth_mesh* mesh);

/* Mesh analysis results (host logic, available on a host-only context).
 * elem_order (optional, [n_tets]) receives the tets grouped by colour (input
 * tet ids); color_offsets (optional, [n_colors+1]) the start of each colour
 * in that list.  Tets of one colour share no node. */
typedef struct {
    int32_t n_nodes, n_tets, n_colors, n_bnodes;
    double volume;
    int32_t n_clusters;        /* element clusters of the cluster path */
    int64_t cluster_rows;      /* node rows of all clusters */
} nlth_mesh_info;
int nlth_mesh_query(const nlth_mesh* mesh, nlth_mesh_info* info, int32_t* elem_order,
                    int32_t* color_offsets);

/*
 * Problem: an ensemble of members sharing one mesh (Section 3: ensembles of
 * input waves and ground properties).  Per member and layer: density, S-wave
 * velocity, Poisson ratio and the springs' reference strain (gamma_ref, where
 * the secant modulus is G0/2).  Per layer: h_max (maximum damping of the
 * Ramberg-Osgood/Masing loop) and whether the layer's springs are nonlinear.
 * Spring table: unit-direction rows n_k (Voigt xx,yy,zz,xy,yz,zx with
 * engineering shear; gamma_k = n_k . eps) and weights c_k; the point tangent
 * is D = K_b m m^T + sum_k c_k G_t,k n_k n_k^T.
 * input_acc[(m*n_steps + n)*3 + c] is the incident base acceleration of
 * member m at t = (n+1) dt (zero at t = 0).
 * Rayleigh damping (Section 2.1): alpha = a*h, beta = b*h per element with
 * (a, b) the least-squares fit of alpha/(4 pi f) + pi beta f to 1 over
 * [f_lo, f_hi]; h = the law's element damping (LAW), h0 (CONST) or 0 (NONE).
 * CG stops when ||r||_2 <= cg_tol ||b||_2 per member; the inner FP32 solve of
 * NLTH_MIXED stops at inner_tol relative or inner_maxit iterations.
 */
typedef struct {
    int32_t n_members;
    int32_t n_layers;
    const double* rho;         /* [n_members*n_layers] */
    const double* vs;
    const double* nu;
    const double* gamma_ref;
    const double* h_max;       /* [n_layers] */
    const int32_t* nonlinear;  /* [n_layers] */
    int32_t n_springs;
    const double* dirs;        /* [n_springs*6] */
    const double* weights;     /* [n_springs] */
    int32_t damping_mode;
    double h0, f_lo, f_hi;
    double dt;
    int32_t n_steps;
    const double* input_acc;   /* [n_members*n_steps*3] */
    double cg_tol;
    int32_t cg_maxit;
    int32_t precision;         /* NLTH_FP64 or NLTH_MIXED */
    double inner_tol;
    int32_t inner_maxit;
    int32_t inner_dtype;       /* storage of D for the inner (FP32) operator: NLTH_INNER_BF16
                                  (default; bfloat16 per point), NLTH_INNER_FP32 (FP32 per
                                  point) or NLTH_INNER_BF16_MEAN (bfloat16, one D per element:
                                  the mean over its four points; the preconditioner then
                                  applies a slightly different operator, which the FP64 outer
                                  iteration corrects) */
    int32_t masing_depth;      /* 0 or 1: the law's three Masing rules (each spring keeps its
                                  last reversal point; a branch runs until it meets the
                                  skeleton, Section 2.1 with the extended Masing rules of its
                                  cited law).  K in 2..8: each spring also keeps the origins of
                                  up to K-1 earlier branches, so an inner loop closes when the
                                  strain passes the last reversal point and the path goes on
                                  along the branch it left (the fourth rule; with the memory
                                  full the oldest point is dropped).  Law state per spring and
                                  point: 36 B, plus 16 B per remembered point beyond the
                                  first.  Other values: NLTH_EINVAL. */
} nlth_problem;

/* Result buffers (caller-owned host memory; NULL fields are skipped).
 * vel[((m*n_steps + n)*n_recv + r)*3 + c]: receiver velocity after step n+1.
 * iters[(m*n_steps + n)*2 + {0,1}]: outer and total inner CG iterations.
 * member_status[m]: NLTH_OK or NLTH_ENOCONV (results valid up to the failing step).
 * vmax[m*n_recv + r]: maximum velocity norm over the run at each receiver. */
typedef struct {
    double* vel;
    int32_t* iters;
    int32_t* member_status;
    double* vmax;
} nlth_result;

/* Synchronous whole-run solve.  Returns NLTH_ENOCONV if any member failed,
 * NLTH_ENOMEM_DEVICE / NLTH_ENOMEM_HOST if it cannot fit even with paging. */
int nlth_solve(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, nlth_result* res);

/* Staged form of nlth_solve: create uploads the problem and allocates all
 * device state (and pinned host state when paging); step advances every
 * member by n_steps (synchronous); read copies the results recorded so far;
 * stats reports phase timers.  The problem's arrays are copied by create.
 * When the whole ensemble does not fit the device budget and the context
 * allows two member sets, create splits the members in two halves (the first
 * ceil(n/2), then the rest), each paging its law state; step alternates them
 * (results, numbering and iteration counts are those of the members run
 * alone: the sets share no arithmetic). */
int nlth_ens_create(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, nlth_ens** out);
int nlth_ens_step(nlth_ens* ens, int32_t n_steps);
int nlth_ens_read(nlth_ens* ens, nlth_result* res);
int nlth_ens_destroy(nlth_ens* ens);

/* Phase timers (HIP events, milliseconds, accumulated since create or the
 * last reset) and counters.  Event timing of individual kernels is on only
 * when `profile` was set with nlth_ens_set_profile (it adds host overhead). */
typedef struct {
    int32_t steps_done;
    int32_t paged;             /* law state streamed from pinned host memory */
    int64_t outer_iters, inner_iters;
    double ms_total;           /* wall time inside nlth_ens_step */
    double ms_ebe64, ms_ebe32, ms_vec, ms_law, ms_other;
    int64_t n_ebe64, n_ebe32, n_law;     /* timed launches */
    int64_t elems_ebe64, elems_ebe32;    /* element-member pairs processed by those launches */
    int64_t h2d_bytes, d2h_bytes;
    double ms_copy;            /* copy-stream busy time while paging */
    int32_t n_members, members_padded, n_colors;
    int64_t device_bytes, host_bytes;
    double ms_gather32;        /* node gather of the inner operator's element outputs or cluster rows */
    int64_t n_gather32;
    double cheb_lo_min;        /* Chebyshev inner bounds of the last step: smallest lower bound and */
    double cheb_hi_max;        /* largest upper bound over the members (0 without Chebyshev) */
    double ms_tail32;          /* operator on the compact rows of the last active members
                                  (element kernel, node gather and dashpot): the inner FP32 one,
                                  or with NLTH_FP64 the PCG's; the mixed path's outer FP64
                                  operator on those rows counts in ms_ebe64 */
    int64_t n_tail32;
    int64_t elems_tail32;      /* element-member pairs of those launches (listed members only) */
    int32_t member_sets;       /* 2: a paged ensemble run as two member sets; 1 otherwise */
} nlth_stats;
int nlth_ens_stats(const nlth_ens* ens, nlth_stats* st);

/* Launch-shape knobs of an ensemble (chosen by the package's autotuner):
 * threads per block of the element-by-element launches (64, 128 or 256), CG
 * iterations between host convergence checks (1..64), and whether those
 * iteration chunks are captured once into a hipGraph and replayed (0/1).
 * It also sets the inner-solve policy of NLTH_MIXED (inner_tol, inner_maxit):
 * a tiny inner_tol with a small inner_maxit gives a fixed number of inner
 * iterations per outer iteration, which keeps every member's lanes busy.
 * A field of 0 (or -1 for use_graph) keeps the current value.  The launch
 * shapes do not change results (converged members are frozen on the device);
 * the inner policy changes the iteration path only within the outer FP64
 * tolerance.  scatter picks how element forces reach the nodes (the default
 * depends on the member slots): per-element outputs summed per node in a
 * fixed order; clusters of consecutive elements summed in LDS in a fixed
 * order, then per node; or one launch per element colour adding into the
 * nodal vector.
 * Out-of-range fields (ebe_block not 0/64/128/256, check_every outside
 * 0..64, inner_maxit outside 0..100000, inner_tol outside [0, 1), cluster_blocks
 * not 0/2/3/4, scatter outside -1..2 or not available for this ensemble,
 * inner_method outside -1..1, Chebyshev with a degree above 64, zero_copy outside
 * -1..1 or 1 for an ensemble whose state is resident, tail_members not -1/0/16/32
 * or above 0 for an ensemble outside 64..256 slots or a mixed one without the
 * element-mean inner D, predictor outside -1..2)
 * give NLTH_EINVAL and
 * change nothing.  Not to be called while the ensemble
 * is stepping on another thread. */
typedef struct {
    int32_t ebe_block;
    int32_t check_every;
    int32_t use_graph;
    int32_t inner_maxit;
    double inner_tol;
    int32_t scatter;           /* -1 keep; 0 element outputs + node gather (fewer than 64 member
                                  slots); 1 one launch per colour; 2 element clusters + node gather
                                  (64..256 slots, a multiple of 64) */
    int32_t cluster_blocks;    /* 0 keep; 2, 3 or 4 co-resident FP32 cluster blocks per CU (default 3) */
    int32_t inner_method;      /* -1 keep; 0 inner CG (default); 1 Chebyshev iteration of degree
                                  inner_maxit (at most 64, inner_tol unused) on the block-Jacobi
                                  preconditioned operator, with each member's spectrum bounds taken
                                  from the Lanczos matrix of the step's first inner CG solve */
    int32_t zero_copy;         /* -1 keep; 0 paged law state moved by the pipelined chunk copies
                                  (default); 1 the law kernel reads and writes the pinned host state
                                  over the host link itself (an ablation of the pipeline; only for an
                                  ensemble whose state is paged) */
    int32_t tail_members;      /* -1 keep; 0 off; 16 or 32: once at most this many members are
                                  still iterating, their solve moves to compact copies of their
                                  rows (16 or 32 lanes instead of all member slots): the plain PCG
                                  of NLTH_FP64, or with NLTH_MIXED (element-mean inner D, inner CG)
                                  the inner CG and then the outer iteration.  Results equal the
                                  full path's to rounding order.  64..256 slots (default 32 there,
                                  0 elsewhere).  The copies take 32 lanes of 172 B per element and
                                  84 B per node for the inner solve, and of 920 B per element and
                                  168 B per node for the FP64 rows, allocated at first use; if that
                                  fails the path stays off for the ensemble */
    int32_t predictor;         /* -1 keep; CG initial guess of a step from the increments of the
                                  previous steps (their history from rest is zero): 0 the last
                                  increment (default), 1 its linear extrapolation 2 du^{n-1} -
                                  du^{n-2}, 2 the quadratic one 3 du^{n-1} - 3 du^{n-2} + du^{n-3}.
                                  Changes the iteration path only, within the CG tolerance */
} nlth_tuning;
int nlth_ens_set_tuning(nlth_ens* ens, const nlth_tuning* t);
int nlth_ens_set_profile(nlth_ens* ens, int32_t profile);
int nlth_ens_reset_stats(nlth_ens* ens);

/* Continuous-batching request loop.  submit admits the request (queued until
 * slots and HBM free up); the result buffers must stay valid until poll/wait
 * reports completion.  Batches take the CG initial guess from the quadratic
 * extrapolation of the increments (tuning predictor 2), which changes a
 * member's iteration path only, within its CG tolerance.  The request's input copy is charged to the host budget
 * from submission until its members take slots, and each batch's copy of its
 * members' inputs while the batch lives.  NLTH_EBUSY if the request can never
 * fit the budgets, or if the host budget cannot hold its input copy now
 * (submit again later).  A request whose batch cannot be made while nothing
 * else runs ends with NLTH_ENOMEM_DEVICE or NLTH_ENOMEM_HOST. */
int nlth_submit(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, nlth_result* res,
                uint64_t* ticket);
int nlth_poll(nlth_ctx* ctx, uint64_t ticket, int32_t* done);
/* returns the request's final status, or NLTH_ETIMEDOUT */
int nlth_wait(nlth_ctx* ctx, uint64_t ticket, double timeout_s);
int nlth_cancel(nlth_ctx* ctx, uint64_t ticket);
/* Forget a finished or cancelled request (its ticket becomes unknown); the
 * context keeps every request's bookkeeping until then.  NLTH_EBUSY while it
 * is queued or running, NLTH_ENOTFOUND for an unknown ticket. */
int nlth_release(nlth_ctx* ctx, uint64_t ticket);

/* Velocity response spectra of ground-velocity records (Section 3 compares
 * the computed surface waveforms through velocity response spectra with
 * damping ratio h = 0.05), on the device.  vel: [n_series][n_steps] samples
 * v_1..v_N at t_n = n dt (v_0 = 0), e.g. receiver components from
 * nlth_result.vel; the velocity is taken linear between samples, so the
 * ground acceleration is constant on each step.  For each period T (> 0,
 * seconds) the oscillator x'' + 2 h w x' + w^2 x = -a_g, w = 2 pi / T, starts
 * at rest and is advanced exactly step by step; out: [n_series][n_periods],
 * kind NLTH_SPEC_VELOCITY max_n |x'_n| (relative velocity) or
 * NLTH_SPEC_PSEUDO_VELOCITY w max_n |x_n|.  Host pointers, caller-owned,
 * read or written during the call (synchronous).  NLTH_EINVAL for NULL
 * pointers, empty sizes, dt <= 0, h outside [0, 1), a period <= 0 or an
 * unknown kind. */
#define NLTH_SPEC_VELOCITY 0
#define NLTH_SPEC_PSEUDO_VELOCITY 1
int nlth_response_spectra(nlth_ctx* ctx, const double* vel, int32_t n_series, int32_t n_steps, double dt,
                          const double* periods, int32_t n_periods, double h, int32_t kind, double* out);

/* Diagnostic: one element-by-element operator application y = Op x for
 * member 0 of `prob` (Eq. 1 left-hand side with K from the given D and C from
 * the given h), on the device, in FP64 or (precision = NLTH_MIXED) the inner
 * FP32 operator with D stored as prob->inner_dtype says.  NLTH_OP_DIAG applies
 * the 3x3 diagonal blocks of A that the block-Jacobi preconditioner inverts:
 * from D per point in FP64, or, for NLTH_MIXED with NLTH_INNER_BF16_MEAN, those
 * of the inner operator (one bfloat16 D per element).  D_ip:
 * [n_tets*4*21] upper triangle of D row by row per integration point (input
 * tet order); h: [n_tets] element damping (NULL = 0); x, y: [3*n_nodes]. */
int nlth_apply_operator(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, int32_t which,
                        int32_t precision, const double* D_ip, const double* h, const double* x,
                        double* y);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * nlth_apply_operator's FP64 application y = Op x for member 0 of `prob`, on
 * caller-owned DEVICE buffers, with no allocation.  D_ip [n_tets*4*21] (input
 * tet order, upper triangle of D row by row per point), h [n_tets] (NULL =
 * 0), x and y [3*n_nodes] (input node order).  Every intermediate lives in a
 * library-held device array of 64 MiB per device (reserved for the life of
 * the process), enough for meshes up to about 67,000 tets; larger meshes give
 * NLTH_EINVAL, as do more than 32 layers.  The work is queued on the
 * context's compute stream and the call returns without waiting: y is ready
 * when that stream has drained.  Calls on one context are ordered by its
 * stream; calls through different contexts (streams) of one device share the
 * array and race when they overlap.  Same kernels, same results as
 * nlth_apply_operator with precision NLTH_FP64. */
int nlth_apply_operator_noalloc(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, int32_t which,
                                const double* D_ip, const double* h, const double* x, double* y);

#ifdef __cplusplus
}
#endif
#endif
