/*
 * Plain FP64 CPU oracle for the nonlinear time-history method of
 * Ichimura, Fujita, Ito, Hori, Lalith, "Accelerating Nonlinear Time-History
 * Analysis with Complex Constitutive Laws via Heterogeneous Memory
 * Management" (arXiv 2604.02755).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the reference the HIP path is
 * checked against; it shares no code with that path.  Only the tests, the
 * package smoke check and the benchmark's CPU-baseline leg may load it.
 *
 * Structure follows the paper's all-CPU baseline (Section 2.2, Algorithm 1):
 * each step assembles the 3x3-block CRS matrices from the current D, solves
 * Eq. 1 by 3x3 block-Jacobi preconditioned CG, then runs the multi-spring law
 * at every integration point (Section 2.1, Eq. 2).  Everything is double
 * precision.  One member (one ground model + one input wave) per call.
 */
#ifndef NLTH_ORACLE_H
#define NLTH_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n_nodes;
    const double* xyz;               /* [n_nodes*3] */
    int n_tets;
    const int* tet10;                /* [n_tets*10], VTK quadratic-tetra order */
    const int* layer;                /* [n_tets] */
    int n_bfaces;
    const int* bface6;               /* [n_bfaces*6] 3 vertices, then mids of ab, bc, ca */
    const unsigned char* bface_kind; /* 0 base (dashpot + incident wave), 1 side (dashpot) */
    int n_recv;
    const int* recv;                 /* receiver nodes */
    const int* alias;                /* optional [n_nodes]: node whose DOFs this node uses
                                        (periodic ties); NULL = identity */
} or_mesh;

typedef struct {
    int n_layers;
    const double* rho;       /* [n_layers] */
    const double* vs;
    const double* nu;
    const double* gamma_ref;
    const double* h_max;
    const int* nonlinear;
    int n_springs;
    const double* dirs;      /* [n_springs*6] Voigt, engineering shear */
    const double* weights;   /* [n_springs] */
    int damping_mode;        /* 0 law, 1 constant h0, 2 none */
    double h0, f_lo, f_hi;
    double dt;
    int n_steps;
    const double* input_acc; /* [n_steps*3], incident base acceleration at t = (n+1) dt */
    double cg_tol;
    int cg_maxit;
    const double* v0;        /* optional [3*n_nodes] initial velocity (NULL = at rest) */
    /* operator-application mode (kernel parity): when apply_which >= 0 the
     * run stops after assembly and writes y = Op x, Op = 0: 4/dt^2 M + 2/dt C + K
     * (with C from apply_h and the dashpots), 1: K, 2: M; K from apply_D */
    int apply_which;
    const double* apply_D;   /* [n_tets*4*21] upper triangle of D per point */
    const double* apply_h;   /* [n_tets] element damping (NULL = 0) */
    const double* apply_x;   /* [3*n_nodes] */
    double* apply_y;         /* [3*n_nodes] */
    int masing_depth;        /* reversal points a spring remembers: 0 or 1 the three-rule law,
                                K > 1 also closes inner loops up to K - 1 deep */
} or_problem;

typedef struct {
    double* vel;       /* [n_steps*n_recv*3] receiver velocity (required) */
    int* iters;        /* [n_steps] CG iterations (optional) */
    double* du_hist;   /* [n_steps*3*n_nodes] displacement increments (optional) */
    double* u_final;   /* [3*n_nodes] (optional) */
    double* v_final;   /* [3*n_nodes] (optional) */
    double* D_final;   /* [n_tets*4*21] upper-triangle row-major D per IP (optional) */
    double* h_final;   /* [n_tets] element damping (optional) */
    double* theta_final; /* [n_tets*4*n_springs*W] gp,gr,tr,gm,dir,skel, then for depth K > 1
                            the count and K - 1 older (gr, tr); W = or_spring_words(K) (optional) */
    double* vmax;      /* [n_recv] largest velocity norm over the run (optional) */
    long law_events[4]; /* over the run: reversals on the skeleton, reversals on a
                           Masing branch, rejoins of the skeleton, inner loops closed */
    double setup_seconds; /* wall time before the first step (pattern, mass, faces) */
    int steps_done;
} or_result;

/* Error codes. */
#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOCONV -5
#define OR_ENOMEM -10

int or_run(const or_mesh* mesh, const or_problem* prob, or_result* res);
const char* or_last_error(void);

/* ---- building blocks exposed for the pins ---- */
int or_tet_geometry(const double* X4x3, double* gL4x3, double* vol);
void or_element_matrices(const double* X4x3, const double* D4x36, double rho,
                         double* Ke900, double* Me900);
void or_face_matrix(const double* X3x3, double* M36, double* normal3, double* area);
void or_rayleigh(double f_lo, double f_hi, double* a_hat, double* b_hat);
double or_ro_inverse(double e, double beta);
/* one spring with a reversal memory of `depth` (state of or_spring_words(depth)
 * doubles, see or_run's theta_final); events[4] accumulates as law_events */
double or_spring_step_mem(double* state, int depth, double dgamma, double G0, double gref, double h_max,
                          double* Gt, double* hk, long* events);
int or_spring_words(int depth);
/* threads of the OpenMP loops (timing of the oracle on a given core count) */
void or_set_threads(int n);
double or_ro_beta(double h_max);
/* single-spring update; state = {gp, gr, tr, gm, dir, skel}; returns tau after
 * the update, writes the tangent and the spring's equivalent damping */
double or_spring_step(double* state6, double dgamma, double G0, double gref, double h_max,
                      double* Gt, double* hk);
/* one integration point: all springs, returns D (6x6 full) and the mean h */
void or_ip_law(const double* deps6, double* state /*[n_springs*6]*/, int n_springs,
               const double* dirs, const double* weights, double G0, double Kb,
               double gref, double h_max, double* D36, double* hmean);

#ifdef __cplusplus
}
#endif
#endif
