// Internal declarations shared by the host runtime and the HIP kernels of
// libnlth.  Layouts (all on the device):
//   member-innermost: every per-member quantity q of node/element/point i is
//   stored at q[i*MB + m] with MB the padded member count, so a wavefront of
//   lanes that share an element but differ in member reads contiguous memory.
//   node vectors   v[(node*3 + c)*MB + m]
//   D per point    D[((ip*21 + k)*ne + e)*MB + m]   (upper triangle, row by row)
//   element h      h[e*MB + m]
//   law state      per chunk of elements [e0, e0+ec): field f in {gp, gr, tr,
//                  gm} (FP64) then {dir, skel} (int32), each
//                  f[((s*4 + ip)*ec + e_local)*MB + m]
//   mesh arrays    conn[k*ne + e], geo[k*ne + e] (k: 12 barycentric-gradient
//                  entries then the volume), in colour-sorted element order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlth {

enum OpMode { OP_A = 0, OP_K = 1, OP_M = 2, OP_RHS = 3 };

constexpr int kMaxPartialBlocks = 512;

// Per-member material of one layer, member-innermost: mat[(l*MAT_N + field)*MB + m]
enum MatField { MAT_RHO = 0, MAT_G0, MAT_KB, MAT_VS, MAT_VP, MAT_GREF, MAT_HMAX, MAT_BETA, MAT_N };

struct DevMesh {
    int ne, nn;
    const int* conn;      // [10][ne]
    const double* geo64;  // [13][ne]
    const float* geo32;   // [13][ne]
    const int* layer;     // [ne]
    // boundary nodes (node-centric dashpot gather)
    int nbn;
    const int* bn_node;   // [nbn]
    const int* bn_ptr;    // [nbn+1] into entries
    const int* bn_face;   // [entries]
    const int* bn_loc;    // [entries] local index (0..5) of the node in the face
    const int* f_node;    // [nf*6]
    const double* f_M;    // [nf*36] int N_a N_b dA
    const double* f_n;    // [nf*3] unit normal
    const int* f_layer;   // [nf]
    const uint8_t* f_kind;
};

struct StepConst {
    double dt;
    double ahat, bhat;   // Rayleigh fit
    int damping_mode;    // 0 law, 1 const, 2 none
    double h0;
};

// ---- kernel launchers (kernels.hip) ----
void launch_fill(hipStream_t s, double* p, double v, long n);
void launch_fill32(hipStream_t s, float* p, float v, long n);
void launch_neg_copy(hipStream_t s, const double* a, double* b, long n);

// element-by-element operator over elements [e0, e1) of the sorted order
template <typename T>
void launch_ebe(hipStream_t s, OpMode mode, const DevMesh& M, int MB, int nm, int e0, int e1,
                const T* D, const double* h, const double* mat, int n_layers, StepConst sc,
                const T* x1, const T* x2, T* y, const int* active);
// node-centric absorbing-boundary dashpot: y += coef * C_abs x1 (+ 2 C_base vI for RHS)
template <typename T>
void launch_dashpot(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int n_layers,
                    T coef, const T* x, T* y, const double* vI, const int* active);
// diagonal 3x3 blocks of A (sym, 6 entries per node) over elements [e0, e1)
void launch_diag(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const double* D,
                 const double* h, const double* mat, int n_layers, StepConst sc, double* diag);
void launch_diag_dashpot(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int n_layers,
                         double coef, double* diag);
void launch_invert_diag(hipStream_t s, int nn, int MB, int nm, const double* diag, double* pinv,
                        float* pinv32);

// law
void launch_law_init(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int n_layers,
                     int ns, const double* dirs, const double* w, double* D, float* D32, double* h);
void launch_theta_init(hipStream_t s, void* theta_chunk, long ec, int ns, int MB);
void launch_law(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int ec, const double* mat,
                int n_layers, const int* nonlinear, int ns, const double* dirs, const double* w,
                const double* du, void* theta_chunk, double* D, float* D32, double* h,
                const int* stepping);

// vectors (FP64 CG)
// dots: partial[k][blk][MB] for k < nd of  sum a_k . b_k
void launch_dots(hipStream_t s, int nd, const double* a0, const double* b0, const double* a1,
                 const double* b1, const double* a2, const double* b2, long nrows, int MB,
                 double* partial, int* nblk_out);
void launch_dots32(hipStream_t s, int nd, const float* a0, const float* b0, const float* a1,
                   const float* b1, long nrows, int MB, double* partial, int* nblk_out);

struct CgScalars {  // per member [MB] device arrays
    double *bb, *rr, *rz, *alpha, *beta, *pAp, *r0;
    int *active, *iters, *status, *stepping;  // stepping: member takes part in this step
    int *inner_active, *inner_iters, *inner_total;
    double *irr, *irz, *ialpha, *ibeta, *ir0;
    int* any_active;  // [1]
};

enum FinalizeStage {
    FIN_START = 0,   // partial {bb, rr, rz}: set active, rz
    FIN_ALPHA,       // partial {pAp}: alpha = rz / pAp
    FIN_BETA,        // partial {rr, rz}: convergence, beta = rz_new / rz (PCG)
    FIN_FCG_START,   // partial {bb, rr}: flexible CG start (outer)
    FIN_FCG_RZ,      // partial {rz}: rz = r.z after the first preconditioner call
    FIN_FCG_BETA,    // partial {zAp, rz}: beta = -alpha zAp / rz_old ; rz = rz_new
    FIN_FCG_RR,      // partial {rr}: outer convergence check
    FIN_IN_START,    // partial {rr, rz} (inner): inner_active, irz
    FIN_IN_ALPHA,    // partial {pAp} inner
    FIN_IN_BETA      // partial {rr, rz} inner
};
void launch_finalize(hipStream_t s, FinalizeStage st, int MB, int nm, const double* partial, int nblk,
                     CgScalars cs, double tol2, int maxit);

// r = b - Ap; z = Pinv r; p = z (members active) ; x zeroed for members with bb == 0 later
void launch_pcg_start(hipStream_t s, int nn, int MB, int nm, const double* b, const double* Ap,
                      const double* pinv, double* r, double* z, double* p, const int* stepping);
void launch_pcg_update(hipStream_t s, int nn, int MB, int nm, double* x, double* r, double* z,
                       const double* p, const double* Ap, const double* pinv, const double* alpha,
                       const int* active);
void launch_axpby_p(hipStream_t s, long n, int MB, int nm, const double* z, double* p,
                    const double* beta, const int* active);
void launch_zero_inactive_start(hipStream_t s, long n, int MB, int nm, double* x, const double* bb,
                                const int* stepping);
// FCG helpers
void launch_xr_update(hipStream_t s, long n, int MB, int nm, double* x, double* r, const double* p,
                      const double* Ap, const double* alpha, const int* active);
void launch_copy_p(hipStream_t s, long n, int MB, int nm, const double* z, double* p, const int* active);
// inner FP32 PCG
void launch_inner_start(hipStream_t s, int nn, int MB, int nm, const double* r, const float* pinv32,
                        float* ir, float* iz, float* ip, float* w, const int* active);
void launch_inner_update(hipStream_t s, int nn, int MB, int nm, float* iz, float* ir, float* w,
                         const float* ip, const float* iAp, const float* pinv32, const double* ialpha,
                         const int* iactive);
void launch_inner_p(hipStream_t s, long n, int MB, int nm, const float* w, float* ip,
                    const double* ibeta, const int* iactive);
void launch_inner_out(hipStream_t s, long n, int MB, int nm, const float* iz, double* z,
                      const int* active);

// Newmark state updates (Section 2.1) and receivers
void launch_newmark(hipStream_t s, long n, int MB, int nm, const double* du, double* u, double* v,
                    double* a, double dt, const int* stepping);
void launch_receivers(hipStream_t s, int nrecv, const int* recv, int MB, int nm, const double* v,
                      double* vel_hist, const int* member_step, int n_steps_max, double* vmax,
                      const int* stepping);
void launch_incident_velocity(hipStream_t s, int MB, int nm, int n_steps, const double* acc,
                              double* vI_all, double dt);
void launch_pick_vI(hipStream_t s, int MB, int nm, int n_steps, const double* vI_all,
                    const int* member_step, double* vI_cur);
void launch_cast32(hipStream_t s, const double* a, float* b, long n);

}  // namespace nlth
