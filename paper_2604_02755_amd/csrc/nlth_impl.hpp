// Internal declarations shared by the host runtime and the HIP kernels of
// libnlth.  Layouts (all on the device):
//   member-innermost: every per-member quantity q of node/element/point i is
//   stored at q[i*MB + m] with MB the padded member count, so a wavefront of
//   lanes that share an element but differ in member reads contiguous memory.
//   node vectors   v[(node*3 + c)*MB + m]
//   elements are grouped in blocks of EB = max(1, 64/MB) so that the EB x MB
//   lanes of a wavefront read contiguous memory:
//   D per point    D[(((e/EB)*84 + ip*21 + k)*EB + e%EB)*MB + m]  (upper
//                  triangle of the symmetric 6x6, row by row)
//   element h      h[e*MB + m]
//   law state      per chunk of ecp elements (a multiple of EB): four FP64
//                  fields {gp, gr, tr, gm} then two int32 fields {dir, skel},
//                  each f[((((el/EB)*ns + s)*4 + ip)*EB + el%EB)*MB + m]
//   mesh arrays    conn[k*ne + e], geo[k*ne + e] (k: 12 barycentric-gradient
//                  entries then the volume), in colour-sorted element order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nlth {

enum OpMode { OP_A = 0, OP_K = 1, OP_M = 2, OP_RHS = 3 };

constexpr int kMaxPartialBlocks = 2048;   // blocks of a fused vector kernel's partial sums
constexpr int kGatherBlocks = 16384;      // blocks of a node gather with partial sums
constexpr int kDashpotBlocks = 1024;      // blocks of a dashpot launch with partial sums
constexpr int kClusterNodes = 48;         // most distinct nodes of an element cluster
constexpr int kClusterElems = 16;         // most elements of an element cluster
// length (in MB-rows of doubles) of the partial-sum buffer
constexpr int kPartialRows = (3 * kMaxPartialBlocks > kGatherBlocks + kDashpotBlocks)
                                 ? 3 * kMaxPartialBlocks : kGatherBlocks + kDashpotBlocks;

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
    // node -> incidences (storage element * 10 + local node), ascending
    const int* inc_ptr;   // [nn+1]
    const int* inc;       // [10*ne]
    const int* celem;     // [ne] storage positions grouped by colour
    const int* bn_of_node;  // [nn] index into bn_node, or -1
    // element clusters: consecutive storage elements with few distinct nodes
    int ncl;
    const int* cl_off;      // [ncl+1] storage positions
    const int* cl_noff;     // [ncl+1] rows of the clusters' node lists
    const uint32_t* cl_lconn; // [ne*4] local nodes of each element, four 8-bit indices per word
    const int* cn_ptr;      // [nn+1] node -> cluster rows
    const int* cn_row;      // [rows] ascending per node
};

struct StepConst {
    double dt;
    double ahat, bhat;   // Rayleigh fit
    int damping_mode;    // 0 law, 1 const, 2 none
    double h0;
};

// ---- kernel launchers (kernels.hip) ----
void launch_fill(hipStream_t s, double* p, double v, long n);
// n int32 from src to dst (either may be device-mapped host memory)
void launch_copy_i32(hipStream_t s, const int* src, int* dst, int n);
void launch_fill32(hipStream_t s, float* p, float v, long n);
void launch_neg_copy(hipStream_t s, const double* a, double* b, long n);

// element-by-element operator over elements [e0, e1) of the sorted order
template <typename T>
void launch_ebe(hipStream_t s, OpMode mode, const DevMesh& M, int MB, int nm, int e0, int e1,
                const T* D, const double* h, const double* mat, int n_layers, StepConst sc,
                const T* x1, const T* x2, T* y, const int* active, bool out);
// y = sum over incident elements of the element outputs f, or over the
// node's cluster rows when clusters is set (+ bscale * base); with partial,
// also the per-member block partials of x . y (*nblk blocks).  MB <= 256.
template <typename T>
void launch_gather(hipStream_t s, const DevMesh& M, int MB, int nm, const T* f, const T* base, T bscale, T* y,
                   const int* active, const T* x, double* partial, int* nblk, bool clusters);
// cluster form of the operator (MB a multiple of 64): cluster node rows to co
void launch_ebe_cluster64(hipStream_t s, OpMode mode, const DevMesh& M, int MB, int nm, const double* D,
                          const double* h, const double* mat, StepConst sc, const double* x1, const double* x2,
                          double* co, const int* active);
void launch_ebe_cluster32(hipStream_t s, const DevMesh& M, int MB, int nm, const float* D32, const uint32_t* D16,
                          const double* h, const double* mat, StepConst sc, const float* x, float* co,
                          const int* active, bool d16_mean);
// node-centric absorbing-boundary dashpot: y += coef * C_abs x (+ 2 C_base vI for
// the right-hand side); with partial (MB <= 256), the per-member block partials
// of x . (C_abs x) are appended after the *nblk already written, *nblk grows
template <typename T>
void launch_dashpot(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int n_layers,
                    T coef, const T* x, T* y, const double* vI, const int* active, double* partial = nullptr,
                    int* nblk = nullptr);
// diagonal 3x3 blocks of A (sym, 6 entries per node) over elements [e0, e1)
void launch_diag(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const double* D,
                 const double* h, const double* mat, int n_layers, StepConst sc, double* diag);
// the same from the bfloat16 element-mean D of the inner operator (closed-form integrals)
void launch_diag_mean(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const uint32_t* D16,
                      const double* h, const double* mat, StepConst sc, double* diag);
void launch_diag_dashpot(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int n_layers,
                         double coef, double* diag);
void launch_invert_diag(hipStream_t s, int nn, int MB, int nm, const double* diag, double* pinv,
                        float* pinv32);

// law
void launch_law_init(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int n_layers,
                     int ns, const double* dirs, const double* w, double* D, float* D32, uint32_t* D16,
                     double* h, int only_m = -1, bool d16_mean = false);
void launch_theta_reset_member(hipStream_t s, void* base, long ecp, int ns, int MB, int m);
void launch_zero_member(hipStream_t s, double* p, long rows, int MB, int m);
// threads per block of the element-by-element launches on this host thread
void set_ebe_block(int bs);
// blocks per CU of the cluster launches on this host thread
void set_cluster_blocks(int b);
// convergence tail: the CG of at most G (16 or 32) listed members on compact
// rows (lane k = member tl[1 + k], tl[0] = the count); partial sums in the
// full [block][MB] layout.  Mixed path: its inner FP32 solve; FP64 path: PCG.
void launch_tail_pack(hipStream_t s, const DevMesh& M, int MB, int G, int n_layers, const int* tl,
                      const uint32_t* D16, const double* h, const double* mat, const float* pinv32, uint32_t* cD,
                      double* ch, double* cmat, float* cpinv);
void launch_tail_unpack(hipStream_t s, long nrows, int MB, int G, const int* tl, const float* c, float* full);
void launch_tail_pack64(hipStream_t s, const DevMesh& M, int MB, int G, int n_layers, const int* tl,
                        const double* D64, const double* h, const double* mat, const double* pinv, double* cD,
                        double* ch, double* cmat, double* cpinv);
// nrows member-innermost FP64 rows, full <-> compact
void launch_tail_rows64(hipStream_t s, long nrows, int MB, int G, const int* tl, const double* src, double* dst,
                        bool unpack);
// operator A on the compact rows summed per element cluster (the mixed path's
// inner operator, or the FP64 one with D per point): G-wide cluster rows
// co[(row * 3 + c) * G + k] for the gather with clusters = true
void launch_ebe32_ctail(hipStream_t s, const DevMesh& M, int G, const int* tl, const uint32_t* cD, const double* ch,
                        const double* cmat, StepConst sc, const float* x, float* co);
void launch_ebe64_ctail(hipStream_t s, const DevMesh& M, int G, const int* tl, const double* cD, const double* ch,
                        const double* cmat, StepConst sc, const double* x, double* co);
template <typename T>
void launch_gather_tail(hipStream_t s, const DevMesh& M, int MB, int nm, int G, const int* tl, const T* fc, T* y,
                        const int* active, const T* x, double* partial, int* nblk, bool clusters = false);
template <typename T>
void launch_dashpot_tail(hipStream_t s, const DevMesh& M, int MB, int nm, int G, const int* tl, const double* cmat,
                         T coef, const T* x, T* y, const int* active, double* partial, int* nblk);
// FP64 PCG on the compact rows: x += a p, r -= a Ap, z = P r with partials
// (r.r, r.z); then p = z + beta p
void launch_tail_pcg_update(hipStream_t s, int nn, int MB, int nm, int G, const int* tl, double* cx, double* cr,
                            double* cz, const double* cp, const double* cAp, const double* cpinv,
                            const double* alpha, const int* active, double* partial, int* nblk);
void launch_tail_p_update(hipStream_t s, long nrows, int nm, int G, const int* tl, const double* cz, double* cp,
                          const double* beta, const int* active);
// r_compact: r in the compact rows (the outer CG on compact rows), else full
void launch_tail_start(hipStream_t s, int nn, int MB, int nm, int G, const int* tl, const double* r, bool r_compact,
                       const float* cpinv, float* cir, float* ciz, float* cip, const int* active, double* partial,
                       int* nblk);
// the mixed path's outer flexible CG on the compact rows
void launch_tail_xr_update(hipStream_t s, long nrows, int MB, int nm, int G, const int* tl, double* cx, double* cr,
                           const double* cp, const double* cAp, const double* alpha, const int* active,
                           double* partial, int* nblk);
void launch_tail_inner_out(hipStream_t s, long nrows, int MB, int nm, int G, const int* tl, const float* ciz,
                           double* cz, const double* cAp, const double* cr, const int* active, double* partial,
                           int* nblk);
void launch_tail_update(hipStream_t s, int nn, int MB, int nm, int G, const int* tl, float* cir, float* cw,
                        const float* ciAp, const float* cpinv, const double* ialpha, const int* iactive,
                        double* partial, int* nblk);
void launch_tail_pz(hipStream_t s, long nrows, int nm, int G, const int* tl, float* ciz, float* cip, const float* cw,
                    const double* ialpha, const double* ibeta, const int* upd);
// inner FP32 operator (A) with D in FP32 (D32) or bfloat16 pairs (D16, if non-null)
void launch_ebe32(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const float* D32,
                  const uint32_t* D16, const double* h, const double* mat, StepConst sc, const float* x, float* y,
                  const int* active, bool out, bool d16_mean);
void launch_theta_init(hipStream_t s, void* theta_chunk, long ecp, int ns, int MB);
void launch_law(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int ec, long ecp, const double* mat,
                int n_layers, const int* nonlinear, int ns, int depth, const double* dirs, const double* w,
                const double* du, void* theta_chunk, double* D, float* D32, uint32_t* D16, double* h,
                const int* stepping, bool d16_mean);

// ---- CG vectors (vec.hip): partial sums go to partial[(k*nblk + blk)*MB + m]
template <typename T>
void launch_dotsv(hipStream_t s, int nd, const T* a0, const T* b0, const T* a1, const T* b1, const T* a2,
                  const T* b2, long nrows, int MB, int nm, const int* flag, double* partial, int* nblk);

struct CgScalars {  // per member [MB] device arrays
    double *bb, *rr, *rz, *alpha, *beta, *pAp, *r0;
    int *active, *iters, *status, *stepping;  // stepping: member takes part in this step
    int *inner_active, *inner_iters, *inner_total;
    int* inner_upd;  // members whose inner alpha was formed this iteration (their iz, ip still update)
    double *irr, *irz, *ialpha, *ibeta, *ir0;
    double* lz;  // inner CG coefficients: alpha_k at [k * MB + m], beta_k at [(kLanczosMax + k) * MB + m]
};

// inner CG iterations whose coefficients are kept for the spectrum estimate
constexpr int kLanczosMax = 64;
// law state per spring and integration point: 4 FP64 + one int32 of flags,
// plus two FP64 per older reversal point kept with a memory of depth > 1
constexpr int kThetaBytes = 36;
constexpr int kMaxMasingDepth = 8;  // the count of older points fits 3 bits of the flags
inline int theta_bytes(int depth) { return kThetaBytes + 16 * ((depth > 1 ? depth : 1) - 1); }
// Chebyshev degree limit; coefficient table cheb[(2 k + 0/1) * MB + m] =
// (c1_k, c2_k), k < kChebMax, and cheb[2 kChebMax * MB + m] = c0
constexpr int kChebMax = 64;

enum FinalizeStage {
    FIN_START = 0,   // (b.b, r.r, r.z): PCG start, active flags
    FIN_ALPHA,       // (p.Ap): alpha = rz / pAp
    FIN_BETA,        // (r.r, r.z): convergence, beta = rz_new / rz (PCG)
    FIN_FCG_START,   // (b.b, r.r): flexible CG start (outer)
    FIN_FCG_RZ,      // (z.Ap, z.r): rz = z.r after the first preconditioner call
    FIN_FCG_BETA,    // (z.Ap, z.r): beta = -alpha z.Ap / rz_old ; rz = z.r
    FIN_FCG_RR,      // (r.r): outer convergence check
    FIN_IN_START,    // (ir.ir, ir.w) inner start
    FIN_IN_ALPHA,    // (ip.iAp) inner alpha
    FIN_IN_BETA,     // (ir.ir, ir.w) inner convergence, beta
    FIN_CHEB_COUNT,  // (-): inner_total += degree for the outer-active members
    FIN_EST_START    // (ir.ir, ir.w) inner CG start on a random vector, for the members in this step
};
// per-member block partials of a compact kernel: lane k's sum over the block's
// rows (a fixed tree in LDS) goes to partial[(j * gridDim + blockIdx) * MB +
// tl[1 + k]], zero for the members not listed
template <int ND, int G>
__device__ __forceinline__ void tail_partials(double acc[ND], int MB, int m, double* __restrict__ partial, int boff,
                                              int nblk)
{
    __shared__ double sh[ND][256];
    __shared__ double pm[ND][256];
    const int t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < ND; ++j) sh[j][t] = acc[j];
    __syncthreads();
    for (int s = 128; s >= G; s >>= 1) {  // s a multiple of G: lane k stays lane k
        if (t < s)
#pragma unroll
            for (int j = 0; j < ND; ++j) sh[j][t] += sh[j][t + s];
        __syncthreads();
    }
    if (t < MB)
#pragma unroll
        for (int j = 0; j < ND; ++j) pm[j][t] = 0.0;
    __syncthreads();
    if (t < G && m >= 0 && m < MB)
#pragma unroll
        for (int j = 0; j < ND; ++j) pm[j][m] = sh[j][t];  // listed members are distinct
    __syncthreads();
    if (t < MB)
#pragma unroll
        for (int j = 0; j < ND; ++j) partial[((size_t)j * nblk + boff + blockIdx.x) * MB + t] = pm[j][t];
}

void launch_finalize(hipStream_t s, FinalizeStage st, int nd, int MB, int nm, const double* partial, int nblk,
                     CgScalars cs, double tol2, int maxit);

void launch_pcg_start(hipStream_t s, int nn, int MB, int nm, const double* b, const double* Ap, const double* pinv,
                      double* r, double* z, double* p, const int* stepping, double* partial, int* nblk);
void launch_pcg_update(hipStream_t s, int nn, int MB, int nm, double* x, double* r, double* z, const double* p,
                       const double* Ap, const double* pinv, const double* alpha, const int* active, double* partial,
                       int* nblk);
template <typename T>
void launch_p_update(hipStream_t s, long nrows, int MB, int nm, const T* z, T* p, const double* beta, const int* active,
                     T* y);
void launch_xr_update(hipStream_t s, long nrows, int MB, int nm, double* x, double* r, const double* p, const double* Ap,
                      const double* alpha, const int* active, double* partial, int* nblk);
void launch_inner_start(hipStream_t s, int nn, int MB, int nm, const double* r, const float* pinv32, float* ir,
                        float* iz, float* ip, float* w, float* iAp, const int* active, double* partial, int* nblk);
void launch_inner_update(hipStream_t s, int nn, int MB, int nm, float* ir, float* w, const float* iAp,
                         const float* pinv32, const double* ialpha, const int* iactive, double* partial, int* nblk);
void launch_inner_pz(hipStream_t s, long nrows, int MB, int nm, float* iz, float* ip, const float* w,
                     const double* ialpha, const double* ibeta, const int* upd);
void launch_inner_out(hipStream_t s, long nrows, int MB, int nm, const float* iz, double* z, const double* Ap,
                      const double* r, const int* active, double* partial, int* nblk);
void launch_zero_if_b0(hipStream_t s, long nrows, int MB, int nm, double* x, const double* bb, const int* stepping);

// Chebyshev inner solve (preconditioner of the outer flexible CG)
void launch_cheb_bounds(hipStream_t s, int MB, int nm, CgScalars cs, int degree, double lo_scale, double hi_scale,
                        float* cheb, double* bounds);
void launch_cheb_hi_estimate(hipStream_t s, int MB, int nm, CgScalars cs, double scale, double* bounds);
void launch_fill_random(hipStream_t s, double* x, long n, uint64_t seed);
void launch_cheb_start(hipStream_t s, int nn, int MB, int nm, const double* r, const float* pinv32,
                       const float* cheb, float* ir, float* iz, float* id, const int* active);
void launch_cheb_update(hipStream_t s, int nn, int MB, int nm, int k, bool last, float* iz, float* ir,
                        const float* id, const float* iAp, float* id_next, const float* pinv32, const float* cheb,
                        const int* active);
void launch_dashpot_rows(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, float coef,
                         const float* x, float* qb, const int* active);
void launch_gather_cheb(hipStream_t s, const DevMesh& M, int MB, int nm, int k, bool last, const float* rows,
                        const float* qb, float* iz, float* ir, const float* id, float* id_next, const float* pinv32,
                        const float* cheb, const int* active);

// Newmark state updates (Section 2.1) and receivers
void launch_newmark(hipStream_t s, long n, int MB, int nm, const double* du, double* u, double* v,
                    double* a, double dt, const int* stepping);
// CG initial guess extrapolated from the previous increments (order 0..2), history shifted
void launch_predict(hipStream_t s, long n, int MB, int nm, int order, double* du, double* d2, double* d3,
                    const int* stepping);
void launch_receivers(hipStream_t s, int nrecv, const int* recv, int MB, int nm, const double* v,
                      double* vel_hist, const int* member_step, int n_steps_max, double* vmax,
                      const int* stepping);
void launch_incident_velocity(hipStream_t s, int MB, int nm, int n_steps, const double* acc,
                              double* vI_all, double dt);
void launch_pick_vI(hipStream_t s, int MB, int nm, int n_steps, const double* vI_all,
                    const int* member_step, double* vI_cur);
void launch_cast32(hipStream_t s, const double* a, float* b, long n);
void launch_response_spectra(hipStream_t s, const double* vel, int ns, int nt, double dt, const double* periods, int np,
                             double h, int kind, double* out);

}  // namespace nlth
