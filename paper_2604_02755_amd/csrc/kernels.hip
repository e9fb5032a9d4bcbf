// HIP kernels (gfx950) for the nonlinear time-history ensemble solver.
//
// Method: Ichimura et al., arXiv 2604.02755.  Section 2.1, Eq. 1 (Newmark
// incremental step), Eq. 2 (K_e from D at the integration points), the
// multi-spring Ramberg-Osgood/Masing law; Section 2.2, Algorithm 4 (EBE
// operator inside CG, law update per step).
//
// All per-member data is member-innermost (index * MB + m): one lane handles
// one (element, member) or (node, member) pair; when MB >= 64 a wavefront
// covers 64 members of one element, so element data is wave-uniform and
// member data is read in contiguous 256/512-byte rows.
//
// Element-by-element scatter is atomic-free: a launch covers one colour of
// the element colouring (no two elements of a colour share a node), and the
// host issues the colours in sequence on one stream.
#include <math.h>

#include "nlth_impl.hpp"

namespace nlth {

// ---------------------------------------------------------------------------
// constants
// ---------------------------------------------------------------------------

// 4-point degree-2 rule: barycentric (a, b, b, b) and permutations, weight V/4.
#define QA_ 0.5854101966249685
#define QB_ 0.1381966011250105

// Consistent mass of the 10-node tet divided by its volume: the classical
// pattern /420 (corner diagonal 6, corner-corner 1, corner and an edge through
// it -4, corner and the opposite-side edge -6, edge diagonal 32, edges sharing
// a vertex 16, opposite edges 8).
__host__ __device__ constexpr double mass_ref(int a, int b)
{
    // edges as vertex pairs
    constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
    if (a < 4 && b < 4) return (a == b ? 6.0 : 1.0) / 420.0;
    if (a < 4 || b < 4) {
        int c = a < 4 ? a : b;
        int e = (a < 4 ? b : a) - 4;
        return (E[e][0] == c || E[e][1] == c ? -4.0 : -6.0) / 420.0;
    }
    if (a == b) return 32.0 / 420.0;
    int ea = a - 4, eb = b - 4;
    bool share = E[ea][0] == E[eb][0] || E[ea][0] == E[eb][1] || E[ea][1] == E[eb][0] ||
                 E[ea][1] == E[eb][1];
    return (share ? 16.0 : 8.0) / 420.0;
}

// index of (r, c) in the row-by-row upper triangle of a symmetric 6x6
__host__ __device__ constexpr int sym6(int r, int c)
{
    return r <= c ? r * 6 - r * (r - 1) / 2 + (c - r) : c * 6 - c * (c - 1) / 2 + (r - c);
}

template <typename T> __device__ __forceinline__ const T* geo_of(const DevMesh& M);
template <> __device__ __forceinline__ const double* geo_of<double>(const DevMesh& M) { return M.geo64; }
template <> __device__ __forceinline__ const float* geo_of<float>(const DevMesh& M) { return M.geo32; }

__device__ __forceinline__ double matv(const double* mat, int l, int f, int MB, int m)
{
    return mat[((long)l * MAT_N + f) * MB + m];
}

// Shape-function gradients of the quadratic tet at integration point j.
template <typename T>
__device__ __forceinline__ void shape_grads(int j, const T gL[4][3], T G[10][3])
{
    T L[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) L[i] = (i == j) ? (T)QA_ : (T)QB_;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a) G[i][a] = ((T)4 * L[i] - (T)1) * gL[i][a];
    constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
#pragma unroll
    for (int e = 0; e < 6; ++e)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            G[4 + e][a] = (T)4 * (L[E[e][0]] * gL[E[e][1]][a] + L[E[e][1]] * gL[E[e][0]][a]);
}

// engineering strain (Voigt xx, yy, zz, xy, yz, zx) of nodal field u at one point
template <typename T>
__device__ __forceinline__ void strain(const T G[10][3], const T u[10][3], T eps[6])
{
#pragma unroll
    for (int k = 0; k < 6; ++k) eps[k] = 0;
#pragma unroll
    for (int n = 0; n < 10; ++n) {
        eps[0] += G[n][0] * u[n][0];
        eps[1] += G[n][1] * u[n][1];
        eps[2] += G[n][2] * u[n][2];
        eps[3] += G[n][1] * u[n][0] + G[n][0] * u[n][1];
        eps[4] += G[n][2] * u[n][1] + G[n][1] * u[n][2];
        eps[5] += G[n][0] * u[n][2] + G[n][2] * u[n][0];
    }
}

// ---------------------------------------------------------------------------
// simple vector kernels
// ---------------------------------------------------------------------------

__global__ void k_fill(double* p, double v, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill32(float* p, float v, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_neg_copy(const double* a, double* b, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = -a[i];
}
__global__ void k_cast32(const double* a, float* b, long n)
{
    long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void k_copy_i32(const int* a, int* b, int n)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

static inline unsigned nblocks(long n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

void launch_copy_i32(hipStream_t s, const int* src, int* dst, int n)
{
    if (n > 0) hipLaunchKernelGGL(k_copy_i32, dim3(nblocks(n)), dim3(256), 0, s, src, dst, n);
}
void launch_fill(hipStream_t s, double* p, double v, long n)
{
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(nblocks(n)), dim3(256), 0, s, p, v, n);
}
void launch_fill32(hipStream_t s, float* p, float v, long n)
{
    if (n > 0) hipLaunchKernelGGL(k_fill32, dim3(nblocks(n)), dim3(256), 0, s, p, v, n);
}
void launch_neg_copy(hipStream_t s, const double* a, double* b, long n)
{
    if (n > 0) hipLaunchKernelGGL(k_neg_copy, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
}
void launch_cast32(hipStream_t s, const double* a, float* b, long n)
{
    if (n > 0) hipLaunchKernelGGL(k_cast32, dim3(nblocks(n)), dim3(256), 0, s, a, b, n);
}

// ---------------------------------------------------------------------------
// element-by-element operator (Eq. 1 left-hand side, Eq. 2 stiffness)
// ---------------------------------------------------------------------------
//
// Per (element, member): gather the 10 nodal displacements, add the mass
// term (consistent P2 mass applied through corner and edge sums), then the
// stiffness term of Eq. 2 with the 4-point rule.  Straight-sided tets make the
// shape-function gradients linear in the barycentrics, so the strain at the
// four points is a combination of four per-element 6-vectors E_k and the
// point forces fold back onto the nodes the same way; D_j is streamed once.

// Voigt symmetric part of u (x) g  (F_cd = u_c g_d, engineering shear)
template <typename T>
__device__ __forceinline__ void vsym_acc(const T u[3], const T g[3], T o[6])
{
    // each component a chain of fused multiply-adds into the accumulator
    o[0] = fma(u[0], g[0], o[0]);
    o[1] = fma(u[1], g[1], o[1]);
    o[2] = fma(u[2], g[2], o[2]);
    o[3] = fma(u[0], g[1], fma(u[1], g[0], o[3]));
    o[4] = fma(u[1], g[2], fma(u[2], g[1], o[4]));
    o[5] = fma(u[2], g[0], fma(u[0], g[2], o[5]));
}

// f += s * sigma . g  (sigma in Voigt order xx, yy, zz, xy, yz, zx)
template <typename T>
__device__ __forceinline__ void tdot_acc(const T sg[6], const T g[3], T s, T f[3])
{
    f[0] += s * (sg[0] * g[0] + sg[3] * g[1] + sg[5] * g[2]);
    f[1] += s * (sg[3] * g[0] + sg[1] * g[1] + sg[4] * g[2]);
    f[2] += s * (sg[5] * g[0] + sg[4] * g[1] + sg[2] * g[2]);
}

// f += sigma . g as chains of fused multiply-adds into f
template <typename T>
__device__ __forceinline__ void tdot_add(const T sg[6], const T g[3], T f[3])
{
    f[0] = fma(sg[0], g[0], fma(sg[3], g[1], fma(sg[5], g[2], f[0])));
    f[1] = fma(sg[3], g[0], fma(sg[1], g[1], fma(sg[4], g[2], f[1])));
    f[2] = fma(sg[5], g[0], fma(sg[4], g[1], fma(sg[2], g[2], f[2])));
}

// index of D(e, j, k) for member m: elements in blocks of EB so that a
// wavefront's lanes (EB elements x MB members) read contiguous memory
__device__ __forceinline__ long d_index(long e, int j, int k, int MB, int EB, int m)
{
    return (((e / EB) * 84 + j * 21 + k) * EB + e % EB) * (long)MB + m;
}

// bfloat16 storage of D for the inner operator: pairs of consecutive upper-
// triangle entries (k = 2q, 2q+1; k = 21 is padding) packed in one 32-bit word
__device__ __forceinline__ long d16_index(long e, int j, int q, int MB, int EB, int m)
{
    return (((e / EB) * 44 + j * 11 + q) * EB + e % EB) * (long)MB + m;
}
// element-mean D of the inner operator in bfloat16 pairs: 11 words per element
__device__ __forceinline__ long d16m_index(long e, int q, int MB, int EB, int m)
{
    return (((e / EB) * 11 + q) * EB + e % EB) * (long)MB + m;
}
__device__ __forceinline__ uint32_t f2bf(double x)
{
    // round to nearest even on the FP32 bit pattern
    const uint32_t u = __float_as_uint((float)x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float bf2f(uint32_t b) { return __uint_as_float(b << 16); }

constexpr int kEdgeOpp[6] = {5, 3, 4, 1, 2, 0};  // edge opposite each edge

// element outputs (the 30 nodal forces of an element-member) stored for the
// gather: row r = 3 * local node + component, element blocks of EB as for D
__device__ __forceinline__ size_t f_index(long e, int r, int MB, int EB, int m)
{
    return (((size_t)(e / EB) * 30 + r) * EB + e % EB) * (size_t)MB + m;
}

// DK: storage of D, 0 = T itself, 1 = bfloat16 pairs (uint32 words).
// OUT = 0: positions [e0, e1) of the colour lists (tets of one colour share no
// node), forces added into y.  OUT = 1: storage positions [e0, e1), forces
// written to the element-output array y (f_index); the grid is a multiple of
// 8 blocks and each XCD takes a contiguous range of elements.
// Forces of one element-member (element e, member m): the 30 nodal values of
// the operator of MODE applied to x1 (and x2), written to f; nbase[n] is the
// offset of node n's row in the nodal vectors.
// element i of an array at a wavefront-uniform base: the byte offset is
// formed in 32 bits, so the load takes the scalar-base + 32-bit vector-offset
// form (no per-lane 64-bit address arithmetic).  i * sizeof(T) < 2^32.
template <typename T>
__device__ __forceinline__ T ld_u(const T* base, uint32_t i)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T));
}

template <typename T>
__device__ __forceinline__ T ld_u_nt(const T* base, uint32_t i)
{
    return __builtin_nontemporal_load(
        reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + i * (uint32_t)sizeof(T)));
}

template <typename T, int DK, int MODE>
__device__ __forceinline__ void ebe_element(const DevMesh& M, int MB, int m, long e, const void* __restrict__ Dv,
                                            const double* __restrict__ h, const double* __restrict__ mat,
                                            const StepConst& sc, const T* __restrict__ x1,
                                            const T* __restrict__ x2, T f[10][3], size_t nbase[10])
{
    const int EB = MB >= 64 ? 1 : 64 / MB;
    const long ne = M.ne;
    const T* geo = geo_of<T>(M);
    T gL[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) gL[k / 3][k % 3] = geo[k * ne + e];
    const T vol = geo[12 * ne + e];
    int nodes[10];
#pragma unroll
    for (int k = 0; k < 10; ++k) nodes[k] = M.conn[k * ne + e];
    const int l = M.layer[e];
    const double rho = matv(mat, l, MAT_RHO, MB, m);
    double he = 0.0;
    if (sc.damping_mode == 0 && h) he = h[e * MB + m];
    else if (sc.damping_mode == 1) he = sc.h0;
    const double dt = sc.dt;
    T sm, sk, cv = 0;
    if (MODE == OP_A) {
        // the quotients by dt involve kernel arguments only (computed once per
        // thread), so no FP64 division is left per element
        const double m4 = 4.0 / (dt * dt), a2 = 2.0 * sc.ahat / dt, b2 = 2.0 * sc.bhat / dt;
        sm = (T)(rho * (double)vol * (m4 + a2 * he));
        sk = (T)(1.0 + b2 * he);
    } else if (MODE == OP_K) {
        sm = 0; sk = 1;
    } else if (MODE == OP_M) {
        sm = (T)(rho * (double)vol); sk = 0;
    } else {  // RHS: M (a + (4/dt + alpha) v) + beta K v
        sm = (T)(rho * (double)vol);
        sk = (T)(sc.bhat * he);
        cv = (T)(4.0 / dt + sc.ahat * he);
    }
    // addresses: a base per node (wave-uniform when a wavefront is one element)
    // plus a 32-bit lane offset, so loads use a scalar base and no 64-bit math
#pragma unroll
    for (int n = 0; n < 10; ++n) nbase[n] = (size_t)nodes[n] * 3 * MB;
    T xk[10][3];
    // ---- mass: consistent P2 mass applied through corner/edge sums; with
    // the scale folded into the coefficients each node's force is a short
    // chain of fused multiply-adds on the corner and edge sums
    const T s420 = sm * (T)(1.0 / 420.0);
    const T c2 = s420 * (T)2, c5 = s420 * (T)5, c6 = s420 * (T)6, c8 = s420 * (T)8, c16 = s420 * (T)16;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T xm[10];
        // the component's offset joins the uniform base, so every load is a
        // scalar base plus the member lane
        const T* x1c = x1 + (size_t)c * MB;
        const T* x2c = (MODE == OP_RHS) ? x2 + (size_t)c * MB : x2;
#pragma unroll
        for (int n = 0; n < 10; ++n) {
            const T v1 = ld_u(x1c + nbase[n], (uint32_t)m);
            xk[n][c] = v1;
            xm[n] = (MODE == OP_RHS) ? ld_u(x2c + nbase[n], (uint32_t)m) + cv * v1 : v1;
        }
        if (MODE == OP_K) {
#pragma unroll
            for (int n = 0; n < 10; ++n) f[n][c] = 0;
        } else {
            constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
            const T Sc = xm[0] + xm[1] + xm[2] + xm[3];
            const T Se = xm[4] + xm[5] + xm[6] + xm[7] + xm[8] + xm[9];
            // corner i: (5 x_i + Sc + 2 A_i - 6 Se) / 420, A_i = the edges at i;
            // edge q (a, b): (2 (x_a + x_b) - 6 Sc + 16 x_q + 16 Se - 8 x_opp) / 420
            const T bc = fma(-c6, Se, s420 * Sc);
            const T be = fma(c16, Se, -c6 * Sc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T A = 0;
#pragma unroll
                for (int q = 0; q < 6; ++q)
                    if (E[q][0] == i || E[q][1] == i) A += xm[4 + q];
                f[i][c] = fma(c5, xm[i], fma(c2, A, bc));
            }
#pragma unroll
            for (int q = 0; q < 6; ++q)
                f[4 + q][c] = fma(c2, xm[E[q][0]] + xm[E[q][1]],
                                  fma(c16, xm[4 + q], fma(-c8, xm[4 + kEdgeOpp[q]], be)));
        }
    }
    // ---- stiffness (Eq. 2)
    if (MODE != OP_M && sk != (T)0) {
        constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
        // E_k = voigt(G_k), G_k = 4 x_k gL_k^T - H + 4 sum_{edges (k,o)} x_ko gL_o^T,
        // H = sum_k x_k gL_k^T: the corner products P_k are formed once
        T Ek[4][6], H[6];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int q = 0; q < 6; ++q) Ek[k][q] = 0;
            vsym_acc<T>(xk[k], gL[k], Ek[k]);
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            H[q] = Ek[0][q] + Ek[1][q] + Ek[2][q] + Ek[3][q];
#pragma unroll
            for (int k = 0; k < 4; ++k) Ek[k][q] = (T)4 * Ek[k][q] - H[q];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            const T u4[3] = {(T)4 * xk[4 + q][0], (T)4 * xk[4 + q][1], (T)4 * xk[4 + q][2]};
            vsym_acc<T>(u4, gL[E[q][1]], Ek[E[q][0]]);
            vsym_acc<T>(u4, gL[E[q][0]], Ek[E[q][1]]);
        }
        T S[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) S[q] = Ek[0][q] + Ek[1][q] + Ek[2][q] + Ek[3][q];
        const T w = sk * vol * (T)0.25;
        const T c1 = (T)(QA_ - QB_);
        T dm[22];  // DK 4: one D for the element, read once
        if constexpr (DK == 4) {
            const size_t eb = (size_t)(e / EB) * EB, ei = (size_t)(e % EB);
            const uint32_t rs = (uint32_t)(EB * MB);
            const uint32_t* D = (const uint32_t*)Dv + (eb * 11 + ei) * MB;
#pragma unroll
            for (int q = 0; q < 11; ++q) {
                const uint32_t wv = ld_u_nt(D, (uint32_t)q * rs + (uint32_t)m);
                dm[2 * q] = (T)bf2f(wv & 0xFFFFu);
                dm[2 * q + 1] = (T)bf2f(wv >> 16);
            }
        }
        if constexpr (DK == 4) {
            // One D for the element: the stress sigma(L) = sum_k L_k D E_k is
            // linear in the barycentrics and the forces integrate in closed form
            // with int L_a L_b dV = V (1 + delta_ab) / 20:
            //   corner i:     (V/20) (4 s_i - T) . gL_i,
            //   edge (a, b):  (4V/20) ((T + s_a) . gL_b + (T + s_b) . gL_a),
            // with s_k = D E_k and T = s_1 + ... + s_4 (the 4-point rule gives the
            // same values for constant D).
            const T v20 = sk * vol * (T)0.05;
            T sgk[4][6], T6[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    T a = 0;
#pragma unroll
                    for (int c = 0; c < 6; ++c) a += dm[sym6(r, c)] * Ek[k][c];
                    sgk[k][r] = a * v20;
                    T6[r] += sgk[k][r];
                }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                T v[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) v[r] = (T)4 * sgk[i][r] - T6[r];
                tdot_add<T>(v, gL[i], f[i]);
            }
            T T4[6];  // the edges' factor 4 folded into their stress sums
#pragma unroll
            for (int r = 0; r < 6; ++r) T4[r] = (T)4 * T6[r];
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const int a = E[q][0], b = E[q][1];
                T va[6], vb[6];
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    va[r] = fma((T)4, sgk[a][r], T4[r]);
                    vb[r] = fma((T)4, sgk[b][r], T4[r]);
                }
                tdot_add<T>(va, gL[b], f[4 + q]);
                tdot_add<T>(vb, gL[a], f[4 + q]);
            }
            return;
        }
        T ST[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            T eps[6], sg[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) eps[q] = (T)QB_ * S[q] + c1 * Ek[j][q];
            T d[22];
            // element base (uniform per wavefront) + 32-bit row offsets
            const size_t eb = (size_t)(e / EB) * EB, ei = (size_t)(e % EB);
            const uint32_t rs = (uint32_t)(EB * MB);  // stride between rows (j, k)
            if constexpr (DK == 4) {
#pragma unroll
                for (int k = 0; k < 22; ++k) d[k] = dm[k];
            } else if constexpr (DK == 0) {
                const T* D = (const T*)Dv + (eb * 84 + ei) * MB;
#pragma unroll
                for (int k = 0; k < 21; ++k)
                    d[k] = ld_u_nt(D, (uint32_t)(j * 21 + k) * rs + (uint32_t)m);
            } else {
                const uint32_t* D = (const uint32_t*)Dv + (eb * 44 + ei) * MB;
#pragma unroll
                for (int q = 0; q < 11; ++q) {
                    const uint32_t wv = ld_u_nt(D, (uint32_t)(j * 11 + q) * rs + (uint32_t)m);
                    d[2 * q] = (T)bf2f(wv & 0xFFFFu);
                    d[2 * q + 1] = (T)bf2f(wv >> 16);
                }
            }
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                T a = 0;
#pragma unroll
                for (int c = 0; c < 6; ++c) a += d[sym6(r, c)] * eps[c];
                sg[r] = a * w;
                ST[r] += sg[r];
            }
            // point-j part of the nodal forces
#pragma unroll
            for (int i = 0; i < 4; ++i) tdot_acc<T>(sg, gL[i], i == j ? (T)3 * c1 : -c1, f[i]);
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                if (E[q][0] == j) tdot_acc<T>(sg, gL[E[q][1]], (T)4 * c1, f[4 + q]);
                if (E[q][1] == j) tdot_acc<T>(sg, gL[E[q][0]], (T)4 * c1, f[4 + q]);
            }
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            T g[3] = {gL[E[q][0]][0] + gL[E[q][1]][0], gL[E[q][0]][1] + gL[E[q][1]][1],
                      gL[E[q][0]][2] + gL[E[q][1]][2]};
            tdot_acc<T>(ST, g, (T)(4.0 * QB_), f[4 + q]);
        }
    }
}

template <typename T, int DK, int MODE, bool WAVE_ELEM, int OUT>
__global__ __launch_bounds__(256) void k_ebe(DevMesh M, int MB, int nm, int e0, int e1,
                                            const void* __restrict__ Dv, const double* __restrict__ h,
                                            const double* __restrict__ mat, StepConst sc,
                                            const T* __restrict__ x1, const T* __restrict__ x2,
                                            T* __restrict__ y, const int* __restrict__ active)
{
    long blk = blockIdx.x;
    if (OUT) blk = (blk % 8) * (gridDim.x / 8) + blk / 8;
    const long t = blk * blockDim.x + threadIdx.x;
    const int m = (int)(t % MB);
    long e = e0 + t / MB;
    if (WAVE_ELEM) e = __builtin_amdgcn_readfirstlane((int)e);  // one element per wavefront
    if (e >= e1 || m >= nm) return;
    if (active && !active[m]) return;
    if (!OUT) e = WAVE_ELEM ? __builtin_amdgcn_readfirstlane(M.celem[e]) : M.celem[e];
    const int EB = MB >= 64 ? 1 : 64 / MB;
    size_t nbase[10];
    T f[10][3];
    ebe_element<T, DK, MODE>(M, MB, m, e, Dv, h, mat, sc, x1, x2, f, nbase);
    if (OUT) {
        // row bases are uniform per wavefront when EB == 1; the lane adds m
        T* fb = y + f_index(e, 0, MB, EB, 0);
        const size_t rs = (size_t)EB * MB;
#pragma unroll
        for (int n = 0; n < 10; ++n)
#pragma unroll
            for (int c = 0; c < 3; ++c) (fb + (3 * n + c) * rs)[m] = f[n][c];
    } else {
#pragma unroll
        for (int n = 0; n < 10; ++n) {
            T* yb = y + nbase[n];
#pragma unroll
            for (int c = 0; c < 3; ++c) yb[(uint32_t)(c * MB + m)] += f[n][c];
        }
    }
}

// Cluster form of the operator (members padded to a multiple of 64): a block
// takes one cluster of consecutive storage elements (at most kClusterNodes
// distinct nodes) and 64 members; its four wavefronts compute four elements
// at a time (one element, 64 members per wavefront) and add their forces into
// the cluster's node rows in LDS, wavefront after wavefront, so the order of
// the sums is fixed.  The cluster's node rows are then written to
// co[(row * 3 + c) * MB + m] (row = the cluster's first row + local node) and
// a gather over the node -> rows lists finishes the sum.
// LDS of a cluster block: the node rows, padded so that NB blocks share a CU
// (160 KB of LDS per CU, allocated in 8 KB steps).  With one bfloat16 D per
// element four FP32 blocks per CU run fastest; with D per point four thrash
// the L2 that holds the nodal rows shared by neighbouring clusters and three
// are faster; two leave too few wavefronts to cover latency.
template <typename T, int NB>
constexpr int cluster_lds_elems()
{
    constexpr int rows = kClusterNodes * 3 * 64;
    constexpr int want = (NB == 3 ? 46 * 1024 : (NB == 2 ? 64 * 1024 : 0)) / (int)sizeof(T);
    return want > rows ? want : rows;
}

template <typename T, int DK, int MODE, int NB>
__global__ __launch_bounds__(256) void k_ebe_cluster(DevMesh M, int MB, int nm, int ngroups, int ncl,
                                                    const void* __restrict__ Dv, const double* __restrict__ h,
                                                    const double* __restrict__ mat, StepConst sc,
                                                    const T* __restrict__ x1, const T* __restrict__ x2,
                                                    T* __restrict__ co, const int* __restrict__ active)
{
    __shared__ T ys[cluster_lds_elems<T, NB>()];
    const long blk = (blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8;  // XCD-contiguous clusters
    const int c = (int)(blk / ngroups), g = (int)(blk % ngroups);
    if (c >= ncl) return;  // whole block: padding of the grid to a multiple of 8
    // the wavefront index is uniform: saying so keeps the element's
    // connectivity and row bases in scalar registers (scalar loads and
    // address arithmetic instead of per-lane 64-bit adds)
    const int t = threadIdx.x, lane = t & 63, w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int m = g * 64 + lane;
    const int e0 = M.cl_off[c], nec = M.cl_off[c + 1] - e0;
    const int r0 = M.cl_noff[c], ncn = M.cl_noff[c + 1] - r0;
    for (int i = t; i < ncn * 3 * 64; i += 256) ys[i] = (T)0;
    const bool act = m < nm && (!active || active[m]);
    __syncthreads();
    for (int r = 0; r < nec; r += 4) {
        const int le = r + w;
        T f[10][3];
        if (le < nec && act) {
            size_t nbase[10];
            ebe_element<T, DK, MODE>(M, MB, m, e0 + le, Dv, h, mat, sc, x1, x2, f, nbase);
        } else {
#pragma unroll
            for (int n = 0; n < 10; ++n) f[n][0] = f[n][1] = f[n][2] = (T)0;
        }
        // local node indices, four per 32-bit word (uniform: scalar loads)
        uint32_t lw[3] = {0u, 0u, 0u};
        if (le < nec) {
            const uint32_t* lp = M.cl_lconn + (size_t)(e0 + le) * 4;
            lw[0] = lp[0];
            lw[1] = lp[1];
            lw[2] = lp[2];
        }
        for (int ww = 0; ww < 4; ++ww) {
            __syncthreads();
            if (w == ww && le < nec) {
                // LDS read-add-write (the no-return LDS atomic add measured 3.5x
                // slower for the whole kernel).  An element's ten nodes are
                // distinct rows: all thirty values are read before any is
                // written back, one LDS round trip instead of ten.
                T* yr[10];
                T v[10][3];
#pragma unroll
                for (int n = 0; n < 10; ++n) {
                    yr[n] = ys + (int)((lw[n / 4] >> (8 * (n % 4))) & 0xFFu) * 3 * 64 + lane;
                    v[n][0] = yr[n][0];
                    v[n][1] = yr[n][64];
                    v[n][2] = yr[n][128];
                }
#pragma unroll
                for (int n = 0; n < 10; ++n) {
                    yr[n][0] = v[n][0] + f[n][0];
                    yr[n][64] = v[n][1] + f[n][1];
                    yr[n][128] = v[n][2] + f[n][2];
                }
            }
        }
    }
    __syncthreads();
    for (int i = t; i < ncn * 3 * 64; i += 256) {
        const int q = i >> 6;  // row * 3 + component within the cluster
        co[((size_t)r0 * 3 + q) * MB + g * 64 + (i & 63)] = ys[i];
    }
}

// blocks of the FP32 cluster launches per CU (a tuning knob, per host thread)
static thread_local int t_cluster_blocks = 3;
void set_cluster_blocks(int b) { t_cluster_blocks = (b == 2 || b == 3 || b == 4) ? b : 3; }

template <typename T, int DK, int NB>
static void cluster_dispatch(hipStream_t s, OpMode mode, const DevMesh& M, int MB, int nm, const void* D,
                             const double* h, const double* mat, StepConst sc, const T* x1, const T* x2, T* co,
                             const int* active)
{
    const int ngroups = MB / 64;
    long g = (long)M.ncl * ngroups;
    g = (g + 7) / 8 * 8;
    const dim3 grid((unsigned)g), b(256);
    switch (mode) {
    case OP_A: hipLaunchKernelGGL((k_ebe_cluster<T, DK, OP_A, NB>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x1, x2, co, active); break;
    case OP_K: hipLaunchKernelGGL((k_ebe_cluster<T, DK, OP_K, NB>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x1, x2, co, active); break;
    case OP_M: hipLaunchKernelGGL((k_ebe_cluster<T, DK, OP_M, NB>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x1, x2, co, active); break;
    case OP_RHS: hipLaunchKernelGGL((k_ebe_cluster<T, DK, OP_RHS, NB>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x1, x2, co, active); break;
    }
}

// FP32 operator (A) with D storage DK, NB blocks per CU
template <int DK>
static void cluster32(hipStream_t s, const DevMesh& M, int MB, int nm, const void* D, const double* h,
                      const double* mat, StepConst sc, const float* x, float* co, const int* active)
{
    const int ngroups = MB / 64;
    long g = (long)M.ncl * ngroups;
    g = (g + 7) / 8 * 8;
    const dim3 grid((unsigned)g), b(256);
    const float* none = nullptr;
    switch (t_cluster_blocks) {
    case 2: hipLaunchKernelGGL((k_ebe_cluster<float, DK, OP_A, 2>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x, none, co, active); break;
    case 4: hipLaunchKernelGGL((k_ebe_cluster<float, DK, OP_A, 4>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x, none, co, active); break;
    default: hipLaunchKernelGGL((k_ebe_cluster<float, DK, OP_A, 3>), grid, b, 0, s, M, MB, nm, ngroups, M.ncl, D, h, mat, sc, x, none, co, active); break;
    }
}

void launch_ebe_cluster64(hipStream_t s, OpMode mode, const DevMesh& M, int MB, int nm, const double* D,
                          const double* h, const double* mat, StepConst sc, const double* x1, const double* x2,
                          double* co, const int* active)
{
    // FP64 rows take 72 KB: two blocks per CU
    cluster_dispatch<double, 0, 2>(s, mode, M, MB, nm, D, h, mat, sc, x1, x2, co, active);
}

void launch_ebe_cluster32(hipStream_t s, const DevMesh& M, int MB, int nm, const float* D32, const uint32_t* D16,
                          const double* h, const double* mat, StepConst sc, const float* x, float* co,
                          const int* active, bool d16_mean)
{
    if (D16 && d16_mean) cluster32<4>(s, M, MB, nm, D16, h, mat, sc, x, co, active);
    else if (D16) cluster32<1>(s, M, MB, nm, D16, h, mat, sc, x, co, active);
    else cluster32<0>(s, M, MB, nm, D32, h, mat, sc, x, co, active);
}

// y = sum of the element outputs at each node (incidences in ascending
// order, so the sum is reproducible) + bscale * base (base may be NULL and may
// alias y).  With DOT the per-member partial sums of x . y over the block's
// nodes go to partial[blockIdx * MB + m] (a fixed tree in LDS).  A block takes
// a contiguous range of nodes, 256 / MB nodes per pass (MB <= 256): with nodes
// in Morton order, interleaving the blocks' passes over the whole range was
// 40 % slower (concurrent blocks then read cluster rows of one small region);
// members with active[m] == 0 keep y and add nothing.
template <typename T, bool DOT, bool CL>
__global__ __launch_bounds__(256) void k_gather(DevMesh M, int MB, int nm, const T* __restrict__ f,
                                               const T* base, T bscale, T* y, const int* __restrict__ active,
                                               const T* __restrict__ x, double* __restrict__ partial)
{
    const int t = threadIdx.x, m = t % MB;
    const int rpb = 256 / MB;
    const int slot = t / MB;
    const bool act = m < nm && (!active || active[m]);
    const int EB = MB >= 64 ? 1 : 64 / MB;
    const size_t rs = (size_t)EB * MB;
    double dot = 0.0;
    const long per = ((M.nn + gridDim.x - 1) / gridDim.x + rpb - 1) / rpb * rpb;
    const long n0 = (long)blockIdx.x * per, n1 = n0 + per < M.nn ? n0 + per : M.nn;
    for (long nd = n0 + slot; nd < n1; nd += rpb) {
        const int node = MB >= 64 ? __builtin_amdgcn_readfirstlane((int)nd) : (int)nd;
        if (!act) continue;
        T a0 = 0, a1 = 0, a2 = 0;
        if (CL) {  // cluster rows of the node, ascending
            const int q1 = M.cn_ptr[node + 1];
#pragma unroll 4
            for (int q = M.cn_ptr[node]; q < q1; ++q) {
                const T* fb = f + (size_t)M.cn_row[q] * 3 * MB + m;
                a0 += fb[0];
                a1 += fb[MB];
                a2 += fb[2 * MB];
            }
        } else {  // element outputs of the node, ascending
            const int q1 = M.inc_ptr[node + 1];
#pragma unroll 4
            for (int q = M.inc_ptr[node]; q < q1; ++q) {
                const int ent = M.inc[q];
                const int e = ent / 10, k = ent - 10 * e;
                const T* fb = f + f_index(e, 3 * k, MB, EB, m);
                a0 += fb[0];
                a1 += fb[rs];
                a2 += fb[2 * rs];
            }
        }
        const size_t yi = (size_t)node * 3 * MB + m;
        if (base) {
            a0 += bscale * base[yi];
            a1 += bscale * base[yi + MB];
            a2 += bscale * base[yi + 2 * MB];
        }
        y[yi] = a0;
        y[yi + MB] = a1;
        y[yi + 2 * MB] = a2;
        if (DOT) dot += (double)x[yi] * (double)a0 + (double)x[yi + MB] * (double)a1 + (double)x[yi + 2 * MB] * (double)a2;
    }
    if (DOT) {
        __shared__ double sh[256];
        sh[t] = dot;
        __syncthreads();
        for (int s = 128; s >= MB; s >>= 1) {
            if (t < s) sh[t] += sh[t + s];
            __syncthreads();
        }
        if (t < MB) partial[(size_t)blockIdx.x * MB + t] = sh[t];
    }
}

// blocks of a gather launch: node passes of 256 / MB nodes, at most maxblk
static int gather_blocks(int nn, int MB, int maxblk)
{
    const long rpb = 256 / MB;
    const long g = (nn + rpb - 1) / rpb;
    return (int)(g < 1 ? 1 : (g > maxblk ? maxblk : g));
}

template <typename T>
void launch_gather(hipStream_t s, const DevMesh& M, int MB, int nm, const T* f, const T* base, T bscale, T* y,
                   const int* active, const T* x, double* partial, int* nblk, bool clusters)
{
    if (partial) {
        const int g = gather_blocks(M.nn, MB, kGatherBlocks);
        *nblk = g;
        if (clusters)
            hipLaunchKernelGGL((k_gather<T, true, true>), dim3(g), dim3(256), 0, s, M, MB, nm, f, base, bscale, y,
                               active, x, partial);
        else
            hipLaunchKernelGGL((k_gather<T, true, false>), dim3(g), dim3(256), 0, s, M, MB, nm, f, base, bscale, y,
                               active, x, partial);
    } else {
        const int g = gather_blocks(M.nn, MB, 1 << 24);
        if (clusters)
            hipLaunchKernelGGL((k_gather<T, false, true>), dim3(g), dim3(256), 0, s, M, MB, nm, f, base, bscale, y,
                               active, x, nullptr);
        else
            hipLaunchKernelGGL((k_gather<T, false, false>), dim3(g), dim3(256), 0, s, M, MB, nm, f, base, bscale, y,
                               active, x, nullptr);
    }
}
template void launch_gather<double>(hipStream_t, const DevMesh&, int, int, const double*, const double*, double,
                                    double*, const int*, const double*, double*, int*, bool);
template void launch_gather<float>(hipStream_t, const DevMesh&, int, int, const float*, const float*, float, float*,
                                   const int*, const float*, double*, int*, bool);

// threads per block of the element-by-element launches (a tuning knob; per
// host thread so concurrent contexts do not interfere)
static thread_local int t_ebe_block = 256;
void set_ebe_block(int bs) { t_ebe_block = (bs == 64 || bs == 128 || bs == 256) ? bs : 256; }

// grid of an element launch: OUT launches round up to a multiple of 8 blocks
static dim3 ebe_grid(long n, bool out)
{
    unsigned g = nblocks(n, t_ebe_block);
    if (out) g = (g + 7) / 8 * 8;
    return dim3(g);
}

template <typename T, int DK, int MODE>
static void ebe_dispatch(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const void* D,
                         const double* h, const double* mat, StepConst sc, const T* x1, const T* x2, T* y,
                         const int* active, bool out)
{
    const dim3 g = ebe_grid((long)(e1 - e0) * MB, out), b(t_ebe_block);
    if (MB >= 64) {
        if (out) hipLaunchKernelGGL((k_ebe<T, DK, MODE, true, 1>), g, b, 0, s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active);
        else hipLaunchKernelGGL((k_ebe<T, DK, MODE, true, 0>), g, b, 0, s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active);
    } else {
        if (out) hipLaunchKernelGGL((k_ebe<T, DK, MODE, false, 1>), g, b, 0, s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active);
        else hipLaunchKernelGGL((k_ebe<T, DK, MODE, false, 0>), g, b, 0, s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active);
    }
}

// inner FP32 operator (Eq. 1 left-hand side) with D stored in FP32 or bfloat16
void launch_ebe32(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const float* D32,
                  const uint32_t* D16, const double* h, const double* mat, StepConst sc, const float* x, float* y,
                  const int* active, bool out, bool d16_mean)
{
    if (e1 <= e0) return;
    if (D16 && d16_mean) ebe_dispatch<float, 4, OP_A>(s, M, MB, nm, e0, e1, D16, h, mat, sc, x, nullptr, y, active, out);
    else if (D16) ebe_dispatch<float, 1, OP_A>(s, M, MB, nm, e0, e1, D16, h, mat, sc, x, nullptr, y, active, out);
    else ebe_dispatch<float, 0, OP_A>(s, M, MB, nm, e0, e1, D32, h, mat, sc, x, nullptr, y, active, out);
}

// ---------------------------------------------------------------------------
// convergence tail: once at most G (16 or 32) members are still iterating,
// their CG runs on compact copies, lane k of a row being member tl[1 + k]
// (tl[0] = the count): the member-innermost rows of the full arrays would
// otherwise be fetched whole for a few members each.  The mixed path packs the
// element-mean D, h, the material rows and the FP32 block-Jacobi inverse once
// per outer iteration for its inner CG; the FP64 PCG packs the FP64 D per
// point, h, the material rows, its inverse and the CG vectors once per step.
// The operator sums its element forces per element cluster into compact
// cluster rows, which a gather sums per node into a compact result.  Partial sums keep the full [block][MB] layout (zero for members not
// listed), so the per-member stage logic is the same.
// ---------------------------------------------------------------------------

// rows of a member-innermost array, listed members only: compact row rc of G
// lanes <-> full row r of MB lanes.  With EBc > 1 the rows are W per element
// and the compact copy is blocked by EBc elements (the D layout of G slots).
template <typename T, bool UNPACK>
__global__ __launch_bounds__(256) void k_tail_rows(long nrows, int MB, int G, int W, int EBc,
                                                  const int* __restrict__ tl, const T* __restrict__ src,
                                                  T* __restrict__ dst)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int k = (int)(t % G);
    const long r = t / G;
    if (r >= nrows || k >= min(tl[0], G)) return;
    const int m = tl[1 + k];
    long rc = r;
    if (EBc > 1) {
        const long e = r / W;
        rc = ((e / EBc) * W + (r - e * W)) * EBc + e % EBc;
    }
    if (UNPACK) dst[r * MB + m] = src[rc * G + k];
    else dst[rc * G + k] = src[r * MB + m];
}

template <typename T>
static void tail_rows(hipStream_t s, long nrows, int MB, int G, int W, int EBc, const int* tl, const T* src, T* dst,
                      bool unpack)
{
    const long n = nrows * G;
    if (n <= 0) return;
    if (unpack)
        hipLaunchKernelGGL((k_tail_rows<T, true>), dim3(nblocks(n)), dim3(256), 0, s, nrows, MB, G, W, EBc, tl, src, dst);
    else
        hipLaunchKernelGGL((k_tail_rows<T, false>), dim3(nblocks(n)), dim3(256), 0, s, nrows, MB, G, W, EBc, tl, src, dst);
}

void launch_tail_pack(hipStream_t s, const DevMesh& M, int MB, int G, int n_layers, const int* tl,
                      const uint32_t* D16, const double* h, const double* mat, const float* pinv32, uint32_t* cD,
                      double* ch, double* cmat, float* cpinv)
{
    tail_rows<uint32_t>(s, (long)M.ne * 11, MB, G, 11, 64 / G, tl, D16, cD, false);
    if (h) tail_rows<double>(s, M.ne, MB, G, 1, 1, tl, h, ch, false);
    tail_rows<double>(s, (long)n_layers * MAT_N, MB, G, 1, 1, tl, mat, cmat, false);
    tail_rows<float>(s, (long)M.nn * 6, MB, G, 1, 1, tl, pinv32, cpinv, false);
}

void launch_tail_unpack(hipStream_t s, long nrows, int MB, int G, const int* tl, const float* c, float* full)
{
    tail_rows<float>(s, nrows, MB, G, 1, 1, tl, c, full, true);
}

void launch_tail_pack64(hipStream_t s, const DevMesh& M, int MB, int G, int n_layers, const int* tl,
                        const double* D64, const double* h, const double* mat, const double* pinv, double* cD,
                        double* ch, double* cmat, double* cpinv)
{
    tail_rows<double>(s, (long)M.ne * 84, MB, G, 84, 64 / G, tl, D64, cD, false);
    if (h) tail_rows<double>(s, M.ne, MB, G, 1, 1, tl, h, ch, false);
    tail_rows<double>(s, (long)n_layers * MAT_N, MB, G, 1, 1, tl, mat, cmat, false);
    tail_rows<double>(s, (long)M.nn * 6, MB, G, 1, 1, tl, pinv, cpinv, false);
}

void launch_tail_rows64(hipStream_t s, long nrows, int MB, int G, const int* tl, const double* src, double* dst,
                        bool unpack)
{
    tail_rows<double>(s, nrows, MB, G, 1, 1, tl, src, dst, unpack);
}

// operator A on the compact rows summed per element cluster (the compact form
// of k_ebe_cluster): one block per cluster; a wavefront holds 64/G element
// slots of G lanes, and each slot adds its element's forces into its own copy
// of the cluster's node rows in LDS (the slots of a wavefront run in
// lockstep), the wavefronts one after another; on the way out the copies are
// summed in slot order and written as G-wide cluster rows
// co[(row * 3 + c) * G + k], which the cluster-row gather completes.  The
// order of every sum is fixed.  The cluster rows take about a third of the
// element outputs' bytes, written once and read once.
template <typename T, int DK, int G>
__global__ __launch_bounds__(256) void k_ebe_ctail(DevMesh M, const int* __restrict__ tl, const void* __restrict__ cD,
                                                  const double* __restrict__ ch, const double* __restrict__ cmat,
                                                  StepConst sc, const T* __restrict__ x, T* __restrict__ co)
{
    constexpr int S = 64 / G, SLOTS = 4 * S, ROWS = kClusterNodes * 3 * G;
    __shared__ T ys[S * ROWS];
    const int c = (int)((blockIdx.x % 8) * (gridDim.x / 8) + blockIdx.x / 8);  // XCD-contiguous clusters
    if (c >= M.ncl) return;  // whole block: padding of the grid to a multiple of 8
    const int t = threadIdx.x, k = t % G, slot = t / G, sw = (t & 63) / G;
    const int w = __builtin_amdgcn_readfirstlane(t >> 6);
    const int e0 = M.cl_off[c], nec = M.cl_off[c + 1] - e0;
    const int r0 = M.cl_noff[c], n3 = (M.cl_noff[c + 1] - r0) * 3 * G;
    for (int i = t; i < S * n3; i += 256) ys[(i / n3) * ROWS + i % n3] = (T)0;
    const bool act = k < min(tl[0], G);
    T* yc = ys + sw * ROWS;
    __syncthreads();
    for (int r = 0; r < nec; r += SLOTS) {
        const int le = r + slot;
        T f[10][3];
        if (le < nec && act) {
            size_t nbase[10];
            ebe_element<T, DK, OP_A>(M, G, k, e0 + le, cD, ch, cmat, sc, x, nullptr, f, nbase);
        } else {
#pragma unroll
            for (int n = 0; n < 10; ++n) f[n][0] = f[n][1] = f[n][2] = (T)0;
        }
        uint32_t lw[3] = {0u, 0u, 0u};
        if (le < nec) {
            const uint32_t* lp = M.cl_lconn + (size_t)(e0 + le) * 4;
            lw[0] = lp[0];
            lw[1] = lp[1];
            lw[2] = lp[2];
        }
        for (int ww = 0; ww < 4; ++ww) {
            __syncthreads();
            if (w == ww && le < nec) {
                // the element's ten distinct node rows: all reads before the writes
                T* yr[10];
                T v[10][3];
#pragma unroll
                for (int n = 0; n < 10; ++n) {
                    yr[n] = yc + (int)((lw[n / 4] >> (8 * (n % 4))) & 0xFFu) * 3 * G + k;
                    v[n][0] = yr[n][0];
                    v[n][1] = yr[n][G];
                    v[n][2] = yr[n][2 * G];
                }
#pragma unroll
                for (int n = 0; n < 10; ++n) {
                    yr[n][0] = v[n][0] + f[n][0];
                    yr[n][G] = v[n][1] + f[n][1];
                    yr[n][2 * G] = v[n][2] + f[n][2];
                }
            }
        }
    }
    __syncthreads();
    for (int i = t; i < n3; i += 256) {
        T v = ys[i];
#pragma unroll
        for (int q = 1; q < S; ++q) v += ys[q * ROWS + i];
        co[(size_t)r0 * 3 * G + i] = v;
    }
}

void launch_ebe64_ctail(hipStream_t s, const DevMesh& M, int G, const int* tl, const double* cD, const double* ch,
                        const double* cmat, StepConst sc, const double* x, double* co)
{
    long g = (M.ncl + 7) / 8 * 8;
    if (M.ncl <= 0) return;
    if (G == 16)
        hipLaunchKernelGGL((k_ebe_ctail<double, 0, 16>), dim3((unsigned)g), dim3(256), 0, s, M, tl, cD, ch, cmat, sc, x,
                           co);
    else
        hipLaunchKernelGGL((k_ebe_ctail<double, 0, 32>), dim3((unsigned)g), dim3(256), 0, s, M, tl, cD, ch, cmat, sc, x,
                           co);
}

void launch_ebe32_ctail(hipStream_t s, const DevMesh& M, int G, const int* tl, const uint32_t* cD, const double* ch,
                        const double* cmat, StepConst sc, const float* x, float* co)
{
    long g = (M.ncl + 7) / 8 * 8;
    if (M.ncl <= 0) return;
    if (G == 16)
        hipLaunchKernelGGL((k_ebe_ctail<float, 4, 16>), dim3((unsigned)g), dim3(256), 0, s, M, tl, cD, ch, cmat, sc, x,
                           co);
    else
        hipLaunchKernelGGL((k_ebe_ctail<float, 4, 32>), dim3((unsigned)g), dim3(256), 0, s, M, tl, cD, ch, cmat, sc, x,
                           co);
}

// node sums of compact element outputs (incidences in ascending order) or,
// with CL, of the compact cluster rows (the node's rows in ascending order;
// the form the operators write) into the compact y of the listed, active
// members; with partial, the x . y partials of the block's nodes
template <typename T, int G, bool CL>
__global__ __launch_bounds__(256) void k_gather_tail(DevMesh M, int MB, int nm, const int* __restrict__ tl,
                                                    const T* __restrict__ fc, T* __restrict__ y,
                                                    const int* __restrict__ active, const T* __restrict__ x,
                                                    double* __restrict__ partial)
{
    constexpr int NPB = 256 / G;  // nodes per block pass
    const int t = threadIdx.x, k = t % G, slot = t / G;
    const int m = k < min(tl[0], G) ? tl[1 + k] : -1;
    const bool act = m >= 0 && m < nm && (!active || active[m]);
    double dot = 0.0;
    const long per = ((M.nn + gridDim.x - 1) / gridDim.x + NPB - 1) / NPB * NPB;
    const long n0 = (long)blockIdx.x * per, n1 = n0 + per < M.nn ? n0 + per : M.nn;
    if (act) {
        for (long nd = n0 + slot; nd < n1; nd += NPB) {
            T a0 = 0, a1 = 0, a2 = 0;
            if (CL) {
                const int q1 = M.cn_ptr[nd + 1];
#pragma unroll 4
                for (int q = M.cn_ptr[nd]; q < q1; ++q) {
                    const T* fb = fc + (size_t)3 * M.cn_row[q] * G + k;
                    a0 += fb[0];
                    a1 += fb[G];
                    a2 += fb[2 * G];
                }
            } else {
                const int q1 = M.inc_ptr[nd + 1];
#pragma unroll 4
                for (int q = M.inc_ptr[nd]; q < q1; ++q) {
                    // incidence e * 10 + local node: its output rows start at 3 * incidence
                    const T* fb = fc + (size_t)3 * M.inc[q] * G + k;
                    a0 += fb[0];
                    a1 += fb[G];
                    a2 += fb[2 * G];
                }
            }
            const size_t yi = (size_t)nd * 3 * G + k;
            y[yi] = a0;
            y[yi + G] = a1;
            y[yi + 2 * G] = a2;
            if (partial)
                dot += (double)x[yi] * (double)a0 + (double)x[yi + G] * (double)a1 + (double)x[yi + 2 * G] * (double)a2;
        }
    }
    if (partial) {
        double acc[1] = {dot};
        tail_partials<1, G>(acc, MB, m, partial, 0, gridDim.x);
    }
}

template <typename T>
void launch_gather_tail(hipStream_t s, const DevMesh& M, int MB, int nm, int G, const int* tl, const T* fc, T* y,
                        const int* active, const T* x, double* partial, int* nblk, bool clusters)
{
    const int g = gather_blocks(M.nn, G, partial ? kGatherBlocks : (1 << 24));
    if (partial) *nblk = g;
    if (clusters) {
        if (G == 16)
            hipLaunchKernelGGL((k_gather_tail<T, 16, true>), dim3(g), dim3(256), 0, s, M, MB, nm, tl, fc, y, active, x,
                               partial);
        else
            hipLaunchKernelGGL((k_gather_tail<T, 32, true>), dim3(g), dim3(256), 0, s, M, MB, nm, tl, fc, y, active, x,
                               partial);
    } else {
        if (G == 16)
            hipLaunchKernelGGL((k_gather_tail<T, 16, false>), dim3(g), dim3(256), 0, s, M, MB, nm, tl, fc, y, active, x,
                               partial);
        else
            hipLaunchKernelGGL((k_gather_tail<T, 32, false>), dim3(g), dim3(256), 0, s, M, MB, nm, tl, fc, y, active, x,
                               partial);
    }
}
template void launch_gather_tail<float>(hipStream_t, const DevMesh&, int, int, int, const int*, const float*, float*,
                                        const int*, const float*, double*, int*, bool);
template void launch_gather_tail<double>(hipStream_t, const DevMesh&, int, int, int, const int*, const double*,
                                         double*, const int*, const double*, double*, int*, bool);

template <typename T>
void launch_ebe(hipStream_t s, OpMode mode, const DevMesh& M, int MB, int nm, int e0, int e1, const T* D,
                const double* h, const double* mat, int, StepConst sc, const T* x1, const T* x2, T* y,
                const int* active, bool out)
{
    if (e1 <= e0) return;
    switch (mode) {
    case OP_A: ebe_dispatch<T, 0, OP_A>(s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active, out); break;
    case OP_K: ebe_dispatch<T, 0, OP_K>(s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active, out); break;
    case OP_M: ebe_dispatch<T, 0, OP_M>(s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active, out); break;
    case OP_RHS: ebe_dispatch<T, 0, OP_RHS>(s, M, MB, nm, e0, e1, D, h, mat, sc, x1, x2, y, active, out); break;
    }
}
template void launch_ebe<double>(hipStream_t, OpMode, const DevMesh&, int, int, int, int, const double*,
                                 const double*, const double*, int, StepConst, const double*,
                                 const double*, double*, const int*, bool);

// ---------------------------------------------------------------------------
// absorbing boundary: node-centric gather over boundary faces (deterministic)
// dashpot on a face: rho (Vp n n^T + Vs (I - n n^T)) times int N_a N_b dA
// ---------------------------------------------------------------------------

// dashpot force at boundary node i (index into the boundary-node lists) for
// member m: coef * sum over its faces of rho (Vp n n^T + Vs (I - n n^T)) int N_a N_b dA x_b,
// plus, with vI, the incident-wave force 2 C_base v_I on base faces
template <typename T>
__device__ __forceinline__ void dashpot_at(const DevMesh& M, int MB, int m, int i, const double* __restrict__ mat,
                                           double coef, const T* __restrict__ x, const double* __restrict__ vI,
                                           double acc[3])
{
    for (int q = M.bn_ptr[i]; q < M.bn_ptr[i + 1]; ++q) {
        const int f = M.bn_face[q], a = M.bn_loc[q];
        const int l = M.f_layer[f];
        const double rho = matv(mat, l, MAT_RHO, MB, m);
        const double vs = matv(mat, l, MAT_VS, MB, m);
        const double vp = matv(mat, l, MAT_VP, MB, m);
        const double* nv = M.f_n + 3 * (long)f;
        double X[3] = {0, 0, 0}, rs = 0;
        for (int b = 0; b < 6; ++b) {
            const double Mab = M.f_M[36 * (long)f + 6 * a + b];
            const long nb = M.f_node[6 * (long)f + b];
            rs += Mab;
            for (int c = 0; c < 3; ++c) X[c] += Mab * (double)x[(nb * 3 + c) * MB + m];
        }
        double nx = nv[0] * X[0] + nv[1] * X[1] + nv[2] * X[2];
        for (int c = 0; c < 3; ++c) acc[c] += coef * rho * (vs * X[c] + (vp - vs) * nx * nv[c]);
        if (vI && M.f_kind[f] == 0) {  // incident wave: 2 C_base v_I
            double V[3] = {vI[0 * MB + m], vI[1 * MB + m], vI[2 * MB + m]};
            double nV = nv[0] * V[0] + nv[1] * V[1] + nv[2] * V[2];
            for (int c = 0; c < 3; ++c) acc[c] += 2.0 * rs * rho * (vs * V[c] + (vp - vs) * nV * nv[c]);
        }
    }
}

// y += dashpot at the boundary nodes; with DOT also the per-member partial
// sums of x . (dashpot x) over the block's nodes, written to
// partial[(boff + blockIdx) * MB + m] (a fixed tree in LDS).  Lane t of a
// block takes member t % MB of boundary node (block pass) * (256 / MB) + t / MB
// when MB <= 256 (a grid-stride loop over the nodes); wider ensembles (no DOT)
// map one (node, member) pair per thread.
template <typename T, bool DOT>
__global__ __launch_bounds__(256) void k_dashpot(DevMesh M, int MB, int nm, const double* __restrict__ mat, double coef,
                                                const T* __restrict__ x, T* __restrict__ y,
                                                const double* __restrict__ vI, const int* __restrict__ active,
                                                double* __restrict__ partial, int boff)
{
    const int t = threadIdx.x;
    int m;
    long first, stride;
    if (MB <= 256) {
        m = t % MB;
        first = (long)blockIdx.x * (256 / MB) + t / MB;
        stride = (long)gridDim.x * (256 / MB);
    } else {
        const long g = (long)blockIdx.x * 256 + t;
        m = (int)(g % MB);
        first = g / MB;
        stride = M.nbn;  // one pair per thread
    }
    const bool act = m < nm && (!active || active[m]);
    double dot = 0.0;
    for (long i = first; i < M.nbn; i += stride) {
        if (!act) continue;
        const int node = M.bn_node[i];
        double acc[3] = {0, 0, 0};
        dashpot_at<T>(M, MB, m, (int)i, mat, coef, x, vI, acc);
        for (int c = 0; c < 3; ++c) {
            const size_t yi = ((size_t)node * 3 + c) * MB + m;
            y[yi] += (T)acc[c];
            if (DOT) dot += (double)x[yi] * (double)(T)acc[c];
        }
    }
    if (DOT) {
        __shared__ double sh[256];
        sh[t] = dot;
        __syncthreads();
        for (int s = 128; s >= MB; s >>= 1) {
            if (t < s) sh[t] += sh[t + s];
            __syncthreads();
        }
        if (t < MB) partial[((size_t)boff + blockIdx.x) * MB + t] = sh[t];
    }
}

template <typename T>
void launch_dashpot(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int, T coef, const T* x,
                    T* y, const double* vI, const int* active, double* partial, int* nblk)
{
    if (M.nbn <= 0) return;
    if (partial && MB <= 256) {
        // appended to the *nblk partials already written (same layout)
        const long rpb = 256 / MB;
        long g = ((long)M.nbn + rpb - 1) / rpb;
        g = g < kDashpotBlocks ? g : kDashpotBlocks;
        hipLaunchKernelGGL((k_dashpot<T, true>), dim3(g), dim3(256), 0, s, M, MB, nm, mat, (double)coef, x, y, vI,
                           active, partial, *nblk);
        *nblk += (int)g;
        return;
    }
    const long g = MB <= 256 ? ((long)M.nbn + 256 / MB - 1) / (256 / MB) : ((long)M.nbn * MB + 255) / 256;
    hipLaunchKernelGGL((k_dashpot<T, false>), dim3(g), dim3(256), 0, s, M, MB, nm, mat, (double)coef, x, y, vI,
                       active, nullptr, 0);
}
template void launch_dashpot<double>(hipStream_t, const DevMesh&, int, int, const double*, int, double,
                                     const double*, double*, const double*, const int*, double*, int*);
template void launch_dashpot<float>(hipStream_t, const DevMesh&, int, int, const double*, int, float,
                                    const float*, float*, const double*, const int*, double*, int*);

// dashpot of the compact rows (material rows packed, lane k = member tl[1 + k]):
// y += coef C x at the boundary nodes for the listed, active members; partials
// of x . (C x) appended after the boff blocks already written
template <typename T, int G>
__global__ __launch_bounds__(256) void k_dashpot_tail(DevMesh M, int MB, int nm, const int* __restrict__ tl,
                                                     const double* __restrict__ cmat, double coef,
                                                     const T* __restrict__ x, T* __restrict__ y,
                                                     const int* __restrict__ active, double* __restrict__ partial,
                                                     int boff, int nblk)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = k < min(tl[0], G) ? tl[1 + k] : -1;
    const bool act = m >= 0 && m < nm && (!active || active[m]);
    double dot = 0.0;
    if (act) {
        for (long i = (long)blockIdx.x * NPB + t / G; i < M.nbn; i += (long)gridDim.x * NPB) {
            const int node = M.bn_node[i];
            double acc[3] = {0, 0, 0};
            dashpot_at<T>(M, G, k, (int)i, cmat, coef, x, nullptr, acc);
            for (int c = 0; c < 3; ++c) {
                const size_t yi = ((size_t)node * 3 + c) * G + k;
                y[yi] += (T)acc[c];
                if (partial) dot += (double)x[yi] * (double)(T)acc[c];
            }
        }
    }
    if (partial) {
        double a1[1] = {dot};
        tail_partials<1, G>(a1, MB, m, partial, boff, nblk);
    }
}

template <typename T>
void launch_dashpot_tail(hipStream_t s, const DevMesh& M, int MB, int nm, int G, const int* tl, const double* cmat,
                         T coef, const T* x, T* y, const int* active, double* partial, int* nblk)
{
    if (M.nbn <= 0) return;
    const long rpb = 256 / G;
    long g = ((long)M.nbn + rpb - 1) / rpb;
    g = g < kDashpotBlocks ? g : kDashpotBlocks;
    const int boff = partial ? *nblk : 0;
    // the partials of one part: rows boff .. boff + g of the gather's layout,
    // so the row count passed as nblk is irrelevant for part 0
    if (G == 16)
        hipLaunchKernelGGL((k_dashpot_tail<T, 16>), dim3(g), dim3(256), 0, s, M, MB, nm, tl, cmat, (double)coef, x, y,
                           active, partial, boff, 0);
    else
        hipLaunchKernelGGL((k_dashpot_tail<T, 32>), dim3(g), dim3(256), 0, s, M, MB, nm, tl, cmat, (double)coef, x, y,
                           active, partial, boff, 0);
    if (partial) *nblk += (int)g;
}
template void launch_dashpot_tail<float>(hipStream_t, const DevMesh&, int, int, int, const int*, const double*, float,
                                         const float*, float*, const int*, double*, int*);
template void launch_dashpot_tail<double>(hipStream_t, const DevMesh&, int, int, int, const int*, const double*,
                                          double, const double*, double*, const int*, double*, int*);

// dashpot rows of the boundary nodes for the fused Chebyshev gather:
// qb[(i * 3 + c) * MB + m] = (dashpot x)(boundary node i), active members only
__global__ __launch_bounds__(256) void k_dashpot_rows(DevMesh M, int MB, int nm, const double* __restrict__ mat,
                                                     double coef, const float* __restrict__ x,
                                                     float* __restrict__ qb, const int* __restrict__ active)
{
    const int t = threadIdx.x, m = t % MB;
    const long first = (long)blockIdx.x * (256 / MB) + t / MB, stride = (long)gridDim.x * (256 / MB);
    if (m >= nm || (active && !active[m])) return;
    for (long i = first; i < M.nbn; i += stride) {
        double acc[3] = {0, 0, 0};
        dashpot_at<float>(M, MB, m, (int)i, mat, coef, x, nullptr, acc);
#pragma unroll
        for (int c = 0; c < 3; ++c) qb[((size_t)i * 3 + c) * MB + m] = (float)acc[c];
    }
}

void launch_dashpot_rows(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, float coef,
                         const float* x, float* qb, const int* active)
{
    if (M.nbn <= 0) return;
    const long g = ((long)M.nbn + 256 / MB - 1) / (256 / MB);  // MB <= 256 on the cluster path
    hipLaunchKernelGGL(k_dashpot_rows, dim3(g), dim3(256), 0, s, M, MB, nm, mat, (double)coef, x, qb, active);
}

// One fused Chebyshev iteration on the cluster path (MB = 64..256): per node
// the cluster rows are summed in ascending order (as the gather does), the
// boundary nodes add their dashpot row, and with q = that sum
//   iz += id,  ir -= q,  id_next = c1_k id + c2_k P ir   (no id_next on the last)
// so the operator result never goes to memory.  Node ranges per block as in
// the gather.
__global__ __launch_bounds__(256) void k_gather_cheb(DevMesh M, int MB, int nm, int k, int last,
                                                    const float* __restrict__ rows, const float* __restrict__ qb,
                                                    float* __restrict__ iz, float* __restrict__ ir,
                                                    const float* __restrict__ id, float* __restrict__ id_next,
                                                    const float* __restrict__ pinv32, const float* __restrict__ cheb,
                                                    const int* __restrict__ active)
{
    const int t = threadIdx.x, m = t % MB;
    const int rpb = 256 / MB;
    const int slot = t / MB;
    const bool act = m < nm && (!active || active[m]);
    if (!act) return;
    float c1 = 0.0f, c2 = 0.0f;
    if (!last) {
        c1 = cheb[(long)(2 * k) * MB + m];
        c2 = cheb[(long)(2 * k + 1) * MB + m];
    }
    const long per = ((M.nn + gridDim.x - 1) / gridDim.x + rpb - 1) / rpb * rpb;
    const long n0 = (long)blockIdx.x * per, n1 = n0 + per < M.nn ? n0 + per : M.nn;
    for (long nd = n0 + slot; nd < n1; nd += rpb) {
        const int node = __builtin_amdgcn_readfirstlane((int)nd);
        float a0 = 0, a1 = 0, a2 = 0;
        const int q1 = M.cn_ptr[node + 1];
#pragma unroll 4
        for (int q = M.cn_ptr[node]; q < q1; ++q) {
            const float* fb = rows + (size_t)M.cn_row[q] * 3 * MB + m;
            a0 += fb[0];
            a1 += fb[MB];
            a2 += fb[2 * MB];
        }
        const int bi = M.bn_of_node[node];
        if (bi >= 0) {
            const float* qp = qb + (size_t)bi * 3 * MB + m;
            a0 += qp[0];
            a1 += qp[MB];
            a2 += qp[2 * MB];
        }
        const size_t yi = (size_t)node * 3 * MB + m;
        const float d0 = id[yi], d1 = id[yi + MB], d2 = id[yi + 2 * MB];
        iz[yi] += d0;
        iz[yi + MB] += d1;
        iz[yi + 2 * MB] += d2;
        const float r0 = ir[yi] - a0, r1 = ir[yi + MB] - a1, r2 = ir[yi + 2 * MB] - a2;
        ir[yi] = r0;
        ir[yi + MB] = r1;
        ir[yi + 2 * MB] = r2;
        if (last) continue;
        const float* pv = pinv32 + (size_t)node * 6 * MB + m;
        const float p0 = pv[0], p1 = pv[MB], p2 = pv[2 * MB], p3 = pv[3 * MB], p4 = pv[4 * MB], p5 = pv[5 * MB];
        const float w0 = p0 * r0 + p1 * r1 + p2 * r2;
        const float w1 = p1 * r0 + p3 * r1 + p4 * r2;
        const float w2 = p2 * r0 + p4 * r1 + p5 * r2;
        id_next[yi] = c1 * d0 + c2 * w0;
        id_next[yi + MB] = c1 * d1 + c2 * w1;
        id_next[yi + 2 * MB] = c1 * d2 + c2 * w2;
    }
}

void launch_gather_cheb(hipStream_t s, const DevMesh& M, int MB, int nm, int k, bool last, const float* rows,
                        const float* qb, float* iz, float* ir, const float* id, float* id_next, const float* pinv32,
                        const float* cheb, const int* active)
{
    const int g = gather_blocks(M.nn, MB, 1 << 24);
    hipLaunchKernelGGL(k_gather_cheb, dim3(g), dim3(256), 0, s, M, MB, nm, k, (int)last, rows, qb, iz, ir, id, id_next,
                       pinv32, cheb, active);
}

// ---------------------------------------------------------------------------
// 3x3 block-Jacobi preconditioner (Section 2.2): diagonal blocks of A
// ---------------------------------------------------------------------------

// Diagonal 3x3 block of node n of one element:
//   c_M rho V Mref(n, n) I + c_K (V/4) sum_j B_n(j)^T D_j B_n(j)
// with B_n^T D B_n [c][d] = sum_{p,q} g_p g_q D[v(c, p)][v(d, q)], g = grad N_n
// at point j and v(c, p) the Voigt index of du_c/dx_p.  Per point the 6 x 6
// coefficients of the quadratic forms in (gx^2, gy^2, gz^2, gx gy, gy gz, gz gx)
// are formed once and shared by the nodes.  A thread takes one element-member
// and one part of the nodes (the 4 corners, edges 01 12 20, or edges 03 13
// 23), so it holds at most 4 blocks: FP64 register pressure sets the
// occupancy here, and each part re-reads D (from L2).
__device__ __forceinline__ constexpr int voigt_of(int c, int p)
{
    return c == p ? c : ((c + p == 1) ? 3 : ((c + p == 3) ? 4 : 5));
}

// adds w g^T C g (the 6 entries of the symmetric 3x3 block) for node n (a
// compile-time index after unrolling) with g = grad N_n at barycentrics L
__device__ __forceinline__ void diag_node_add(int n, const double L[4], const double gL[4][3], const double C[6][6],
                                              double w, double acc[6])
{
    constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
    double g[3];
    if (n < 4) {
#pragma unroll
        for (int a = 0; a < 3; ++a) g[a] = (4.0 * L[n] - 1.0) * gL[n][a];
    } else {
        const int ea = E[n - 4][0], eb = E[n - 4][1];
#pragma unroll
        for (int a = 0; a < 3; ++a) g[a] = 4.0 * (L[ea] * gL[eb][a] + L[eb] * gL[ea][a]);
    }
    const double gg[6] = {g[0] * g[0], g[1] * g[1], g[2] * g[2], g[0] * g[1], g[1] * g[2], g[2] * g[0]};
#pragma unroll
    for (int cd = 0; cd < 6; ++cd) {
        double a = 0.0;
#pragma unroll
        for (int pq = 0; pq < 6; ++pq) a += gg[pq] * C[cd][pq];
        acc[cd] += w * a;
    }
}

__global__ __launch_bounds__(256) void k_diag(DevMesh M, int MB, int nm, int e0, int e1,
                                             const double* __restrict__ D, const double* __restrict__ h,
                                             const double* __restrict__ mat, StepConst sc,
                                             double* __restrict__ diag)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(t % MB);
    long r = t / MB;
    if (MB >= 64) r = __builtin_amdgcn_readfirstlane((int)r);  // wavefront-uniform element and part
    const int part = (int)(r % 3);
    const long pos = e0 + r / 3;  // position in the colour lists
    if (pos >= e1 || m >= nm) return;
    const long e = MB >= 64 ? (long)__builtin_amdgcn_readfirstlane(M.celem[pos]) : (long)M.celem[pos];
    const long ne = M.ne;
    double gL[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) gL[k / 3][k % 3] = M.geo64[k * ne + e];
    const double vol = M.geo64[12 * ne + e];
    const int l = M.layer[e];
    const double rho = matv(mat, l, MAT_RHO, MB, m);
    double he = 0.0;
    if (sc.damping_mode == 0 && h) he = h[e * MB + m];
    else if (sc.damping_mode == 1) he = sc.h0;
    const double dt = sc.dt;
    const double sm = rho * vol * (4.0 / (dt * dt) + 2.0 * sc.ahat * he / dt);
    const double w = (1.0 + 2.0 * sc.bhat * he / dt) * vol * 0.25;
    constexpr int PQ[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {2, 0}};
    constexpr int CD[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    double blk[4][6];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < 6; ++k) blk[i][k] = 0.0;
    const int EB = MB >= 64 ? 1 : 64 / MB;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {
        double C[6][6];  // C[cd][pq]
        {
            double d[21];
            const double* Dj = D + d_index(e, j, 0, MB, EB, 0);  // uniform when MB >= 64
            const uint32_t rs = (uint32_t)(EB * MB);
#pragma unroll
            for (int k = 0; k < 21; ++k) d[k] = ld_u(Dj, (uint32_t)k * rs + (uint32_t)m);
#pragma unroll
            for (int cd = 0; cd < 6; ++cd)
#pragma unroll
                for (int pq = 0; pq < 6; ++pq) {
                    const int c = CD[cd][0], dd = CD[cd][1], p = PQ[pq][0], q = PQ[pq][1];
                    double v = d[sym6(voigt_of(c, p), voigt_of(dd, q))];
                    if (p != q) v += d[sym6(voigt_of(c, q), voigt_of(dd, p))];
                    C[cd][pq] = v;
                }
        }
        double L[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) L[i] = (i == j) ? QA_ : QB_;
        if (part == 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) diag_node_add(i, L, gL, C, w, blk[i]);
        } else if (part == 1) {
#pragma unroll
            for (int i = 0; i < 3; ++i) diag_node_add(4 + i, L, gL, C, w, blk[i]);
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i) diag_node_add(7 + i, L, gL, C, w, blk[i]);
        }
    }
    const int nn = part == 0 ? 4 : 3, n0 = part == 0 ? 0 : 1 + 3 * part;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= nn) break;
        const int n = n0 + i;
        const long node = M.conn[n * ne + e];
        const double md = sm * mass_ref(n, n);
        double* dg = diag + node * 6 * MB;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            double& o = *reinterpret_cast<double*>(reinterpret_cast<char*>(dg) + (uint32_t)(k * MB + m) * 8u);
            o += blk[i][k] + ((k == 0 || k == 3 || k == 5) ? md : 0.0);
        }
    }
}

// Diagonal blocks of the inner operator (one D per element, the bfloat16
// element mean): with D constant over the element the stiffness block of
// node n is C : int grad N_n grad N_n^T dV, and that integral has a closed
// form in the barycentric gradients g (int L_a^2 = V/10, int L_a L_b = V/20,
// int L_a = V/4): corner a 0.6 V g_a g_a^T; edge (a, b)
// 1.6 V (g_a g_a^T + g_b g_b^T) + 0.8 V (g_a g_b^T + g_b g_a^T).  One lane
// per element-member of a colour (the colour's elements share no node).
__global__ __launch_bounds__(256) void k_diag_mean(DevMesh M, int MB, int nm, int e0, int e1,
                                                  const uint32_t* __restrict__ D16, const double* __restrict__ h,
                                                  const double* __restrict__ mat, StepConst sc,
                                                  double* __restrict__ diag)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(t % MB);
    long r = t / MB;
    if (MB >= 64) r = __builtin_amdgcn_readfirstlane((int)r);
    const long pos = e0 + r;
    if (pos >= e1 || m >= nm) return;
    const long e = MB >= 64 ? (long)__builtin_amdgcn_readfirstlane(M.celem[pos]) : (long)M.celem[pos];
    const long ne = M.ne;
    double gL[4][3];
#pragma unroll
    for (int k = 0; k < 12; ++k) gL[k / 3][k % 3] = M.geo64[k * ne + e];
    const double vol = M.geo64[12 * ne + e];
    const int l = M.layer[e];
    const double rho = matv(mat, l, MAT_RHO, MB, m);
    double he = 0.0;
    if (sc.damping_mode == 0 && h) he = h[e * MB + m];
    else if (sc.damping_mode == 1) he = sc.h0;
    const double dt = sc.dt;
    const double sm = rho * vol * (4.0 / (dt * dt) + 2.0 * sc.ahat * he / dt);
    const double sk = (1.0 + 2.0 * sc.bhat * he / dt) * vol;
    constexpr int PQ[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {1, 2}, {2, 0}};
    constexpr int CD[6][2] = {{0, 0}, {0, 1}, {0, 2}, {1, 1}, {1, 2}, {2, 2}};
    constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
    const int EB = MB >= 64 ? 1 : 64 / MB;
    double C[6][6];
    {
        double d[22];
#pragma unroll
        for (int q = 0; q < 11; ++q) {
            const uint32_t wv = D16[d16m_index(e, q, MB, EB, m)];
            d[2 * q] = (double)bf2f(wv & 0xFFFFu);
            d[2 * q + 1] = (double)bf2f(wv >> 16);
        }
#pragma unroll
        for (int cd = 0; cd < 6; ++cd)
#pragma unroll
            for (int pq = 0; pq < 6; ++pq) {
                const int c = CD[cd][0], dd = CD[cd][1], p = PQ[pq][0], q = PQ[pq][1];
                double v = d[sym6(voigt_of(c, p), voigt_of(dd, q))];
                if (p != q) v += d[sym6(voigt_of(c, q), voigt_of(dd, p))];
                C[cd][pq] = v;
            }
    }
#pragma unroll
    for (int n = 0; n < 10; ++n) {
        double G[6];  // int d_p N_n d_q N_n dV / V in the PQ order
        if (n < 4) {
#pragma unroll
            for (int pq = 0; pq < 6; ++pq) G[pq] = 0.6 * gL[n][PQ[pq][0]] * gL[n][PQ[pq][1]];
        } else {
            const int a = E[n - 4][0], b = E[n - 4][1];
#pragma unroll
            for (int pq = 0; pq < 6; ++pq) {
                const int p = PQ[pq][0], q = PQ[pq][1];
                G[pq] = 1.6 * (gL[a][p] * gL[a][q] + gL[b][p] * gL[b][q]) +
                        0.8 * (gL[a][p] * gL[b][q] + gL[b][p] * gL[a][q]);
            }
        }
        const long node = M.conn[n * ne + e];
        const double md = sm * mass_ref(n, n);
        double* dg = diag + node * 6 * MB;
#pragma unroll
        for (int cd = 0; cd < 6; ++cd) {
            double a = 0.0;
#pragma unroll
            for (int pq = 0; pq < 6; ++pq) a += G[pq] * C[cd][pq];
            double& o = *reinterpret_cast<double*>(reinterpret_cast<char*>(dg) + (uint32_t)(cd * MB + m) * 8u);
            o += sk * a + ((cd == 0 || cd == 3 || cd == 5) ? md : 0.0);
        }
    }
}

void launch_diag_mean(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const uint32_t* D16,
                      const double* h, const double* mat, StepConst sc, double* diag)
{
    const long n = (long)(e1 - e0) * MB;
    if (n > 0) hipLaunchKernelGGL(k_diag_mean, dim3(nblocks(n)), dim3(256), 0, s, M, MB, nm, e0, e1, D16, h, mat, sc, diag);
}

void launch_diag(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int e1, const double* D, const double* h,
                 const double* mat, int, StepConst sc, double* diag)
{
    long n = (long)(e1 - e0) * 3 * MB;
    if (n > 0) hipLaunchKernelGGL(k_diag, dim3(nblocks(n)), dim3(256), 0, s, M, MB, nm, e0, e1, D, h, mat, sc, diag);
}

__global__ void k_diag_dashpot(DevMesh M, int MB, int nm, const double* __restrict__ mat, double coef,
                               double* __restrict__ diag)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(t % MB);
    const long i = t / MB;
    if (i >= M.nbn || m >= nm) return;
    const long node = M.bn_node[i];
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int q = M.bn_ptr[i]; q < M.bn_ptr[i + 1]; ++q) {
        const int f = M.bn_face[q], a = M.bn_loc[q];
        const int l = M.f_layer[f];
        const double rho = matv(mat, l, MAT_RHO, MB, m);
        const double vs = matv(mat, l, MAT_VS, MB, m);
        const double vp = matv(mat, l, MAT_VP, MB, m);
        const double* n = M.f_n + 3 * (long)f;
        const double Maa = M.f_M[36 * (long)f + 7 * a] * coef * rho;
        acc[0] += Maa * (vs + (vp - vs) * n[0] * n[0]);
        acc[1] += Maa * ((vp - vs) * n[0] * n[1]);
        acc[2] += Maa * ((vp - vs) * n[0] * n[2]);
        acc[3] += Maa * (vs + (vp - vs) * n[1] * n[1]);
        acc[4] += Maa * ((vp - vs) * n[1] * n[2]);
        acc[5] += Maa * (vs + (vp - vs) * n[2] * n[2]);
    }
    for (int k = 0; k < 6; ++k) diag[(node * 6 + k) * MB + m] += acc[k];
}

void launch_diag_dashpot(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int, double coef,
                         double* diag)
{
    long n = (long)M.nbn * MB;
    if (n > 0) hipLaunchKernelGGL(k_diag_dashpot, dim3(nblocks(n)), dim3(256), 0, s, M, MB, nm, mat, coef, diag);
}

__global__ void k_invert_diag(int nn, int MB, int nm, const double* __restrict__ diag,
                              double* __restrict__ pinv, float* __restrict__ pinv32)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(t % MB);
    const long i = t / MB;
    if (i >= nn || m >= nm) return;
    double a[6];
    for (int k = 0; k < 6; ++k) a[k] = diag[(i * 6 + k) * MB + m];
    // a = [a0 a1 a2; a1 a3 a4; a2 a4 a5]
    const double c00 = a[3] * a[5] - a[4] * a[4];
    const double c01 = a[2] * a[4] - a[1] * a[5];
    const double c02 = a[1] * a[4] - a[2] * a[3];
    const double c11 = a[0] * a[5] - a[2] * a[2];
    const double c12 = a[1] * a[2] - a[0] * a[4];
    const double c22 = a[0] * a[3] - a[1] * a[1];
    const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
    double inv[6] = {0, 0, 0, 0, 0, 0};
    if (det != 0.0) {
        const double r = 1.0 / det;
        inv[0] = c00 * r; inv[1] = c01 * r; inv[2] = c02 * r;
        inv[3] = c11 * r; inv[4] = c12 * r; inv[5] = c22 * r;
    }
    for (int k = 0; k < 6; ++k) {
        pinv[(i * 6 + k) * MB + m] = inv[k];
        if (pinv32) pinv32[(i * 6 + k) * MB + m] = (float)inv[k];
    }
}

void launch_invert_diag(hipStream_t s, int nn, int MB, int nm, const double* diag, double* pinv, float* pinv32)
{
    long n = (long)nn * MB;
    if (n > 0) hipLaunchKernelGGL(k_invert_diag, dim3(nblocks(n)), dim3(256), 0, s, nn, MB, nm, diag, pinv, pinv32);
}

// ---------------------------------------------------------------------------
// multi-spring law (Section 2.1): modified Ramberg-Osgood skeleton + Masing
// ---------------------------------------------------------------------------

// normalised skeleton inverse: s with s (1 + |2s|^beta) = e.  Newton in FP32
// (hardware log2/exp2 and reciprocal) from the upper bound
// min(|e|, (|e| / 2^beta)^(1/(1+beta))), on which the iteration decreases
// monotonically, then in FP64 until the step is below 2^-44 |s|.  The FP64
// power is evaluated once, p0 = (2 s0)^beta at the FP32 root s0, and at the
// later iterates s = s0 (1 + d) as p0 (1 + d)^beta from its series, which is
// exact to rounding for |d| < 1e-4 (the FP32 root is good to ~1e-7).  The FP64
// steps divide by the derivative at s0 (a chord step: it differs from the
// derivative at s by ~1e-7 relative, so each step still squares the error to
// rounding; two steps in the usual case).  *pw receives |2s|^beta at the last
// FP64 iterate.
__device__ __forceinline__ float pow2s_f32(float s, float beta)
{
    return __builtin_amdgcn_exp2f(beta * __builtin_amdgcn_logf(2.0f * s));
}

__device__ __forceinline__ double pow2s_f64(double s, double beta) { return exp2(beta * log2(2.0 * s)); }

// 1/x in FP64 from the FP32 hardware reciprocal (1 ulp) and one Newton step:
// relative error ~1e-14 for x within the FP32 normal range
__device__ __forceinline__ double rcp_refined(double x)
{
    const double r = (double)__builtin_amdgcn_rcpf((float)x);
    return r * fma(-x, r, 2.0);
}

// (2 s)^beta for 2 s > 0 in the FP64 normal range, without the library's
// special-case handling and extra-precise argument: log2 of the mantissa
// reduced to [sqrt(1/2), sqrt(2)) from the series
// ln m = 2 (f + f^3/3 + f^5/5 + ...), f = (m - 1)/(m + 1), |f| < 0.172,
// to f^21; 2^y as 2^n e^t, n = rint(y), |t| <= ln2/2, from the Taylor series
// of e^t to t^12.  Relative error below 1e-14 while |beta log2(2 s)| < 60.
// a constant materialised in scalar registers where it is used: keeps the
// compiler from hoisting the series coefficients below out of the spring loop
// into vector registers (38 of them, which then spill)
__device__ __forceinline__ double sconst(double c)
{
    asm volatile("" : "+s"(c));
    return c;
}

__device__ __forceinline__ double pow2s_fast(double s, double beta)
{
    const double x = 2.0 * s;
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    int ex = __builtin_amdgcn_frexp_exp(x);
    if (m < sconst(0.70710678118654752)) {
        m *= 2.0;
        --ex;
    }
    const double f = (m - 1.0) * rcp_refined(m + 1.0), f2 = f * f;
    double q = sconst(1.0 / 21);
    q = fma(q, f2, sconst(1.0 / 19));
    q = fma(q, f2, sconst(1.0 / 17));
    q = fma(q, f2, sconst(1.0 / 15));
    q = fma(q, f2, sconst(1.0 / 13));
    q = fma(q, f2, sconst(1.0 / 11));
    q = fma(q, f2, sconst(1.0 / 9));
    q = fma(q, f2, sconst(1.0 / 7));
    q = fma(q, f2, sconst(1.0 / 5));
    q = fma(q, f2, sconst(1.0 / 3));
    const double lnm = 2.0 * f * fma(q, f2, 1.0);
    const double y = beta * fma(lnm, sconst(1.4426950408889634), (double)ex);
    const double n = __builtin_rint(y), t = (y - n) * sconst(0.69314718055994531);
    double r = sconst(1.0 / 479001600.0);  // 1/12!
    r = fma(r, t, sconst(1.0 / 39916800.0));
    r = fma(r, t, sconst(1.0 / 3628800.0));
    r = fma(r, t, sconst(1.0 / 362880.0));
    r = fma(r, t, sconst(1.0 / 40320.0));
    r = fma(r, t, sconst(1.0 / 5040.0));
    r = fma(r, t, sconst(1.0 / 720.0));
    r = fma(r, t, sconst(1.0 / 120.0));
    r = fma(r, t, sconst(1.0 / 24.0));
    r = fma(r, t, sconst(1.0 / 6.0));
    r = fma(r, t, sconst(0.5));
    r = fma(r, t, 1.0);
    r = fma(r, t, 1.0);
    return __builtin_amdgcn_ldexp(r, (int)n);
}

__device__ __forceinline__ double ro_inverse_pw(double e, double beta, double* pw)
{
    const double a = fabs(e);
    if (!(a >= 1e-30)) {  // (2a)^beta < 1e-27: s = a to FP64 precision
        *pw = a == 0.0 ? 0.0 : pow2s_f64(a, beta);
        return e;
    }
    const float af = (float)a, bf = (float)beta, bp1f = 1.0f + bf;
    float sf = fminf(af, __builtin_amdgcn_exp2f((__builtin_amdgcn_logf(af) - bf) * __builtin_amdgcn_rcpf(bp1f)));
#pragma unroll 1
    for (int it = 0; it < 12; ++it) {
        const float p = pow2s_f32(sf, bf);
        const float f = sf * (1.0f + p) - af;
        if (f <= 0.0f) break;
        const float ds = f * __builtin_amdgcn_rcpf(fmaf(bp1f, p, 1.0f));
        sf -= ds;
        if (ds <= 1e-7f * sf) break;
    }
    const double c1 = beta, c2 = 0.5 * beta * (beta - 1.0), c3 = c2 * (beta - 2.0) * (1.0 / 3.0);
    double s = (double)sf, s0 = 0.0, p0 = 0.0, r0 = 0.0, rd = 0.0, p = 0.0;
    bool fresh = true;  // take the power afresh at the current iterate
#pragma unroll 1
    for (int it = 0; it < 60; ++it) {
        if (fresh) {
            s0 = s;
            p0 = p = pow2s_fast(s0, beta);
            r0 = rcp_refined(s0);
            rd = rcp_refined(fma(1.0 + beta, p0, 1.0));
        }
        const double ds = fma(s, 1.0 + p, -a) * rd;
        s -= ds;
        const double d = (s - s0) * r0;
        fresh = !(fabs(d) < 1e-4);  // far from the FP32 root (its iteration cap)
        if (!fresh) {
            p = p0 * fma(d, fma(d, fma(d, c3, c2), c1), 1.0);
            if (fabs(ds) <= 0x1p-44 * s) break;
        }
    }
    *pw = p;
    return e < 0 ? -s : s;
}

struct SpringPar { double G0, gref, hmax, beta; };

// Law state of a chunk of ecp elements (ecp a multiple of EB): four FP64
// fields (gp, gr, tr, sm: the strain, the reversal strain and stress, and the
// normalised skeleton stress at the largest strain reached on the skeleton)
// then one int32 field packing the loading direction,
// the skeleton flag and the count of older reversal points kept,
// (dir + 1) | skel << 2 | count << 3 (36 B per spring and point); with a
// reversal memory of depth K > 1 the int32 field is followed by 2 (K - 1)
// FP64 fields, the older points' (gr, tr) pairs, oldest first (36 + 16 (K - 1)
// B).  Within a field: element blocks of EB, then spring, point,
// element-in-block, member.
__device__ __forceinline__ int theta_flags(int dir, int skel) { return (dir + 1) | (skel << 2); }

struct ThetaView {
    double* d;
    int* i;
    double* od;    // older reversal points: gr of point k at od[2k * field_n], tr at od[(2k + 1) * field_n]
    long field_n;  // entries per field = ecp * 4 * ns * MB
    int ns, MB, EB;
    __device__ __forceinline__ long at(long el, int s, int j, int m) const
    {
        return (((el / EB) * ns + s) * 4 + j) * (long)EB * MB * 1 + (el % EB) * MB + m;
    }
};

__device__ __forceinline__ ThetaView theta_view(void* base, long ecp, int ns, int MB)
{
    ThetaView v;
    v.field_n = ecp * 4 * (long)ns * MB;
    v.d = (double*)base;
    v.i = (int*)(v.d + 4 * v.field_n);
    v.od = (double*)(v.i + v.field_n);  // field_n is a multiple of 4: 8-byte aligned
    v.ns = ns;
    v.MB = MB;
    v.EB = MB >= 64 ? 1 : 64 / MB;
    return v;
}

__global__ void k_theta_init(void* base, long ecp, int ns, int MB)
{
    ThetaView v = theta_view(base, ecp, ns, MB);
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= v.field_n) return;
    for (int f = 0; f < 4; ++f) v.d[f * v.field_n + i] = 0.0;
    v.i[i] = theta_flags(0, 1);  // no loading yet, on the skeleton
}

void launch_theta_init(hipStream_t s, void* base, long ecp, int ns, int MB)
{
    long n = ecp * 4 * (long)ns * MB;
    if (n > 0) hipLaunchKernelGGL(k_theta_init, dim3(nblocks(n)), dim3(256), 0, s, base, ecp, ns, MB);
}

// write D of point j in FP64 and in the inner operator's storage (FP32 or
// bfloat16 pairs, whichever is allocated)
__device__ __forceinline__ void store_D(const double d[21], long e, int j, int MB, int EB, int m,
                                        double* __restrict__ D, float* __restrict__ D32, uint32_t* __restrict__ D16)
{
#pragma unroll
    for (int k = 0; k < 21; ++k) {
        const long idx = d_index(e, j, k, MB, EB, m);
        D[idx] = d[k];
        if (D32) D32[idx] = (float)d[k];
    }
    if (D16) {
#pragma unroll
        for (int q = 0; q < 11; ++q) {
            const uint32_t lo = f2bf(d[2 * q]);
            const uint32_t hi = (2 * q + 1 < 21) ? f2bf(d[2 * q + 1]) : 0u;
            D16[d16_index(e, j, q, MB, EB, m)] = lo | (hi << 16);
        }
    }
}

// D of a point from the spring tangents: Kb m m^T + sum c_k G_k n_k n_k^T
__global__ void k_law_init(DevMesh M, int MB, int nm, const double* __restrict__ mat, int ns,
                           const double* __restrict__ dirs, const double* __restrict__ w,
                           double* __restrict__ D, float* __restrict__ D32, uint32_t* __restrict__ D16,
                           double* __restrict__ h, int only_m, bool d16_mean)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = only_m >= 0 ? only_m : (int)(t % MB);
    const long e = only_m >= 0 ? t : t / MB;
    if (e >= M.ne || m >= nm) return;
    const int EB = MB >= 64 ? 1 : 64 / MB;
    const int l = M.layer[e];
    const double G0 = matv(mat, l, MAT_G0, MB, m), Kb = matv(mat, l, MAT_KB, MB, m);
    double d[21];
    for (int k = 0; k < 21; ++k) d[k] = 0;
    for (int s = 0; s < ns; ++s) {
        const double* n = dirs + 6 * s;
        const double c = w[s] * G0;
        for (int r = 0; r < 6; ++r)
            for (int q = r; q < 6; ++q) d[sym6(r, q)] += c * n[r] * n[q];
    }
    for (int r = 0; r < 3; ++r)
        for (int q = r; q < 3; ++q) d[sym6(r, q)] += Kb;
    for (int j = 0; j < 4; ++j) store_D(d, e, j, MB, EB, m, D, D32, d16_mean ? nullptr : D16);
    if (d16_mean && D16)
        for (int q = 0; q < 11; ++q)
            D16[d16m_index(e, q, MB, EB, m)] = f2bf(d[2 * q]) | ((2 * q + 1 < 21 ? f2bf(d[2 * q + 1]) : 0u) << 16);
    h[e * MB + m] = 0.0;
}

void launch_law_init(hipStream_t s, const DevMesh& M, int MB, int nm, const double* mat, int, int ns,
                     const double* dirs, const double* w, double* D, float* D32, uint32_t* D16, double* h,
                     int only_m, bool d16_mean)
{
    long n = only_m >= 0 ? (long)M.ne : (long)M.ne * MB;
    if (n > 0)
        hipLaunchKernelGGL(k_law_init, dim3(nblocks(n)), dim3(256), 0, s, M, MB, nm, mat, ns, dirs, w, D, D32, D16, h,
                           only_m, d16_mean);
}

// reset the law state of one member (serving: a new request takes the slot)
__global__ void k_theta_reset_member(void* base, long ecp, int ns, int MB, int m)
{
    ThetaView v = theta_view(base, ecp, ns, MB);
    const long n = ecp * 4 * (long)ns;  // (element, spring, point) triples
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n) return;
    const long el = t / (4L * ns);
    const int s = (int)((t / 4) % ns), j = (int)(t % 4);
    const long idx = v.at(el, s, j, m);
    for (int f = 0; f < 4; ++f) v.d[f * v.field_n + idx] = 0.0;
    v.i[idx] = theta_flags(0, 1);
}

void launch_theta_reset_member(hipStream_t s, void* base, long ecp, int ns, int MB, int m)
{
    long n = ecp * 4 * (long)ns;
    if (n > 0) hipLaunchKernelGGL(k_theta_reset_member, dim3(nblocks(n)), dim3(256), 0, s, base, ecp, ns, MB, m);
}

// zero column m of a member-innermost array with `rows` rows
__global__ void k_zero_member(double* p, long rows, int MB, int m)
{
    const long r = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (r < rows) p[r * MB + m] = 0.0;
}

void launch_zero_member(hipStream_t s, double* p, long rows, int MB, int m)
{
    if (rows > 0) hipLaunchKernelGGL(k_zero_member, dim3(nblocks(rows)), dim3(256), 0, s, p, rows, MB, m);
}

// One lane per (element, point, member) of the chunk [e0, e0 + ec), the four
// points of an element-member in adjacent lanes: strain increment at the point
// from du, then every spring's Masing/RO update and tangent,
// D = Kb m m^T + sum c_k G_t n n^T at the point, and the element damping h
// (the mean over the four points, summed across the four lanes).
// WAVE_ELEM: a wavefront covers one element (MB >= 16): its geometry and
// connectivity are then wave-uniform and live in scalar registers.
// LDS_NS > 0 (at most that many springs): each lane parks its springs' c_k G_k
// in LDS during the spring loop and forms D after it, so the 21 FP64
// accumulators of D are not live across the skeleton inversions: 139
// registers instead of 178 (3 wavefronts per SIMD instead of 2), and with the
// launch bound of 4 wavefronts per SIMD 128 registers and 36 B of spills
// (4 % faster again); 0: D accumulated in registers.
// MEM: a reversal memory of `depth` > 1 points (inner loops close, as the
// oracle's law with that depth); false: the three-rule law.
constexpr int kLawLdsSprings = 16;
template <bool WAVE_ELEM, int LDS_NS, bool MEM>
__global__ __launch_bounds__(256, LDS_NS > 0 ? 4 : 1) void k_law(DevMesh M, int MB, int nm, int e0, int ec, long ecp,
                                            const double* __restrict__ mat, const int* __restrict__ nonlinear,
                                            int ns, int depth, const double* __restrict__ dirs,
                                            const double* __restrict__ w, const double* __restrict__ du,
                                            void* theta, double* __restrict__ D, float* __restrict__ D32,
                                            uint32_t* __restrict__ D16, double* __restrict__ h,
                                            const int* __restrict__ stepping, bool d16_mean)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int j = (int)(t & 3);
    const long q = t >> 2;
    const int m = (int)(q % MB);
    long el = q / MB;
    if (WAVE_ELEM) el = __builtin_amdgcn_readfirstlane((int)el);
    if (el >= ec || m >= nm) return;
    if (stepping && !stepping[m]) return;
    const long e = e0 + el;
    const long ne = M.ne;
    const int l = M.layer[e];
    if (!nonlinear[l]) return;
    const int EB = MB >= 64 ? 1 : 64 / MB;
    SpringPar P;
    P.G0 = matv(mat, l, MAT_G0, MB, m);
    P.gref = matv(mat, l, MAT_GREF, MB, m);
    P.hmax = matv(mat, l, MAT_HMAX, MB, m);
    P.beta = matv(mat, l, MAT_BETA, MB, m);
    const double Kb = matv(mat, l, MAT_KB, MB, m);
    const double rgref = 1.0 / P.gref;
    // strain increment at point j, node by node (gradient of N_n at the point
    // times the node's increment)
    double ej[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    {
        double gL[4][3];
#pragma unroll
        for (int k = 0; k < 12; ++k) gL[k / 3][k % 3] = M.geo64[k * ne + e];
        double L[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) L[i] = (i == j) ? QA_ : QB_;
        constexpr int E[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};
#pragma unroll
        for (int n = 0; n < 10; ++n) {
            const long node = M.conn[n * ne + e];
            const double* un = du + node * 3 * MB + m;
            const double u0 = un[0], u1 = un[MB], u2 = un[2 * MB];
            double g[3];
#pragma unroll
            for (int a = 0; a < 3; ++a)
                g[a] = n < 4 ? (4.0 * L[n] - 1.0) * gL[n][a]
                             : 4.0 * (L[E[n - 4][0]] * gL[E[n - 4][1]][a] + L[E[n - 4][1]] * gL[E[n - 4][0]][a]);
            ej[0] += g[0] * u0;
            ej[1] += g[1] * u1;
            ej[2] += g[2] * u2;
            ej[3] += g[1] * u0 + g[0] * u1;
            ej[4] += g[2] * u1 + g[1] * u2;
            ej[5] += g[0] * u2 + g[2] * u0;
        }
    }
    ThetaView th = theta_view(theta, ecp, ns, MB);
    const long fn = th.field_n;
    __shared__ double cgs[LDS_NS > 0 ? LDS_NS * 256 : 1];
    if (LDS_NS > 0) {
        // each spring's strain increment waits in its LDS slot (the slot takes
        // c_k G_k after the update), so the strain is not live across the loop
#pragma unroll 1
        for (int sp = 0; sp < ns; ++sp) {
            const double* n = dirs + 6 * sp;
            cgs[sp * 256 + threadIdx.x] =
                n[0] * ej[0] + n[1] * ej[1] + n[2] * ej[2] + n[3] * ej[3] + n[4] * ej[4] + n[5] * ej[5];
        }
    }
    double d[21];
#pragma unroll
    for (int k = 0; k < 21; ++k) d[k] = 0;
    double hs = 0.0;
    // the next spring's state is loaded while this one is updated
    long nidx = th.at(el, 0, j, m);
    double ngp = th.d[nidx], ngr = th.d[fn + nidx], ntr = th.d[2 * fn + nidx], nsm = th.d[3 * fn + nidx];
    int nfl = th.i[nidx];
#pragma unroll 1
    for (int sp = 0; sp < ns; ++sp) {
        const double* n = dirs + 6 * sp;
        const double dg = LDS_NS > 0 ? cgs[sp * 256 + threadIdx.x]
                                     : n[0] * ej[0] + n[1] * ej[1] + n[2] * ej[2] + n[3] * ej[3] + n[4] * ej[4] +
                                           n[5] * ej[5];
        const long idx = nidx;
        double gp = ngp, gr = ngr, tr = ntr, sm = nsm;
        int dir = (nfl & 3) - 1, skel = (nfl >> 2) & 1;
        int cnt = MEM ? nfl >> 3 : 0;  // older reversal points kept
        if (sp + 1 < ns) {
            nidx = th.at(el, sp + 1, j, m);
            ngp = th.d[nidx]; ngr = th.d[fn + nidx]; ntr = th.d[2 * fn + nidx]; nsm = th.d[3 * fn + nidx];
            nfl = th.i[nidx];
        }
        const int dsg = dg > 0.0 ? 1 : (dg < 0.0 ? -1 : 0);
        const bool reverse = dsg != 0 && dir != 0 && dsg != dir;
        // largest strain reached on the skeleton: |gp| while on it; off it, from
        // the stored normalised skeleton stress sm through the explicit forward
        // relation gm = gref sm (1 + pm), pm = (2 sm)^beta, whose power also
        // gives the damping of an off-skeleton spring
        double pm = 0.0, gm = fabs(gp);
        if ((!skel || reverse) && sm > 0.0) {
            pm = pow2s_fast(sm, P.beta);
            if (!skel) gm = P.gref * sm * (1.0 + pm);
        }
        bool rev2 = false;     // reversal on a branch: the skeleton inverted at rev_arg
        double rev_arg = 0.0;
        if (dsg != 0) {
            if (reverse) {  // a Masing branch starts here
                double trev = 0.0;
                if (skel) {
                    // the skeleton stress at gp = +-gm is +-sm (stored by the last update on the skeleton)
                    trev = P.G0 * P.gref * copysign(sm, gp);
                } else {
                    rev_arg = 0.5 * (gp - gr);
                    if (MEM) {
                        double pk;
                        trev = tr + 2.0 * P.G0 * P.gref * ro_inverse_pw(rev_arg * rgref, P.beta, &pk);
                    } else {
                        rev2 = true;
                    }
                }
                if (MEM) {
                    // the origin of the branch being left is kept (the oldest dropped when
                    // full); a closed loop below may replace the new branch
                    if (!skel) {
                        if (cnt == depth - 1) {
                            for (int k = 0; k + 1 < cnt; ++k) {
                                th.od[(2 * k) * fn + idx] = th.od[(2 * k + 2) * fn + idx];
                                th.od[(2 * k + 1) * fn + idx] = th.od[(2 * k + 3) * fn + idx];
                            }
                            --cnt;
                        }
                        th.od[(2 * cnt) * fn + idx] = gr;
                        th.od[(2 * cnt + 1) * fn + idx] = tr;
                        ++cnt;
                    }
                }
                if (!rev2) tr = trev;
                gr = gp;
                skel = 0;
            }
            dir = dsg;
            const double g = gp + dg;
            if (!skel && (double)dsg * g >= gm) {  // rejoin the skeleton
                skel = 1;
                cnt = 0;
            }
            if (MEM) {  // closed inner loops: on along the branch before the previous one
                while (!skel && cnt >= 2 && (double)dsg * g >= (double)dsg * th.od[(2 * cnt - 2) * fn + idx]) {
                    gr = th.od[(2 * cnt - 4) * fn + idx];
                    tr = th.od[(2 * cnt - 3) * fn + idx];
                    cnt -= 2;
                }
            }
            gp = g;
        }
        const double xi = skel ? gp : 0.5 * (gp - gr);
        // the inversions through one copy of the solver: a branch reversal's, then xi's
        double s_rev = 0.0, s_xi = 0.0, pw = 0.0;
#pragma unroll 1
        for (int k = 0; k < 2; ++k) {
            if (k == 0 && !rev2) continue;
            double pk;
            const double sv = ro_inverse_pw((k == 0 ? rev_arg : xi) * rgref, P.beta, &pk);
            if (k == 0) s_rev = sv;
            else { s_xi = sv; pw = pk; }
        }
        if (rev2) tr += 2.0 * P.G0 * P.gref * s_rev;
        if (skel) sm = fabs(s_xi);  // on the skeleton gm = |gp|
        if (dsg != 0) {
            th.d[idx] = gp; th.d[fn + idx] = gr; th.d[2 * fn + idx] = tr; th.d[3 * fn + idx] = sm;
            th.i[idx] = theta_flags(dir, skel) | (cnt << 3);
        }
        const double Gt = P.G0 / (1.0 + (1.0 + P.beta) * pw);
        // damping 1 - S(em)/em at em = gm/gref: with em = s (1 + (2s)^beta) at s = S(em)
        // it is p/(1 + p), p the power at the skeleton stress of the largest strain
        const double ph = skel ? pw : pm;
        const double hk = P.hmax * ph / (1.0 + ph);
        hs += hk;
        const double c = w[sp] * Gt;
        if (LDS_NS > 0) {
            cgs[sp * 256 + threadIdx.x] = c;
        } else {
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int qq = r; qq < 6; ++qq) d[sym6(r, qq)] += c * n[r] * n[qq];
        }
    }
    if (LDS_NS > 0) {
#pragma unroll 1
        for (int sp = 0; sp < ns; ++sp) {
            const double* n = dirs + 6 * sp;
            const double c = cgs[sp * 256 + threadIdx.x];
#pragma unroll
            for (int r = 0; r < 6; ++r)
#pragma unroll
                for (int qq = r; qq < 6; ++qq) d[sym6(r, qq)] += c * n[r] * n[qq];
        }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int qq = r; qq < 3; ++qq) d[sym6(r, qq)] += Kb;
    store_D(d, e, j, MB, EB, m, D, D32, d16_mean ? nullptr : D16);
    if (d16_mean && D16) {  // element-mean D of the inner operator (the four point lanes)
#pragma unroll
        for (int k = 0; k < 21; ++k) {
            d[k] += __shfl_xor(d[k], 1);
            d[k] += __shfl_xor(d[k], 2);
        }
        if (j == 0)
#pragma unroll
            for (int q = 0; q < 11; ++q)
                D16[d16m_index(e, q, MB, EB, m)] =
                    f2bf(0.25 * d[2 * q]) | ((2 * q + 1 < 21 ? f2bf(0.25 * d[2 * q + 1]) : 0u) << 16);
    }
    // element damping: mean over the 4 points (adjacent lanes) and the springs
    double hsum = hs / ns;
    hsum += __shfl_xor(hsum, 1);
    hsum += __shfl_xor(hsum, 2);
    if (j == 0) h[e * MB + m] = 0.25 * hsum;
}

template <int LDS_NS, bool MEM>
static void law_dispatch(hipStream_t s, dim3 g, const DevMesh& M, int MB, int nm, int e0, int ec, long ecp,
                         const double* mat, const int* nonlinear, int ns, int depth, const double* dirs,
                         const double* w, const double* du, void* theta, double* D, float* D32, uint32_t* D16,
                         double* h, const int* stepping, bool d16_mean)
{
    if (MB >= 16)
        hipLaunchKernelGGL((k_law<true, LDS_NS, MEM>), g, dim3(256), 0, s, M, MB, nm, e0, ec, ecp, mat, nonlinear, ns,
                           depth, dirs, w, du, theta, D, D32, D16, h, stepping, d16_mean);
    else
        hipLaunchKernelGGL((k_law<false, LDS_NS, MEM>), g, dim3(256), 0, s, M, MB, nm, e0, ec, ecp, mat, nonlinear, ns,
                           depth, dirs, w, du, theta, D, D32, D16, h, stepping, d16_mean);
}

void launch_law(hipStream_t s, const DevMesh& M, int MB, int nm, int e0, int ec, long ecp, const double* mat, int,
                const int* nonlinear, int ns, int depth, const double* dirs, const double* w, const double* du,
                void* theta, double* D, float* D32, uint32_t* D16, double* h, const int* stepping, bool d16_mean)
{
    long n = (long)ec * MB * 4;
    if (n <= 0) return;
    const dim3 g(nblocks(n));
    const bool small = ns <= kLawLdsSprings, mem = depth > 1;
    if (small && !mem)
        law_dispatch<kLawLdsSprings, false>(s, g, M, MB, nm, e0, ec, ecp, mat, nonlinear, ns, depth, dirs, w, du,
                                            theta, D, D32, D16, h, stepping, d16_mean);
    else if (small)
        law_dispatch<kLawLdsSprings, true>(s, g, M, MB, nm, e0, ec, ecp, mat, nonlinear, ns, depth, dirs, w, du,
                                           theta, D, D32, D16, h, stepping, d16_mean);
    else if (!mem)
        law_dispatch<0, false>(s, g, M, MB, nm, e0, ec, ecp, mat, nonlinear, ns, depth, dirs, w, du, theta, D, D32,
                               D16, h, stepping, d16_mean);
    else
        law_dispatch<0, true>(s, g, M, MB, nm, e0, ec, ecp, mat, nonlinear, ns, depth, dirs, w, du, theta, D, D32,
                              D16, h, stepping, d16_mean);
}

// ---------------------------------------------------------------------------
// Newmark state updates (Section 2.1), receivers, incident wave
// ---------------------------------------------------------------------------

__global__ void k_newmark(long n, int MB, int nm, const double* __restrict__ du, double* __restrict__ u,
                          double* __restrict__ v, double* __restrict__ a, double dt, const int* __restrict__ stepping)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(i % MB);
    if (i >= n || m >= nm || !stepping[m]) return;
    const double d = du[i], vo = v[i];
    u[i] += d;
    a[i] = -a[i] - 4.0 / dt * vo + 4.0 / (dt * dt) * d;
    v[i] = -vo + 2.0 / dt * d;
}

void launch_newmark(hipStream_t s, long n, int MB, int nm, const double* du, double* u, double* v, double* a,
                    double dt, const int* stepping)
{
    long N = n * MB;
    hipLaunchKernelGGL(k_newmark, dim3(nblocks(N)), dim3(256), 0, s, N, MB, nm, du, u, v, a, dt, stepping);
}

// Initial guess of the step's CG from the increments of the previous steps
// (du holds du^{n-1}, d2 du^{n-2}, d3 du^{n-3}; zero before a member's first
// steps, which is its true history from rest), extrapolated by a polynomial
// of degree `order` in time: 0 keeps du^{n-1}, 1 gives 2 du^{n-1} - du^{n-2},
// 2 gives 3 du^{n-1} - 3 du^{n-2} + du^{n-3}.  The history shifts every step
// whatever the order.
__global__ void k_predict(long n, int MB, int nm, int order, double* __restrict__ du, double* __restrict__ d2,
                          double* __restrict__ d3, const int* __restrict__ stepping)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(i % MB);
    if (i >= n || m >= nm || !stepping[m]) return;
    const double a = du[i], b = d2[i], c = d3[i];
    d3[i] = b;
    d2[i] = a;
    if (order == 1) du[i] = 2.0 * a - b;
    else if (order == 2) du[i] = 3.0 * (a - b) + c;
}

void launch_predict(hipStream_t s, long n, int MB, int nm, int order, double* du, double* d2, double* d3,
                    const int* stepping)
{
    const long N = n * MB;
    hipLaunchKernelGGL(k_predict, dim3(nblocks(N)), dim3(256), 0, s, N, MB, nm, order, du, d2, d3, stepping);
}

__global__ void k_receivers(int nrecv, const int* __restrict__ recv, int MB, int nm, const double* __restrict__ v,
                            double* __restrict__ hist, const int* __restrict__ member_step, int ns,
                            double* __restrict__ vmax, const int* __restrict__ stepping)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    const int m = (int)(t % MB);
    const long r = t / MB;
    if (r >= nrecv || m >= nm || !stepping[m]) return;
    const long node = recv[r];
    const int step = member_step[m];
    double nrm = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double val = v[(node * 3 + c) * MB + m];
        hist[(((long)m * ns + step) * nrecv + r) * 3 + c] = val;
        nrm += val * val;
    }
    nrm = sqrt(nrm);
    const long vi = (long)m * nrecv + r;
    if (nrm > vmax[vi]) vmax[vi] = nrm;
}

void launch_receivers(hipStream_t s, int nrecv, const int* recv, int MB, int nm, const double* v, double* hist,
                      const int* member_step, int ns, double* vmax, const int* stepping)
{
    long n = (long)nrecv * MB;
    if (n > 0)
        hipLaunchKernelGGL(k_receivers, dim3(nblocks(n)), dim3(256), 0, s, nrecv, recv, MB, nm, v, hist, member_step,
                           ns, vmax, stepping);
}

// incident velocity by the trapezoid rule from the incident acceleration
// (zero at t = 0): one thread per (member, component), sequential in time
__global__ void k_incident_velocity(int nm, int ns, const double* __restrict__ acc, double* __restrict__ vI, double dt)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nm * 3) return;
    const int m = t / 3, c = t % 3;
    double v = 0.0, ap = 0.0;
    for (int n = 0; n < ns; ++n) {
        const double an = acc[((long)m * ns + n) * 3 + c];
        v += 0.5 * dt * (ap + an);
        ap = an;
        vI[((long)m * ns + n) * 3 + c] = v;
    }
}

void launch_incident_velocity(hipStream_t s, int, int nm, int ns, const double* acc, double* vI, double dt)
{
    hipLaunchKernelGGL(k_incident_velocity, dim3(nblocks(nm * 3)), dim3(256), 0, s, nm, ns, acc, vI, dt);
}

// incident velocity of each member at its current step, member-innermost [3][MB]
__global__ void k_pick_vI(int MB, int nm, int ns, const double* __restrict__ vI_all, const int* __restrict__ member_step,
                          double* __restrict__ vI_cur)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= MB * 3) return;
    const int m = t % MB, c = t / MB;
    double v = 0.0;
    if (m < nm) {
        const int st = member_step[m];
        if (st >= 0 && st < ns) v = vI_all[((long)m * ns + st) * 3 + c];
    }
    vI_cur[c * MB + m] = v;
}

void launch_pick_vI(hipStream_t s, int MB, int nm, int ns, const double* vI_all, const int* member_step,
                    double* vI_cur)
{
    hipLaunchKernelGGL(k_pick_vI, dim3(nblocks(MB * 3)), dim3(256), 0, s, MB, nm, ns, vI_all, member_step, vI_cur);
}

__global__ void k_record_iters(int MB, int nm, int ns, const int* __restrict__ member_step,
                               const int* __restrict__ stepping, const int* __restrict__ iters,
                               const int* __restrict__ inner_total, int* __restrict__ out)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= nm || !stepping[m]) return;
    const int st = member_step[m];
    if (st < 0 || st >= ns) return;
    out[((long)m * ns + st) * 2] = iters[m];
    out[((long)m * ns + st) * 2 + 1] = inner_total[m];
}

void launch_record_iters(hipStream_t s, int MB, int nm, int ns, const int* member_step, const int* stepping,
                         const int* iters, const int* inner_total, int* out)
{
    hipLaunchKernelGGL(k_record_iters, dim3(nblocks(MB)), dim3(256), 0, s, MB, nm, ns, member_step, stepping, iters,
                       inner_total, out);
}

}  // namespace nlth
