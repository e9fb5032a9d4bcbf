// CG vector kernels of libnlth: fused updates with the dot products of the
// next step folded into the same pass, per-member deterministic reductions,
// and the per-member scalar logic of the CG variants.
//
// Vectors are member-innermost (v[(row)*MB + m]).  A thread handles VEC
// consecutive members of one row (16-byte loads when MB is a multiple of 4)
// and loops over rows with a grid stride; a block of 256 threads covers
// 256/(MB/VEC) rows per iteration.  Partial sums are reduced in LDS by a
// fixed tree and written as partial[(k*nblk + blk)*MB + m]; the finalize
// kernel reduces them over blocks by a fixed tree as well, so results do not
// depend on timing.
#include <math.h>

#include "nlth_impl.hpp"

namespace nlth {

constexpr int kMaxBlocks = kMaxPartialBlocks;

template <typename T, int VEC> struct Pk { T a[VEC]; };

template <typename T, int VEC>
__device__ __forceinline__ Pk<T, VEC> ld(const T* __restrict__ p)
{
    Pk<T, VEC> r;
    if constexpr (VEC == 4 && sizeof(T) == 4) {
        const float4 q = *reinterpret_cast<const float4*>(p);
        r.a[0] = q.x; r.a[1] = q.y; r.a[2] = q.z; r.a[3] = q.w;
    } else if constexpr (VEC == 4 && sizeof(T) == 8) {
        const double2 q0 = *reinterpret_cast<const double2*>(p);
        const double2 q1 = *reinterpret_cast<const double2*>(p + 2);
        r.a[0] = q0.x; r.a[1] = q0.y; r.a[2] = q1.x; r.a[3] = q1.y;
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) r.a[v] = p[v];
    }
    return r;
}

template <typename T, int VEC>
__device__ __forceinline__ void st(T* __restrict__ p, const Pk<T, VEC>& r)
{
    if constexpr (VEC == 4 && sizeof(T) == 4) {
        *reinterpret_cast<float4*>(p) = make_float4(r.a[0], r.a[1], r.a[2], r.a[3]);
    } else if constexpr (VEC == 4 && sizeof(T) == 8) {
        *reinterpret_cast<double2*>(p) = make_double2(r.a[0], r.a[1]);
        *reinterpret_cast<double2*>(p + 2) = make_double2(r.a[2], r.a[3]);
    } else {
#pragma unroll
        for (int v = 0; v < VEC; ++v) p[v] = r.a[v];
    }
}

static inline int vec_of(int MB) { return (MB % 4 == 0) ? 4 : 1; }

static inline int grid_for(long rows, int rpb)
{
    long g = (rows + rpb - 1) / rpb;
    if (g > kMaxBlocks) g = kMaxBlocks;
    if (g < 1) g = 1;
    return (int)g;
}

// block-level reduction of ND accumulators per member and store of partials
template <int ND, int VEC>
__device__ __forceinline__ void block_partials(double acc[ND][VEC], int QB, int MB, double* __restrict__ partial)
{
    __shared__ double sh[ND][VEC][256];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < ND; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) sh[k][v][t] = acc[k][v];
    __syncthreads();
    for (int s = 128; s >= QB; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int k = 0; k < ND; ++k)
#pragma unroll
                for (int v = 0; v < VEC; ++v) sh[k][v][t] += sh[k][v][t + s];
        __syncthreads();
    }
    if (t < QB) {
        const int m0 = t * VEC;
#pragma unroll
        for (int k = 0; k < ND; ++k)
#pragma unroll
            for (int v = 0; v < VEC; ++v) partial[((long)k * gridDim.x + blockIdx.x) * MB + m0 + v] = sh[k][v][t];
    }
}

__device__ __forceinline__ bool member_mask(const int* __restrict__ flag, int m0, int VEC, int nm, bool act[4])
{
    bool any = false;
    for (int v = 0; v < VEC; ++v) {
        const int m = m0 + v;
        act[v] = m < nm && (flag ? flag[m] != 0 : true);
        any |= act[v];
    }
    return any;
}

// ---------------------------------------------------------------------------
// generic partial dots sum_rows a_k . b_k
// ---------------------------------------------------------------------------

template <typename T, int VEC, int ND>
__global__ __launch_bounds__(256) void k_dotsv(const T* __restrict__ a0, const T* __restrict__ b0,
                                              const T* __restrict__ a1, const T* __restrict__ b1,
                                              const T* __restrict__ a2, const T* __restrict__ b2, long nrows,
                                              int MB, int nm, const int* __restrict__ flag,
                                              double* __restrict__ partial)
{
    const int QB = MB / VEC, rpb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, rl = t / QB, m0 = q * VEC;
    double acc[ND][VEC];
#pragma unroll
    for (int k = 0; k < ND; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
    bool act[4];
    if (member_mask(flag, m0, VEC, nm, act)) {
        for (long row = (long)blockIdx.x * rpb + rl; row < nrows; row += (long)gridDim.x * rpb) {
            const long i = row * MB + m0;
            const Pk<T, VEC> A0 = ld<T, VEC>(a0 + i), B0 = ld<T, VEC>(b0 + i);
#pragma unroll
            for (int v = 0; v < VEC; ++v) acc[0][v] += (double)A0.a[v] * (double)B0.a[v];
            if constexpr (ND > 1) {
                const Pk<T, VEC> A1 = ld<T, VEC>(a1 + i), B1 = ld<T, VEC>(b1 + i);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[1][v] += (double)A1.a[v] * (double)B1.a[v];
            }
            if constexpr (ND > 2) {
                const Pk<T, VEC> A2 = ld<T, VEC>(a2 + i), B2 = ld<T, VEC>(b2 + i);
#pragma unroll
                for (int v = 0; v < VEC; ++v) acc[2][v] += (double)A2.a[v] * (double)B2.a[v];
            }
        }
    }
    block_partials<ND, VEC>(acc, QB, MB, partial);
}

template <typename T>
void launch_dotsv(hipStream_t s, int nd, const T* a0, const T* b0, const T* a1, const T* b1, const T* a2,
                  const T* b2, long nrows, int MB, int nm, const int* flag, double* partial, int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC, rpb = 256 / QB;
    const int g = grid_for(nrows, rpb);
    *nblk = g;
#define DOTS_L(V, N) hipLaunchKernelGGL((k_dotsv<T, V, N>), dim3(g), dim3(256), 0, s, a0, b0, a1, b1, a2, b2, nrows, MB, nm, flag, partial)
    if (VEC == 4) {
        if (nd == 1) DOTS_L(4, 1); else if (nd == 2) DOTS_L(4, 2); else DOTS_L(4, 3);
    } else {
        if (nd == 1) DOTS_L(1, 1); else if (nd == 2) DOTS_L(1, 2); else DOTS_L(1, 3);
    }
#undef DOTS_L
}
template void launch_dotsv<double>(hipStream_t, int, const double*, const double*, const double*, const double*,
                                   const double*, const double*, long, int, int, const int*, double*, int*);
template void launch_dotsv<float>(hipStream_t, int, const float*, const float*, const float*, const float*,
                                  const float*, const float*, long, int, int, const int*, double*, int*);

// ---------------------------------------------------------------------------
// per-node updates with the block-Jacobi 3x3 symmetric inverse
// ---------------------------------------------------------------------------

template <typename T, int VEC>
__device__ __forceinline__ void pinv_apply(const T* __restrict__ pinv, long node, int MB, int m0, const Pk<T, VEC> r[3],
                                           Pk<T, VEC> z[3])
{
    Pk<T, VEC> a[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) a[k] = ld<T, VEC>(pinv + (node * 6 + k) * MB + m0);
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        z[0].a[v] = a[0].a[v] * r[0].a[v] + a[1].a[v] * r[1].a[v] + a[2].a[v] * r[2].a[v];
        z[1].a[v] = a[1].a[v] * r[0].a[v] + a[3].a[v] * r[1].a[v] + a[4].a[v] * r[2].a[v];
        z[2].a[v] = a[2].a[v] * r[0].a[v] + a[4].a[v] * r[1].a[v] + a[5].a[v] * r[2].a[v];
    }
}

// FP64 PCG start: r = b - Ap, z = P r, p = z; partials (b.b, r.r, r.z)
template <int VEC>
__global__ __launch_bounds__(256) void k_pcg_start(int nn, int MB, int nm, const double* __restrict__ b,
                                                  const double* __restrict__ Ap, const double* __restrict__ pinv,
                                                  double* __restrict__ r, double* __restrict__ z,
                                                  double* __restrict__ p, const int* __restrict__ stepping,
                                                  double* __restrict__ partial)
{
    const int QB = MB / VEC, npb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    double acc[3][VEC];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
    bool act[4];
    if (member_mask(stepping, m0, VEC, nm, act)) {
        for (long node = (long)blockIdx.x * npb + t / QB; node < nn; node += (long)gridDim.x * npb) {
            Pk<double, VEC> R[3], Z[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * MB + m0;
                const Pk<double, VEC> B = ld<double, VEC>(b + i), A = ld<double, VEC>(Ap + i);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    R[c].a[v] = act[v] ? B.a[v] - A.a[v] : 0.0;
                    acc[0][v] += B.a[v] * B.a[v];
                }
            }
            pinv_apply<double, VEC>(pinv, node, MB, m0, R, Z);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * MB + m0;
                st<double, VEC>(r + i, R[c]);
                st<double, VEC>(z + i, Z[c]);
                st<double, VEC>(p + i, Z[c]);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    acc[1][v] += R[c].a[v] * R[c].a[v];
                    acc[2][v] += R[c].a[v] * Z[c].a[v];
                }
            }
        }
    }
    block_partials<3, VEC>(acc, QB, MB, partial);
}

void launch_pcg_start(hipStream_t s, int nn, int MB, int nm, const double* b, const double* Ap, const double* pinv,
                      double* r, double* z, double* p, const int* stepping, double* partial, int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nn, 256 / QB);
    *nblk = g;
    if (VEC == 4) hipLaunchKernelGGL((k_pcg_start<4>), dim3(g), dim3(256), 0, s, nn, MB, nm, b, Ap, pinv, r, z, p, stepping, partial);
    else hipLaunchKernelGGL((k_pcg_start<1>), dim3(g), dim3(256), 0, s, nn, MB, nm, b, Ap, pinv, r, z, p, stepping, partial);
}

// FP64 PCG: x += a p, r -= a Ap, z = P r; partials (r.r, r.z)
template <int VEC>
__global__ __launch_bounds__(256) void k_pcg_update(int nn, int MB, int nm, double* __restrict__ x,
                                                   double* __restrict__ r, double* __restrict__ z,
                                                   const double* __restrict__ p, const double* __restrict__ Ap,
                                                   const double* __restrict__ pinv, const double* __restrict__ alpha,
                                                   const int* __restrict__ active, double* __restrict__ partial)
{
    const int QB = MB / VEC, npb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    double acc[2][VEC];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
    bool act[4];
    if (member_mask(active, m0, VEC, nm, act)) {
        double al[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) al[v] = act[v] ? alpha[m0 + v] : 0.0;
        for (long node = (long)blockIdx.x * npb + t / QB; node < nn; node += (long)gridDim.x * npb) {
            Pk<double, VEC> R[3], Z[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * MB + m0;
                Pk<double, VEC> X = ld<double, VEC>(x + i);
                const Pk<double, VEC> P = ld<double, VEC>(p + i), A = ld<double, VEC>(Ap + i);
                R[c] = ld<double, VEC>(r + i);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    X.a[v] += al[v] * P.a[v];
                    R[c].a[v] -= al[v] * A.a[v];
                }
                st<double, VEC>(x + i, X);
                st<double, VEC>(r + i, R[c]);
            }
            pinv_apply<double, VEC>(pinv, node, MB, m0, R, Z);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                st<double, VEC>(z + (node * 3 + c) * MB + m0, Z[c]);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    acc[0][v] += R[c].a[v] * R[c].a[v];
                    acc[1][v] += R[c].a[v] * Z[c].a[v];
                }
            }
        }
    }
    block_partials<2, VEC>(acc, QB, MB, partial);
}

void launch_pcg_update(hipStream_t s, int nn, int MB, int nm, double* x, double* r, double* z, const double* p,
                       const double* Ap, const double* pinv, const double* alpha, const int* active, double* partial,
                       int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nn, 256 / QB);
    *nblk = g;
    if (VEC == 4) hipLaunchKernelGGL((k_pcg_update<4>), dim3(g), dim3(256), 0, s, nn, MB, nm, x, r, z, p, Ap, pinv, alpha, active, partial);
    else hipLaunchKernelGGL((k_pcg_update<1>), dim3(g), dim3(256), 0, s, nn, MB, nm, x, r, z, p, Ap, pinv, alpha, active, partial);
}

// p = z + beta p for active members (beta == NULL: p = z); y = 0 everywhere
template <typename T, int VEC>
__global__ __launch_bounds__(256) void k_p_update(long nrows, int MB, int nm, const T* __restrict__ z,
                                                 T* __restrict__ p, const double* __restrict__ beta,
                                                 const int* __restrict__ active, T* __restrict__ y)
{
    const int QB = MB / VEC, rpb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    bool act[4];
    const bool any = member_mask(active, m0, VEC, nm, act);
    T be[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) be[v] = (beta && act[v]) ? (T)beta[m0 + v] : (T)0;
    Pk<T, VEC> zero;
#pragma unroll
    for (int v = 0; v < VEC; ++v) zero.a[v] = 0;
    for (long row = (long)blockIdx.x * rpb + t / QB; row < nrows; row += (long)gridDim.x * rpb) {
        const long i = row * MB + m0;
        if (any) {
            const Pk<T, VEC> Z = ld<T, VEC>(z + i);
            Pk<T, VEC> P = ld<T, VEC>(p + i);
#pragma unroll
            for (int v = 0; v < VEC; ++v)
                if (act[v]) P.a[v] = Z.a[v] + be[v] * P.a[v];
            st<T, VEC>(p + i, P);
        }
        if (y) st<T, VEC>(y + i, zero);
    }
}

template <typename T>
void launch_p_update(hipStream_t s, long nrows, int MB, int nm, const T* z, T* p, const double* beta, const int* active,
                     T* y)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nrows, 256 / QB);
    if (VEC == 4) hipLaunchKernelGGL((k_p_update<T, 4>), dim3(g), dim3(256), 0, s, nrows, MB, nm, z, p, beta, active, y);
    else hipLaunchKernelGGL((k_p_update<T, 1>), dim3(g), dim3(256), 0, s, nrows, MB, nm, z, p, beta, active, y);
}
template void launch_p_update<double>(hipStream_t, long, int, int, const double*, double*, const double*, const int*, double*);
template void launch_p_update<float>(hipStream_t, long, int, int, const float*, float*, const double*, const int*, float*);

// flexible CG: x += a p, r -= a Ap; partial r.r
template <int VEC>
__global__ __launch_bounds__(256) void k_xr_update(long nrows, int MB, int nm, double* __restrict__ x,
                                                  double* __restrict__ r, const double* __restrict__ p,
                                                  const double* __restrict__ Ap, const double* __restrict__ alpha,
                                                  const int* __restrict__ active, double* __restrict__ partial)
{
    const int QB = MB / VEC, rpb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    double acc[1][VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) acc[0][v] = 0.0;
    bool act[4];
    if (member_mask(active, m0, VEC, nm, act)) {
        double al[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) al[v] = act[v] ? alpha[m0 + v] : 0.0;
        for (long row = (long)blockIdx.x * rpb + t / QB; row < nrows; row += (long)gridDim.x * rpb) {
            const long i = row * MB + m0;
            Pk<double, VEC> X = ld<double, VEC>(x + i), R = ld<double, VEC>(r + i);
            const Pk<double, VEC> P = ld<double, VEC>(p + i), A = ld<double, VEC>(Ap + i);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                X.a[v] += al[v] * P.a[v];
                R.a[v] -= al[v] * A.a[v];
                acc[0][v] += R.a[v] * R.a[v];
            }
            st<double, VEC>(x + i, X);
            st<double, VEC>(r + i, R);
        }
    }
    block_partials<1, VEC>(acc, QB, MB, partial);
}

void launch_xr_update(hipStream_t s, long nrows, int MB, int nm, double* x, double* r, const double* p, const double* Ap,
                      const double* alpha, const int* active, double* partial, int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nrows, 256 / QB);
    *nblk = g;
    if (VEC == 4) hipLaunchKernelGGL((k_xr_update<4>), dim3(g), dim3(256), 0, s, nrows, MB, nm, x, r, p, Ap, alpha, active, partial);
    else hipLaunchKernelGGL((k_xr_update<1>), dim3(g), dim3(256), 0, s, nrows, MB, nm, x, r, p, Ap, alpha, active, partial);
}

// inner FP32 PCG start on A w = r: ir = r, iz = 0, ip = P ir; partials
// (ir.ir, ir.ip).  w and iAp need no clearing: the first iteration writes
// them before reading them, and a member outside the mask multiplies its
// (finite, stale) iAp by a zero alpha.
template <int VEC>
__global__ __launch_bounds__(256) void k_inner_start(int nn, int MB, int nm, const double* __restrict__ r,
                                                    const float* __restrict__ pinv32, float* __restrict__ ir,
                                                    float* __restrict__ iz, float* __restrict__ ip,
                                                    float* __restrict__ w, float* __restrict__ iAp,
                                                    const int* __restrict__ active, double* __restrict__ partial)
{
    const int QB = MB / VEC, npb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    double acc[2][VEC];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
    bool act[4];
    const bool any = member_mask(active, m0, VEC, nm, act);
    Pk<float, VEC> zero;
#pragma unroll
    for (int v = 0; v < VEC; ++v) zero.a[v] = 0.0f;
    for (long node = (long)blockIdx.x * npb + t / QB; node < nn; node += (long)gridDim.x * npb) {
        if (any) {
            Pk<float, VEC> R[3], W[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const Pk<double, VEC> Rd = ld<double, VEC>(r + (node * 3 + c) * MB + m0);
#pragma unroll
                for (int v = 0; v < VEC; ++v) R[c].a[v] = act[v] ? (float)Rd.a[v] : 0.0f;
            }
            pinv_apply<float, VEC>(pinv32, node, MB, m0, R, W);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * MB + m0;
                st<float, VEC>(ir + i, R[c]);
                st<float, VEC>(iz + i, zero);
                st<float, VEC>(ip + i, W[c]);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    acc[0][v] += (double)R[c].a[v] * (double)R[c].a[v];
                    acc[1][v] += (double)R[c].a[v] * (double)W[c].a[v];
                }
            }
        }
    }
    block_partials<2, VEC>(acc, QB, MB, partial);
}

void launch_inner_start(hipStream_t s, int nn, int MB, int nm, const double* r, const float* pinv32, float* ir,
                        float* iz, float* ip, float* w, float* iAp, const int* active, double* partial, int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nn, 256 / QB);
    *nblk = g;
    if (VEC == 4) hipLaunchKernelGGL((k_inner_start<4>), dim3(g), dim3(256), 0, s, nn, MB, nm, r, pinv32, ir, iz, ip, w, iAp, active, partial);
    else hipLaunchKernelGGL((k_inner_start<1>), dim3(g), dim3(256), 0, s, nn, MB, nm, r, pinv32, ir, iz, ip, w, iAp, active, partial);
}

// inner: ir -= a iAp, w = P ir; partials (ir.ir, ir.w).  (iz += a ip is
// done with the p update, which reads ip anyway: 4 B less per DOF.)
template <int VEC>
__global__ __launch_bounds__(256) void k_inner_update(int nn, int MB, int nm, float* __restrict__ ir,
                                                     float* __restrict__ w, const float* __restrict__ iAp,
                                                     const float* __restrict__ pinv32,
                                                     const double* __restrict__ ialpha,
                                                     const int* __restrict__ iactive, double* __restrict__ partial)
{
    const int QB = MB / VEC, npb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    double acc[2][VEC];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
    bool act[4];
    if (member_mask(iactive, m0, VEC, nm, act)) {
        float al[VEC];
#pragma unroll
        for (int v = 0; v < VEC; ++v) al[v] = act[v] ? (float)ialpha[m0 + v] : 0.0f;
        for (long node = (long)blockIdx.x * npb + t / QB; node < nn; node += (long)gridDim.x * npb) {
            Pk<float, VEC> R[3], W[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * MB + m0;
                const Pk<float, VEC> A = ld<float, VEC>(iAp + i);
                R[c] = ld<float, VEC>(ir + i);
#pragma unroll
                for (int v = 0; v < VEC; ++v) R[c].a[v] -= al[v] * A.a[v];
                st<float, VEC>(ir + i, R[c]);
            }
            pinv_apply<float, VEC>(pinv32, node, MB, m0, R, W);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                st<float, VEC>(w + (node * 3 + c) * MB + m0, W[c]);
#pragma unroll
                for (int v = 0; v < VEC; ++v) {
                    acc[0][v] += (double)R[c].a[v] * (double)R[c].a[v];
                    acc[1][v] += (double)R[c].a[v] * (double)W[c].a[v];
                }
            }
        }
    }
    block_partials<2, VEC>(acc, QB, MB, partial);
}

void launch_inner_update(hipStream_t s, int nn, int MB, int nm, float* ir, float* w, const float* iAp,
                         const float* pinv32, const double* ialpha, const int* iactive, double* partial, int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nn, 256 / QB);
    *nblk = g;
    if (VEC == 4) hipLaunchKernelGGL((k_inner_update<4>), dim3(g), dim3(256), 0, s, nn, MB, nm, ir, w, iAp, pinv32, ialpha, iactive, partial);
    else hipLaunchKernelGGL((k_inner_update<1>), dim3(g), dim3(256), 0, s, nn, MB, nm, ir, w, iAp, pinv32, ialpha, iactive, partial);
}

// inner: iz += a ip (with this iteration's ip), then ip = w + b ip, for the
// members whose alpha was formed this iteration (upd); a member that has just
// converged takes its last iz update, and its ip is not used again
template <int VEC>
__global__ __launch_bounds__(256) void k_inner_pz(long nrows, int MB, int nm, float* __restrict__ iz,
                                                 float* __restrict__ ip, const float* __restrict__ w,
                                                 const double* __restrict__ ialpha, const double* __restrict__ ibeta,
                                                 const int* __restrict__ upd)
{
    const int QB = MB / VEC, rpb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    bool act[4];
    if (!member_mask(upd, m0, VEC, nm, act)) return;
    float al[VEC], be[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        al[v] = act[v] ? (float)ialpha[m0 + v] : 0.0f;
        be[v] = act[v] ? (float)ibeta[m0 + v] : 0.0f;
    }
    for (long row = (long)blockIdx.x * rpb + t / QB; row < nrows; row += (long)gridDim.x * rpb) {
        const long i = row * MB + m0;
        Pk<float, VEC> Z = ld<float, VEC>(iz + i), P = ld<float, VEC>(ip + i);
        const Pk<float, VEC> W = ld<float, VEC>(w + i);
#pragma unroll
        for (int v = 0; v < VEC; ++v)
            if (act[v]) {
                Z.a[v] += al[v] * P.a[v];
                P.a[v] = W.a[v] + be[v] * P.a[v];
            }
        st<float, VEC>(iz + i, Z);
        st<float, VEC>(ip + i, P);
    }
}

void launch_inner_pz(hipStream_t s, long nrows, int MB, int nm, float* iz, float* ip, const float* w,
                     const double* ialpha, const double* ibeta, const int* upd)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nrows, 256 / QB);
    if (VEC == 4) hipLaunchKernelGGL((k_inner_pz<4>), dim3(g), dim3(256), 0, s, nrows, MB, nm, iz, ip, w, ialpha, ibeta, upd);
    else hipLaunchKernelGGL((k_inner_pz<1>), dim3(g), dim3(256), 0, s, nrows, MB, nm, iz, ip, w, ialpha, ibeta, upd);
}

// preconditioner output z = iz (FP64) for outer-active members (0 for the
// others, whose z is not used again in the step); partials (z.Ap, z.r)
template <int VEC>
__global__ __launch_bounds__(256) void k_inner_out(long nrows, int MB, int nm, const float* __restrict__ iz,
                                                  double* __restrict__ z, const double* __restrict__ Ap,
                                                  const double* __restrict__ r, const int* __restrict__ active,
                                                  double* __restrict__ partial)
{
    const int QB = MB / VEC, rpb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    double acc[2][VEC];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int v = 0; v < VEC; ++v) acc[k][v] = 0.0;
    bool act[4];
    if (member_mask(active, m0, VEC, nm, act)) {
        for (long row = (long)blockIdx.x * rpb + t / QB; row < nrows; row += (long)gridDim.x * rpb) {
            const long i = row * MB + m0;
            const Pk<float, VEC> Zf = ld<float, VEC>(iz + i);
            const Pk<double, VEC> A = ld<double, VEC>(Ap + i), R = ld<double, VEC>(r + i);
            Pk<double, VEC> Z;
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                Z.a[v] = act[v] ? (double)Zf.a[v] : 0.0;
                acc[0][v] += Z.a[v] * A.a[v];
                acc[1][v] += Z.a[v] * R.a[v];
            }
            st<double, VEC>(z + i, Z);
        }
    }
    block_partials<2, VEC>(acc, QB, MB, partial);
}

void launch_inner_out(hipStream_t s, long nrows, int MB, int nm, const float* iz, double* z, const double* Ap,
                      const double* r, const int* active, double* partial, int* nblk)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nrows, 256 / QB);
    *nblk = g;
    if (VEC == 4) hipLaunchKernelGGL((k_inner_out<4>), dim3(g), dim3(256), 0, s, nrows, MB, nm, iz, z, Ap, r, active, partial);
    else hipLaunchKernelGGL((k_inner_out<1>), dim3(g), dim3(256), 0, s, nrows, MB, nm, iz, z, Ap, r, active, partial);
}

// ---------------------------------------------------------------------------
// inner CG of the convergence tail on compact rows (lane k = member tl[1 + k],
// G lanes per row): the start, update and p/z steps above, partials in the
// full [block][MB] layout
// ---------------------------------------------------------------------------

__device__ __forceinline__ int tail_member(const int* __restrict__ tl, int k, int G)
{
    return k < min(tl[0], G) ? tl[1 + k] : -1;
}

template <int G, bool CR>
__global__ __launch_bounds__(256) void k_tail_start(int nn, int MB, int nm, const int* __restrict__ tl,
                                                   const double* __restrict__ r, const float* __restrict__ cpinv,
                                                   float* __restrict__ cir, float* __restrict__ ciz,
                                                   float* __restrict__ cip, const int* __restrict__ active,
                                                   double* __restrict__ partial)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    double acc[2] = {0.0, 0.0};
    if (m >= 0 && m < nm && (!active || active[m])) {
        for (long node = (long)blockIdx.x * NPB + t / G; node < nn; node += (long)gridDim.x * NPB) {
            Pk<float, 1> R[3], W[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) R[c].a[0] = (float)(CR ? r[(node * 3 + c) * G + k] : r[(node * 3 + c) * MB + m]);
            pinv_apply<float, 1>(cpinv, node, G, k, R, W);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * G + k;
                cir[i] = R[c].a[0];
                ciz[i] = 0.0f;
                cip[i] = W[c].a[0];
                acc[0] += (double)R[c].a[0] * (double)R[c].a[0];
                acc[1] += (double)R[c].a[0] * (double)W[c].a[0];
            }
        }
    }
    tail_partials<2, G>(acc, MB, m, partial, 0, gridDim.x);
}

template <int G>
__global__ __launch_bounds__(256) void k_tail_update(int nn, int MB, int nm, const int* __restrict__ tl,
                                                    float* __restrict__ cir, float* __restrict__ cw,
                                                    const float* __restrict__ ciAp, const float* __restrict__ cpinv,
                                                    const double* __restrict__ ialpha,
                                                    const int* __restrict__ iactive, double* __restrict__ partial)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    double acc[2] = {0.0, 0.0};
    if (m >= 0 && m < nm && iactive[m]) {
        const float al = (float)ialpha[m];
        for (long node = (long)blockIdx.x * NPB + t / G; node < nn; node += (long)gridDim.x * NPB) {
            Pk<float, 1> R[3], W[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * G + k;
                R[c].a[0] = cir[i] - al * ciAp[i];
                cir[i] = R[c].a[0];
            }
            pinv_apply<float, 1>(cpinv, node, G, k, R, W);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cw[(node * 3 + c) * G + k] = W[c].a[0];
                acc[0] += (double)R[c].a[0] * (double)R[c].a[0];
                acc[1] += (double)R[c].a[0] * (double)W[c].a[0];
            }
        }
    }
    tail_partials<2, G>(acc, MB, m, partial, 0, gridDim.x);
}

template <int G>
__global__ __launch_bounds__(256) void k_tail_pz(long nrows, int nm, const int* __restrict__ tl,
                                                float* __restrict__ ciz, float* __restrict__ cip,
                                                const float* __restrict__ cw, const double* __restrict__ ialpha,
                                                const double* __restrict__ ibeta, const int* __restrict__ upd)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    if (m < 0 || m >= nm || !upd[m]) return;
    const float al = (float)ialpha[m], be = (float)ibeta[m];
    for (long row = (long)blockIdx.x * NPB + t / G; row < nrows; row += (long)gridDim.x * NPB) {
        const long i = row * G + k;
        const float P = cip[i];
        ciz[i] += al * P;
        cip[i] = cw[i] + be * P;
    }
}

// FP64 PCG on the compact rows (the tail of the plain FP64 path): the update
// of k_pcg_update and the p step of k_p_update for the listed members
template <int G>
__global__ __launch_bounds__(256) void k_tail_pcg_update(int nn, int MB, int nm, const int* __restrict__ tl,
                                                        double* __restrict__ cx, double* __restrict__ cr,
                                                        double* __restrict__ cz, const double* __restrict__ cp,
                                                        const double* __restrict__ cAp,
                                                        const double* __restrict__ cpinv,
                                                        const double* __restrict__ alpha,
                                                        const int* __restrict__ active, double* __restrict__ partial)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    double acc[2] = {0.0, 0.0};
    if (m >= 0 && m < nm && active[m]) {
        const double al = alpha[m];
        for (long node = (long)blockIdx.x * NPB + t / G; node < nn; node += (long)gridDim.x * NPB) {
            Pk<double, 1> R[3], Z[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const long i = (node * 3 + c) * G + k;
                cx[i] += al * cp[i];
                R[c].a[0] = cr[i] - al * cAp[i];
                cr[i] = R[c].a[0];
            }
            pinv_apply<double, 1>(cpinv, node, G, k, R, Z);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                cz[(node * 3 + c) * G + k] = Z[c].a[0];
                acc[0] += R[c].a[0] * R[c].a[0];
                acc[1] += R[c].a[0] * Z[c].a[0];
            }
        }
    }
    tail_partials<2, G>(acc, MB, m, partial, 0, gridDim.x);
}

template <int G>
__global__ __launch_bounds__(256) void k_tail_p_update(long nrows, int nm, const int* __restrict__ tl,
                                                      const double* __restrict__ cz, double* __restrict__ cp,
                                                      const double* __restrict__ beta,
                                                      const int* __restrict__ active)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    if (m < 0 || m >= nm || !active[m]) return;
    const double be = beta[m];
    for (long row = (long)blockIdx.x * NPB + t / G; row < nrows; row += (long)gridDim.x * NPB) {
        const long i = row * G + k;
        cp[i] = cz[i] + be * cp[i];
    }
}

void launch_tail_pcg_update(hipStream_t s, int nn, int MB, int nm, int G, const int* tl, double* cx, double* cr,
                            double* cz, const double* cp, const double* cAp, const double* cpinv,
                            const double* alpha, const int* active, double* partial, int* nblk)
{
    const int g = grid_for(nn, 256 / G);
    *nblk = g;
    if (G == 16)
        hipLaunchKernelGGL((k_tail_pcg_update<16>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, cx, cr, cz, cp, cAp, cpinv,
                           alpha, active, partial);
    else
        hipLaunchKernelGGL((k_tail_pcg_update<32>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, cx, cr, cz, cp, cAp, cpinv,
                           alpha, active, partial);
}

void launch_tail_p_update(hipStream_t s, long nrows, int nm, int G, const int* tl, const double* cz, double* cp,
                          const double* beta, const int* active)
{
    const int g = grid_for(nrows, 256 / G);
    if (G == 16) hipLaunchKernelGGL((k_tail_p_update<16>), dim3(g), dim3(256), 0, s, nrows, nm, tl, cz, cp, beta, active);
    else hipLaunchKernelGGL((k_tail_p_update<32>), dim3(g), dim3(256), 0, s, nrows, nm, tl, cz, cp, beta, active);
}

void launch_tail_start(hipStream_t s, int nn, int MB, int nm, int G, const int* tl, const double* r, bool r_compact,
                       const float* cpinv, float* cir, float* ciz, float* cip, const int* active, double* partial,
                       int* nblk)
{
    const int g = grid_for(nn, 256 / G);
    *nblk = g;
    if (G == 16 && r_compact)
        hipLaunchKernelGGL((k_tail_start<16, true>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, r, cpinv, cir, ciz, cip, active, partial);
    else if (G == 16)
        hipLaunchKernelGGL((k_tail_start<16, false>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, r, cpinv, cir, ciz, cip, active, partial);
    else if (r_compact)
        hipLaunchKernelGGL((k_tail_start<32, true>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, r, cpinv, cir, ciz, cip, active, partial);
    else
        hipLaunchKernelGGL((k_tail_start<32, false>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, r, cpinv, cir, ciz, cip, active, partial);
}

// outer flexible CG of the mixed path on the compact rows: x += a p, r -= a Ap
// with the partial r.r (k_xr_update), and z = iz for the outer-active members
// with the partials (z.Ap, z.r) (k_inner_out)
template <int G>
__global__ __launch_bounds__(256) void k_tail_xr_update(long nrows, int MB, int nm, const int* __restrict__ tl,
                                                       double* __restrict__ cx, double* __restrict__ cr,
                                                       const double* __restrict__ cp, const double* __restrict__ cAp,
                                                       const double* __restrict__ alpha,
                                                       const int* __restrict__ active, double* __restrict__ partial)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    double acc[1] = {0.0};
    if (m >= 0 && m < nm && active[m]) {
        const double al = alpha[m];
        for (long row = (long)blockIdx.x * NPB + t / G; row < nrows; row += (long)gridDim.x * NPB) {
            const long i = row * G + k;
            cx[i] += al * cp[i];
            const double R = cr[i] - al * cAp[i];
            cr[i] = R;
            acc[0] += R * R;
        }
    }
    tail_partials<1, G>(acc, MB, m, partial, 0, gridDim.x);
}

template <int G>
__global__ __launch_bounds__(256) void k_tail_inner_out(long nrows, int MB, int nm, const int* __restrict__ tl,
                                                       const float* __restrict__ ciz, double* __restrict__ cz,
                                                       const double* __restrict__ cAp, const double* __restrict__ cr,
                                                       const int* __restrict__ active, double* __restrict__ partial)
{
    constexpr int NPB = 256 / G;
    const int t = threadIdx.x, k = t % G;
    const int m = tail_member(tl, k, G);
    double acc[2] = {0.0, 0.0};
    if (m >= 0 && m < nm) {
        const bool act = active[m] != 0;
        for (long row = (long)blockIdx.x * NPB + t / G; row < nrows; row += (long)gridDim.x * NPB) {
            const long i = row * G + k;
            const double Z = act ? (double)ciz[i] : 0.0;
            acc[0] += Z * cAp[i];
            acc[1] += Z * cr[i];
            cz[i] = Z;
        }
    }
    tail_partials<2, G>(acc, MB, m, partial, 0, gridDim.x);
}

void launch_tail_xr_update(hipStream_t s, long nrows, int MB, int nm, int G, const int* tl, double* cx, double* cr,
                           const double* cp, const double* cAp, const double* alpha, const int* active,
                           double* partial, int* nblk)
{
    const int g = grid_for(nrows, 256 / G);
    *nblk = g;
    if (G == 16)
        hipLaunchKernelGGL((k_tail_xr_update<16>), dim3(g), dim3(256), 0, s, nrows, MB, nm, tl, cx, cr, cp, cAp, alpha, active, partial);
    else
        hipLaunchKernelGGL((k_tail_xr_update<32>), dim3(g), dim3(256), 0, s, nrows, MB, nm, tl, cx, cr, cp, cAp, alpha, active, partial);
}

void launch_tail_inner_out(hipStream_t s, long nrows, int MB, int nm, int G, const int* tl, const float* ciz,
                           double* cz, const double* cAp, const double* cr, const int* active, double* partial,
                           int* nblk)
{
    const int g = grid_for(nrows, 256 / G);
    *nblk = g;
    if (G == 16)
        hipLaunchKernelGGL((k_tail_inner_out<16>), dim3(g), dim3(256), 0, s, nrows, MB, nm, tl, ciz, cz, cAp, cr, active, partial);
    else
        hipLaunchKernelGGL((k_tail_inner_out<32>), dim3(g), dim3(256), 0, s, nrows, MB, nm, tl, ciz, cz, cAp, cr, active, partial);
}

void launch_tail_update(hipStream_t s, int nn, int MB, int nm, int G, const int* tl, float* cir, float* cw,
                        const float* ciAp, const float* cpinv, const double* ialpha, const int* iactive,
                        double* partial, int* nblk)
{
    const int g = grid_for(nn, 256 / G);
    *nblk = g;
    if (G == 16) hipLaunchKernelGGL((k_tail_update<16>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, cir, cw, ciAp, cpinv, ialpha, iactive, partial);
    else hipLaunchKernelGGL((k_tail_update<32>), dim3(g), dim3(256), 0, s, nn, MB, nm, tl, cir, cw, ciAp, cpinv, ialpha, iactive, partial);
}

void launch_tail_pz(hipStream_t s, long nrows, int nm, int G, const int* tl, float* ciz, float* cip, const float* cw,
                    const double* ialpha, const double* ibeta, const int* upd)
{
    const int g = grid_for(nrows, 256 / G);
    if (G == 16) hipLaunchKernelGGL((k_tail_pz<16>), dim3(g), dim3(256), 0, s, nrows, nm, tl, ciz, cip, cw, ialpha, ibeta, upd);
    else hipLaunchKernelGGL((k_tail_pz<32>), dim3(g), dim3(256), 0, s, nrows, nm, tl, ciz, cip, cw, ialpha, ibeta, upd);
}

// ---------------------------------------------------------------------------
// Chebyshev inner solve: A z = r by the Chebyshev iteration on the block-
// Jacobi preconditioned operator (Saad, Iterative Methods for Sparse Linear
// Systems, 2nd ed., Algorithm 12.1), with the spectrum bounds of each member
// taken from the Lanczos matrix of an inner CG solve of the same step.  It
// needs no inner products, so an iteration is the operator plus one update.
// ---------------------------------------------------------------------------

// eigenvalues of the Lanczos tridiagonal below x (Sturm count); T from the CG
// coefficients: T_00 = 1/a_0, T_ii = 1/a_i + b_{i-1}/a_{i-1}, T_{i,i+1}^2 = b_i/a_i^2
__device__ int lanczos_count(const double* __restrict__ lz, int MB, int m, int n, double x)
{
    int cnt = 0;
    double q = 1.0;
    for (int i = 0; i < n; ++i) {
        const double ai = lz[(long)i * MB + m];
        double diag = 1.0 / ai;
        double off2 = 0.0;
        if (i > 0) {
            const double ap = lz[(long)(i - 1) * MB + m], bp = lz[(long)(kLanczosMax + i - 1) * MB + m];
            diag += bp / ap;
            off2 = bp / (ap * ap);
        }
        q = diag - x - (i > 0 ? off2 / q : 0.0);
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// Ritz extremes of member m's Lanczos matrix (0, 0 without coefficients)
__device__ void lanczos_extremes(const CgScalars& cs, int MB, int m, double* lmin, double* lmax)
{
    const int n = cs.inner_iters[m] < kLanczosMax ? cs.inner_iters[m] : kLanczosMax;
    *lmin = *lmax = 0.0;
    if (n <= 0) return;
    // Gershgorin interval of T, then bisection on the Sturm count
    double g0 = 1e300, g1 = -1e300;
    for (int i = 0; i < n; ++i) {
        const double ai = cs.lz[(long)i * MB + m];
        double diag = 1.0 / ai, rad = 0.0;
        if (i > 0) {
            const double ap = cs.lz[(long)(i - 1) * MB + m], bp = cs.lz[(long)(kLanczosMax + i - 1) * MB + m];
            diag += bp / ap;
            rad += sqrt(fabs(bp)) / fabs(ap);
        }
        if (i + 1 < n) rad += sqrt(fabs(cs.lz[(long)(kLanczosMax + i) * MB + m])) / fabs(ai);
        g0 = fmin(g0, diag - rad);
        g1 = fmax(g1, diag + rad);
    }
    if (!(g1 > g0)) return;  // non-finite coefficients
    double a = g0, b = g1;  // smallest: count(a) = 0, count(b) >= 1
    for (int it = 0; it < 200 && b - a > 1e-12 * fabs(b); ++it) {
        const double x = 0.5 * (a + b);
        if (lanczos_count(cs.lz, MB, m, n, x) >= 1) b = x;
        else a = x;
    }
    *lmin = 0.5 * (a + b);
    a = g0; b = g1;  // largest: count(a) < n, count(b) = n
    for (int it = 0; it < 200 && b - a > 1e-12 * fabs(b); ++it) {
        const double x = 0.5 * (a + b);
        if (lanczos_count(cs.lz, MB, m, n, x) >= n) b = x;
        else a = x;
    }
    *lmax = 0.5 * (a + b);
}

// One block.  Lower bound per member: its smallest Ritz value (x lo_scale).
// Upper bound shared by the members and never lowered: hi_scale x the
// largest Ritz value over the members and the steps so far (bounds[2 MB]).
// A Ritz value lies inside the spectrum, so the largest one can fall short
// of the true largest eigenvalue when a member's residual has little weight
// there, and Chebyshev amplifies the components above the upper bound; the
// members share the mesh, whose consistent mass sets the top of the spectrum.
__global__ __launch_bounds__(256) void k_cheb_bounds(int MB, int nm, CgScalars cs, int degree, double lo_scale,
                                                    double hi_scale, float* __restrict__ cheb,
                                                    double* __restrict__ bounds)
{
    __shared__ double smax[256];
    const int t = threadIdx.x;
    double mx = 0.0;
    for (int m = t; m < nm; m += 256) {
        double lmin, lmax;
        lanczos_extremes(cs, MB, m, &lmin, &lmax);
        if (lmax > 0.0 && isfinite(lmax)) mx = fmax(mx, lmax);
        bounds[m] = (lmin > 0.0 && isfinite(lmin) && lmin < lmax) ? lmin * lo_scale : 0.0;
    }
    smax[t] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) smax[t] = fmax(smax[t], smax[t + s]);
        __syncthreads();
    }
    const double hi = fmax(smax[0] * hi_scale, bounds[2 * MB]);
    __syncthreads();
    if (t == 0) bounds[2 * MB] = hi;
    if (!(hi > 0.0)) return;
    for (int m = t; m < nm; m += 256) {
        double lo = bounds[m];
        if (!(lo > 0.0) || lo > 0.99 * hi) lo = 0.01 * hi;  // no usable estimate
        bounds[m] = lo;
        bounds[MB + m] = hi;
        const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
        double rho = 1.0 / sigma;
        for (int k = 0; k < degree && k < kChebMax; ++k) {
            const double rn = 1.0 / (2.0 * sigma - rho);
            cheb[(long)(2 * k) * MB + m] = (float)(rn * rho);
            cheb[(long)(2 * k + 1) * MB + m] = (float)(2.0 * rn / delta);
            rho = rn;
        }
        cheb[(long)(2 * kChebMax) * MB + m] = (float)(1.0 / theta);
    }
}

void launch_cheb_bounds(hipStream_t s, int MB, int nm, CgScalars cs, int degree, double lo_scale, double hi_scale,
                        float* cheb, double* bounds)
{
    hipLaunchKernelGGL(k_cheb_bounds, dim3(1), dim3(256), 0, s, MB, nm, cs, degree, lo_scale, hi_scale, cheb, bounds);
}

// Upper spectrum bound from inner CG iterations on a random right-hand side
// (which weights every eigenvector): bounds[2 MB] = max(bounds[2 MB], scale x
// the largest Ritz value over the members).
__global__ __launch_bounds__(256) void k_cheb_hi_estimate(int MB, int nm, CgScalars cs, double scale,
                                                         double* __restrict__ bounds)
{
    __shared__ double smax[256];
    const int t = threadIdx.x;
    double mx = 0.0;
    for (int m = t; m < nm; m += 256) {
        double lmin, lmax;
        lanczos_extremes(cs, MB, m, &lmin, &lmax);
        if (lmax > 0.0 && isfinite(lmax)) mx = fmax(mx, lmax);
    }
    smax[t] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s) smax[t] = fmax(smax[t], smax[t + s]);
        __syncthreads();
    }
    if (t == 0) bounds[2 * MB] = fmax(bounds[2 * MB], smax[0] * scale);
}

void launch_cheb_hi_estimate(hipStream_t s, int MB, int nm, CgScalars cs, double scale, double* bounds)
{
    hipLaunchKernelGGL(k_cheb_hi_estimate, dim3(1), dim3(256), 0, s, MB, nm, cs, scale, bounds);
}

// x[i] uniform in [-1, 1) from the SplitMix64 sequence (Steele, Lea, Flood,
// OOPSLA 2014) at counter seed + i
__global__ void k_fill_random(double* __restrict__ x, long n, uint64_t seed)
{
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t z = seed + (uint64_t)(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    x[i] = (double)(z >> 11) * 0x1.0p-52 - 1.0;
}

void launch_fill_random(hipStream_t s, double* x, long n, uint64_t seed)
{
    if (n > 0) hipLaunchKernelGGL(k_fill_random, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, seed);
}

// start: ir = r, iz = 0, id = c0 P ir (members outside active: zeros)
template <int VEC>
__global__ __launch_bounds__(256) void k_cheb_start(int nn, int MB, int nm, const double* __restrict__ r,
                                                   const float* __restrict__ pinv32, const float* __restrict__ cheb,
                                                   float* __restrict__ ir, float* __restrict__ iz,
                                                   float* __restrict__ id, const int* __restrict__ active)
{
    const int QB = MB / VEC, npb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    bool act[4];
    if (!member_mask(active, m0, VEC, nm, act)) return;
    float c0[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) c0[v] = cheb[(long)(2 * kChebMax) * MB + m0 + v];
    Pk<float, VEC> zero;
#pragma unroll
    for (int v = 0; v < VEC; ++v) zero.a[v] = 0.0f;
    for (long node = (long)blockIdx.x * npb + t / QB; node < nn; node += (long)gridDim.x * npb) {
        Pk<float, VEC> R[3], W[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const Pk<double, VEC> Rd = ld<double, VEC>(r + (node * 3 + c) * MB + m0);
#pragma unroll
            for (int v = 0; v < VEC; ++v) R[c].a[v] = act[v] ? (float)Rd.a[v] : 0.0f;
        }
        pinv_apply<float, VEC>(pinv32, node, MB, m0, R, W);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long i = (node * 3 + c) * MB + m0;
#pragma unroll
            for (int v = 0; v < VEC; ++v) W[c].a[v] *= c0[v];
            st<float, VEC>(ir + i, R[c]);
            st<float, VEC>(iz + i, zero);
            st<float, VEC>(id + i, W[c]);
        }
    }
}

void launch_cheb_start(hipStream_t s, int nn, int MB, int nm, const double* r, const float* pinv32,
                       const float* cheb, float* ir, float* iz, float* id, const int* active)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nn, 256 / QB);
    if (VEC == 4) hipLaunchKernelGGL((k_cheb_start<4>), dim3(g), dim3(256), 0, s, nn, MB, nm, r, pinv32, cheb, ir, iz, id, active);
    else hipLaunchKernelGGL((k_cheb_start<1>), dim3(g), dim3(256), 0, s, nn, MB, nm, r, pinv32, cheb, ir, iz, id, active);
}

// iteration k after iAp = A id: iz += id, ir -= iAp, id_next = c1_k id + c2_k P ir
// (id_next is not formed on the last iteration)
template <int VEC>
__global__ __launch_bounds__(256) void k_cheb_update(int nn, int MB, int nm, int k, bool last, float* __restrict__ iz,
                                                    float* __restrict__ ir, const float* __restrict__ id,
                                                    const float* __restrict__ iAp, float* __restrict__ id_next,
                                                    const float* __restrict__ pinv32, const float* __restrict__ cheb,
                                                    const int* __restrict__ active)
{
    const int QB = MB / VEC, npb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    bool act[4];
    if (!member_mask(active, m0, VEC, nm, act)) return;
    float c1[VEC], c2[VEC];
#pragma unroll
    for (int v = 0; v < VEC; ++v) {
        c1[v] = cheb[(long)(2 * k) * MB + m0 + v];
        c2[v] = cheb[(long)(2 * k + 1) * MB + m0 + v];
    }
    for (long node = (long)blockIdx.x * npb + t / QB; node < nn; node += (long)gridDim.x * npb) {
        Pk<float, VEC> R[3], D[3], W[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const long i = (node * 3 + c) * MB + m0;
            Pk<float, VEC> Z = ld<float, VEC>(iz + i);
            D[c] = ld<float, VEC>(id + i);
            const Pk<float, VEC> A = ld<float, VEC>(iAp + i);
            R[c] = ld<float, VEC>(ir + i);
#pragma unroll
            for (int v = 0; v < VEC; ++v) {
                if (!act[v]) continue;
                Z.a[v] += D[c].a[v];
                R[c].a[v] -= A.a[v];
            }
            st<float, VEC>(iz + i, Z);
            st<float, VEC>(ir + i, R[c]);
        }
        if (last) continue;
        pinv_apply<float, VEC>(pinv32, node, MB, m0, R, W);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int v = 0; v < VEC; ++v) W[c].a[v] = act[v] ? c1[v] * D[c].a[v] + c2[v] * W[c].a[v] : 0.0f;
            st<float, VEC>(id_next + (node * 3 + c) * MB + m0, W[c]);
        }
    }
}

void launch_cheb_update(hipStream_t s, int nn, int MB, int nm, int k, bool last, float* iz, float* ir,
                        const float* id, const float* iAp, float* id_next, const float* pinv32, const float* cheb,
                        const int* active)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nn, 256 / QB);
    if (VEC == 4) hipLaunchKernelGGL((k_cheb_update<4>), dim3(g), dim3(256), 0, s, nn, MB, nm, k, last, iz, ir, id, iAp, id_next, pinv32, cheb, active);
    else hipLaunchKernelGGL((k_cheb_update<1>), dim3(g), dim3(256), 0, s, nn, MB, nm, k, last, iz, ir, id, iAp, id_next, pinv32, cheb, active);
}

// ---------------------------------------------------------------------------
// per-member scalar logic: one block per member reduces its partials by a
// fixed tree, then thread 0 applies the stage
// ---------------------------------------------------------------------------

__device__ void stage_logic(int stage, int m, int MB, const double S[3], CgScalars& cs, double tol2, int maxit)
{
    switch (stage) {
    case FIN_START:  // S = (b.b, r.r, r.z)
        cs.bb[m] = S[0];
        cs.rr[m] = S[1];
        cs.rz[m] = S[2];
        cs.iters[m] = 0;
        cs.active[m] = cs.stepping[m] && S[0] > 0.0 && S[1] > tol2 * S[0];
        break;
    case FIN_ALPHA:  // S = (p.Ap)
        cs.pAp[m] = S[0];
        cs.alpha[m] = cs.active[m] ? cs.rz[m] / S[0] : 0.0;
        break;
    case FIN_BETA:  // S = (r.r, r.z)
        if (cs.active[m]) {
            cs.iters[m] += 1;
            cs.rr[m] = S[0];
            if (S[0] <= tol2 * cs.bb[m]) {
                cs.active[m] = 0;
            } else if (cs.iters[m] >= maxit) {
                cs.active[m] = 0;
                cs.status[m] = -5;
            } else {
                cs.beta[m] = S[1] / cs.rz[m];
                cs.rz[m] = S[1];
            }
        }
        break;
    case FIN_FCG_START:  // S = (b.b, r.r, -)
        cs.bb[m] = S[0];
        cs.rr[m] = S[1];
        cs.iters[m] = 0;
        cs.inner_total[m] = 0;
        cs.active[m] = cs.stepping[m] && S[0] > 0.0 && S[1] > tol2 * S[0];
        break;
    case FIN_FCG_RZ:  // S = (z.Ap, z.r)
        cs.rz[m] = S[1];
        break;
    case FIN_FCG_RR:  // S = (r.r)
        if (cs.active[m]) {
            cs.iters[m] += 1;
            cs.rr[m] = S[0];
            if (S[0] <= tol2 * cs.bb[m]) cs.active[m] = 0;
            else if (cs.iters[m] >= maxit) { cs.active[m] = 0; cs.status[m] = -5; }
        }
        break;
    case FIN_FCG_BETA:  // S = (z.Ap, z.r): flexible (Polak-Ribiere) beta
        if (cs.active[m]) {
            cs.beta[m] = -cs.alpha[m] * S[0] / cs.rz[m];
            cs.rz[m] = S[1];
        }
        break;
    case FIN_IN_START:  // S = (ir.ir, ir.w)
        cs.ir0[m] = S[0];
        cs.irz[m] = S[1];
        cs.inner_iters[m] = 0;
        cs.inner_active[m] = cs.active[m] && S[0] > 0.0;
        break;
    case FIN_IN_ALPHA:  // S = (ip.iAp)
        cs.ialpha[m] = cs.inner_active[m] ? cs.irz[m] / S[0] : 0.0;
        cs.inner_upd[m] = cs.inner_active[m];
        if (cs.inner_active[m] && cs.inner_iters[m] < kLanczosMax)
            cs.lz[(long)cs.inner_iters[m] * MB + m] = cs.ialpha[m];
        break;
    case FIN_IN_BETA:  // S = (ir.ir, ir.w)
        if (cs.inner_active[m]) {
            cs.inner_iters[m] += 1;
            cs.inner_total[m] += 1;
            if (S[0] <= tol2 * cs.ir0[m] || cs.inner_iters[m] >= maxit) {
                cs.inner_active[m] = 0;
            } else {
                cs.ibeta[m] = S[1] / cs.irz[m];
                cs.irz[m] = S[1];
                if (cs.inner_iters[m] <= kLanczosMax)
                    cs.lz[(long)(kLanczosMax + cs.inner_iters[m] - 1) * MB + m] = cs.ibeta[m];
            }
        }
        break;
    case FIN_CHEB_COUNT:  // maxit = the Chebyshev degree
        if (cs.active[m]) cs.inner_total[m] += maxit;
        break;
    case FIN_EST_START:  // S = (ir.ir, ir.w)
        cs.ir0[m] = S[0];
        cs.irz[m] = S[1];
        cs.inner_iters[m] = 0;
        cs.inner_active[m] = cs.stepping[m] && S[0] > 0.0;
        break;
    }
}

__global__ __launch_bounds__(256) void k_finalize(int stage, int nd, int MB, int nm, const double* __restrict__ partial,
                                                 int nblk, CgScalars cs, double tol2, int maxit)
{
    const int m = blockIdx.x;
    if (m >= nm) return;
    __shared__ double sh[3][256];
    const int t = threadIdx.x;
    for (int k = 0; k < 3; ++k) {
        double a = 0.0;
        if (k < nd)
            for (int b = t; b < nblk; b += 256) a += partial[((long)k * nblk + b) * MB + m];
        sh[k][t] = a;
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
            for (int k = 0; k < 3; ++k) sh[k][t] += sh[k][t + s];
        __syncthreads();
    }
    if (t == 0) {
        double S[3] = {sh[0][0], sh[1][0], sh[2][0]};
        stage_logic(stage, m, MB, S, cs, tol2, maxit);
    }
}

void launch_finalize(hipStream_t s, FinalizeStage st, int nd, int MB, int nm, const double* partial, int nblk,
                     CgScalars cs, double tol2, int maxit)
{
    hipLaunchKernelGGL(k_finalize, dim3(nm), dim3(256), 0, s, (int)st, nd, MB, nm, partial, nblk, cs, tol2, maxit);
}

}  // namespace nlth

namespace nlth {

// members whose right-hand side is zero take du = 0 (Eq. 1 with b = 0)
template <int VEC>
__global__ __launch_bounds__(256) void k_zero_if_b0(long nrows, int MB, int nm, double* __restrict__ x,
                                                   const double* __restrict__ bb, const int* __restrict__ stepping)
{
    const int QB = MB / VEC, rpb = 256 / QB;
    const int t = threadIdx.x, q = t % QB, m0 = q * VEC;
    bool zero[4], any = false;
    for (int v = 0; v < VEC; ++v) {
        const int m = m0 + v;
        zero[v] = m < nm && stepping[m] && bb[m] == 0.0;
        any |= zero[v];
    }
    if (!any) return;
    for (long row = (long)blockIdx.x * rpb + t / QB; row < nrows; row += (long)gridDim.x * rpb) {
        Pk<double, VEC> X = ld<double, VEC>(x + row * MB + m0);
        for (int v = 0; v < VEC; ++v)
            if (zero[v]) X.a[v] = 0.0;
        st<double, VEC>(x + row * MB + m0, X);
    }
}

void launch_zero_if_b0(hipStream_t s, long nrows, int MB, int nm, double* x, const double* bb, const int* stepping)
{
    const int VEC = vec_of(MB), QB = MB / VEC;
    const int g = grid_for(nrows, 256 / QB);
    if (VEC == 4) hipLaunchKernelGGL((k_zero_if_b0<4>), dim3(g), dim3(256), 0, s, nrows, MB, nm, x, bb, stepping);
    else hipLaunchKernelGGL((k_zero_if_b0<1>), dim3(g), dim3(256), 0, s, nrows, MB, nm, x, bb, stepping);
}

}  // namespace nlth
