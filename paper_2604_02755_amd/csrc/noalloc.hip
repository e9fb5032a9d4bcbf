// Allocation-free form of the diagnostic operator application, for callers
// that cannot allocate device memory: code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc.  The caller passes device
// buffers for the inputs and the output; every intermediate (the material
// table, D and h in the library's storage layout, x and y in storage node
// order, the element outputs) lives in one file-scope device array of
// kScratchBytes that each device the library runs on holds until the process
// ends.  Its device address comes from hipGetSymbolAddress, taken once per
// device when a context is created on it (in host code the array's name is
// only a host-side stand-in).  The kernels are those of nlth_apply_operator's
// FP64 path (one member slot: element outputs, then the node gather, then the
// dashpot), so the two entry points give the same results.
#include <math.h>
#include <string.h>

#include <cstdio>

#include "runtime.hpp"

namespace nlth {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // per device
constexpr int kNoAllocMaxLayers = 32;
constexpr int kScratchDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices];

// Device address of `scratch` on `device`, which must be current; taken once
// per device and kept.
void scratch_setup(int device)
{
    if (device < 0 || device >= kScratchDevices) throw Error{NLTH_EDEVICE, "device index beyond the scratch table"};
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_ptr[device]) return;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        throw Error{NLTH_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch_ptr[device] = p;
}

static char* scratch_of(int device)
{
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return (device >= 0 && device < kScratchDevices) ? (char*)g_scratch_ptr[device] : nullptr;
}

// per-layer material of member 0, passed by value (MB = 1 layout of the table)
struct LayerMat {
    int n;  // n_layers * MAT_N entries
    double v[kNoAllocMaxLayers * MAT_N];
};

__global__ void k_noalloc_mat(LayerMat lm, double* __restrict__ mat)
{
    for (int t = threadIdx.x; t < lm.n; t += blockDim.x) mat[t] = lm.v[t];
}

// D (input tet order, [n_tets][4][21]) and h into the storage layout of one
// member slot: elements of the storage order in blocks of 64
__global__ void k_noalloc_D(int ne, const int* __restrict__ order, const double* __restrict__ Din,
                            const double* __restrict__ hin, double* __restrict__ D, double* __restrict__ h)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= (long)ne * 84) return;
    const int pos = (int)(t / 84), q = (int)(t % 84);
    const long e0 = order[pos];
    D[((long)(pos / 64) * 84 + q) * 64 + pos % 64] = Din[e0 * 84 + q];
    if (q == 0) h[pos] = hin ? hin[e0] : 0.0;
}

// nodal vector, input node order -> storage order (forward) or back
__global__ void k_noalloc_perm(long n3, const int* __restrict__ node_new, const double* __restrict__ src,
                               double* __restrict__ dst, int forward)
{
    const long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (t >= n3) return;
    const long i = t / 3, c = t % 3;
    const long s = 3L * node_new[i] + c;
    if (forward) dst[s] = src[t];
    else dst[t] = src[s];
}

void rayleigh_coefficients(double f_lo, double f_hi, double* a, double* b);

}  // namespace nlth

using namespace nlth;

struct nlth_ctx : Ctx {};
struct nlth_mesh : Mesh {};

static size_t round256(size_t n) { return (n + 255) / 256 * 256; }

extern "C" int nlth_apply_operator_noalloc(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob,
                                           int32_t which, const double* D_ip, const double* h, const double* x,
                                           double* y)
{
    Ctx* c = ctx;
    try {
        if (!ctx || !mesh || !prob || !D_ip || !x || !y) throw Error{NLTH_EINVAL, "NULL argument"};
        if (ctx->host_only) throw Error{NLTH_EDEVICE, "host-only context"};
        if (mesh->ctx != ctx) throw Error{NLTH_EINVAL, "mesh belongs to another context"};
        if (which < NLTH_OP_A || which > NLTH_OP_M) throw Error{NLTH_EINVAL, "which must be NLTH_OP_A/K/M"};
        const int nl = prob->n_layers;
        if (nl <= 0 || nl > kNoAllocMaxLayers)
            throw Error{NLTH_EINVAL, "problem: n_layers must be in 1..32 for the allocation-free apply"};
        if (nl <= mesh->max_layer) throw Error{NLTH_EINVAL, "problem: mesh uses a layer id >= n_layers"};
        if (!prob->rho || !prob->vs || !prob->nu || !prob->gamma_ref || !prob->h_max)
            throw Error{NLTH_EINVAL, "problem: a required array is NULL"};
        if (!(prob->dt > 0)) throw Error{NLTH_EINVAL, "problem: dt must be positive"};
        if (prob->damping_mode < NLTH_DAMPING_LAW || prob->damping_mode > NLTH_DAMPING_NONE)
            throw Error{NLTH_EINVAL, "problem: unknown damping mode"};
        if (prob->damping_mode != NLTH_DAMPING_NONE && !(prob->f_lo > 0 && prob->f_hi > prob->f_lo))
            throw Error{NLTH_EINVAL, "problem: Rayleigh band needs 0 < f_lo < f_hi"};
        const int ne = mesh->ne, nn = mesh->nn;
        const int ne_pad = (ne + 63) / 64 * 64;
        const long n3 = 3L * nn;
        // scratch regions
        const size_t o_mat = 0;
        const size_t o_D = o_mat + round256((size_t)nl * MAT_N * 8);
        const size_t o_h = o_D + round256((size_t)ne_pad * 84 * 8);
        const size_t o_x = o_h + round256((size_t)ne_pad * 8);
        const size_t o_y = o_x + round256((size_t)n3 * 8);
        const size_t o_f = o_y + round256((size_t)n3 * 8);
        const size_t need = o_f + round256((size_t)ne_pad * 30 * 8);
        if (need > kScratchBytes) {
            char buf[200];
            snprintf(buf, sizeof buf,
                     "mesh of %d tets and %d nodes needs %.1f MiB of scratch; the allocation-free apply holds "
                     "at most %.0f MiB (about 67,000 tets)",
                     ne, nn, need / 1048576.0, kScratchBytes / 1048576.0);
            throw Error{NLTH_EINVAL, buf};
        }
        LayerMat lm{};
        lm.n = nl * MAT_N;
        for (int l = 0; l < nl; ++l) {
            const double rho = prob->rho[l], vs = prob->vs[l], nu = prob->nu[l], hm = prob->h_max[l];
            if (!(rho > 0 && vs > 0 && nu > -1.0 && nu < 0.5))
                throw Error{NLTH_EINVAL, "problem: layer needs rho > 0, vs > 0, -1 < nu < 0.5"};
            const double G0 = rho * vs * vs, lam = 2.0 * G0 * nu / (1.0 - 2.0 * nu);
            double* col = lm.v + (size_t)l * MAT_N;
            col[MAT_RHO] = rho;
            col[MAT_G0] = G0;
            col[MAT_KB] = lam + 2.0 * G0 / 3.0;
            col[MAT_VS] = vs;
            col[MAT_VP] = sqrt((lam + 2.0 * G0) / rho);
            col[MAT_GREF] = prob->gamma_ref[l];
            col[MAT_HMAX] = hm;
            col[MAT_BETA] = 2.0 * M_PI * hm / (2.0 - M_PI * hm);
        }
        StepConst sc{};
        sc.dt = prob->dt;
        sc.damping_mode = prob->damping_mode;
        sc.h0 = prob->h0;
        if (prob->damping_mode == NLTH_DAMPING_NONE) sc.ahat = sc.bhat = 0.0;
        else rayleigh_coefficients(prob->f_lo, prob->f_hi, &sc.ahat, &sc.bhat);

        std::lock_guard<std::mutex> g(ctx->mu);
        NLTH_HIP(hipSetDevice(ctx->device));
        char* base = scratch_of(ctx->device);
        if (!base) throw Error{NLTH_EDEVICE, "scratch address not set up on this device"};
        double* mat = (double*)(base + o_mat);
        double* Ds = (double*)(base + o_D);
        double* hs = (double*)(base + o_h);
        double* xs = (double*)(base + o_x);
        double* ys = (double*)(base + o_y);
        double* f = (double*)(base + o_f);
        hipStream_t s = ctx->stream;
        const DevMesh dm = mesh->dev();
        hipLaunchKernelGGL(k_noalloc_mat, dim3(1), dim3(256), 0, s, lm, mat);
        const long nD = (long)ne * 84;
        hipLaunchKernelGGL(k_noalloc_D, dim3((unsigned)((nD + 255) / 256)), dim3(256), 0, s, ne,
                           mesh->order_d.as<int>(), D_ip, h, Ds, hs);
        hipLaunchKernelGGL(k_noalloc_perm, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3,
                           mesh->node_new_d.as<int>(), x, xs, 1);
        set_ebe_block(256);
        launch_ebe<double>(s, (OpMode)which, dm, 1, 1, 0, ne, Ds, hs, mat, nl, sc, xs, nullptr, f, nullptr, true);
        launch_gather<double>(s, dm, 1, 1, f, nullptr, 0.0, ys, nullptr, xs, nullptr, nullptr, false);
        if (which == NLTH_OP_A)
            launch_dashpot<double>(s, dm, 1, 1, mat, nl, 2.0 / prob->dt, xs, ys, nullptr, nullptr);
        hipLaunchKernelGGL(k_noalloc_perm, dim3((unsigned)((n3 + 255) / 256)), dim3(256), 0, s, n3,
                           mesh->node_new_d.as<int>(), ys, y, 0);
        NLTH_HIP(hipGetLastError());
        return NLTH_OK;
    } catch (const Error& e) {
        set_error(c, e);
        return e.code;
    }
}
