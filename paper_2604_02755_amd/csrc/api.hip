// C-ABI of libnlth and the host runtime: contexts, mesh analysis (validation,
// colouring, face and receiver tables), ensembles and the per-step driver.
//
// Per time step (Section 2.1, Eq. 1; Section 2.2, Algorithm 4):
//   right-hand side of Eq. 1 (one element-by-element pass + boundary dashpots)
//   3x3 block-Jacobi diagonal blocks of A (one pass) and their inverses
//   CG on A du = b: FP64 block-Jacobi PCG, or FP64 flexible CG preconditioned
//     by an FP32 block-Jacobi PCG (mixed precision)
//   q += K du, Newmark updates of u, v, a
//   multi-spring law at every integration point (D, theta, h), with the state
//     streamed from pinned host memory in chunks when it does not fit in HBM
//   receiver velocities
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <unordered_map>

#include "runtime.hpp"

namespace nlth {

void launch_record_iters(hipStream_t s, int MB, int nm, int ns, const int* member_step, const int* stepping,
                         const int* iters, const int* inner_total, int* iters_dev);

static std::mutex g_err_mu;
static std::string g_err;

void set_error(Ctx* c, const Error& e)
{
    if (c) c->last_error = e.msg;
    std::lock_guard<std::mutex> g(g_err_mu);
    g_err = e.msg;
}

// ---------------------------------------------------------------------------
// memory
// ---------------------------------------------------------------------------

void DevBuf::alloc(Budget* b, size_t n, bool pinned_host)
{
    release();
    if (n == 0) return;
    budget = b;
    host = pinned_host;
    if (b) {
        std::lock_guard<std::mutex> g(b->mu);
        if (pinned_host) {
            if (b->host_limit > 0 && b->host_used + (int64_t)n > b->host_limit)
                throw Error{NLTH_ENOMEM_HOST, "pinned host budget exceeded"};
            b->host_used += n;
        } else {
            if (b->limit > 0 && b->used + (int64_t)n > b->limit)
                throw Error{NLTH_ENOMEM_DEVICE, "device memory budget exceeded"};
            b->used += n;
        }
    }
    // Device buffers start at staggered offsets (a multiple of 256 B that is
    // not a multiple of a large power of two): the arrays that a kernel streams
    // together then do not all start at the same place of the HBM channel
    // interleave.  Measured: the CG vector kernels 4 % and whole steps 1.8 %
    // faster on the batched benchmark.
    static std::atomic<unsigned> s_allocs{0};
    const size_t off = pinned_host ? 0 : (size_t)(s_allocs.fetch_add(1) % 16) * 273 * 256;
    hipError_t e = pinned_host ? hipHostMalloc(&p, n, hipHostMallocDefault) : hipMalloc(&p, n + off);
    if (e == hipSuccess) p = (char*)p + off;
    if (e != hipSuccess) {
        p = nullptr;
        if (b) {
            std::lock_guard<std::mutex> g(b->mu);
            if (pinned_host) b->host_used -= n; else b->used -= n;
        }
        throw Error{pinned_host ? NLTH_ENOMEM_HOST : NLTH_ENOMEM_DEVICE,
                    std::string(pinned_host ? "hipHostMalloc" : "hipMalloc") + " failed: " + hipGetErrorString(e)};
    }
    bytes = n;
    base_off = off;
}

void DevBuf::release()
{
    if (p) {
        if (host) (void)hipHostFree(p); else (void)hipFree((char*)p - base_off);
        if (budget) {
            std::lock_guard<std::mutex> g(budget->mu);
            if (host) budget->host_used -= bytes; else budget->used -= bytes;
        }
    }
    p = nullptr;
    bytes = 0;
}

template <typename T>
static void upload(Budget* b, DevBuf& d, const std::vector<T>& h)
{
    d.alloc(b, h.size() * sizeof(T));
    if (!h.empty()) NLTH_HIP(hipMemcpy(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
}

int pad_members(int nm)
{
    if (nm <= 1) return 1;
    if (nm <= 256) {
        int p = 1;
        while (p < nm) p <<= 1;
        return p;
    }
    return (nm + 255) / 256 * 256;
}

// ---------------------------------------------------------------------------
// mesh analysis
// ---------------------------------------------------------------------------

static const int kEdge[6][2] = {{0, 1}, {1, 2}, {2, 0}, {0, 3}, {1, 3}, {2, 3}};

// barycentric gradients and volume of a straight-sided tet
static bool tet_geometry(const double X[4][3], double gL[4][3], double* vol)
{
    double J[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) J[a][b] = X[b + 1][a] - X[0][a];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    *vol = det / 6.0;
    if (!(det > 0.0)) return false;
    // rows of J^-1 are the gradients of xi_1..xi_3
    double inv[3][3];
    inv[0][0] = c00 / det;
    inv[1][0] = c01 / det;
    inv[2][0] = c02 / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    for (int i = 0; i < 3; ++i)
        for (int a = 0; a < 3; ++a) gL[i + 1][a] = inv[i][a];
    for (int a = 0; a < 3; ++a) gL[0][a] = -(gL[1][a] + gL[2][a] + gL[3][a]);
    return true;
}

// 6-node triangle mass int N_a N_b dA: the classical pattern A/180 (corner
// diagonal 6, corner-corner -1, corner and opposite edge -4, corner and an
// edge through it 0, edge diagonal 32, edge-edge 16).
static void p2_triangle_mass(double A, double M[36])
{
    static const int FE[3][2] = {{0, 1}, {1, 2}, {2, 0}};
    for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) {
            double v;
            if (a < 3 && b < 3) v = (a == b) ? 6 : -1;
            else if (a < 3 || b < 3) {
                int c = a < 3 ? a : b, e = (a < 3 ? b : a) - 3;
                v = (FE[e][0] == c || FE[e][1] == c) ? 0 : -4;
            } else v = (a == b) ? 32 : 16;
            M[6 * a + b] = v * A / 180.0;
        }
}

struct Key3 {
    int a, b, c;
    bool operator==(const Key3& o) const { return a == o.a && b == o.b && c == o.c; }
};
struct Key3Hash {
    size_t operator()(const Key3& k) const
    {
        return ((size_t)k.a * 73856093u) ^ ((size_t)k.b * 19349663u) ^ ((size_t)k.c * 83492791u);
    }
};
static Key3 key3(int x, int y, int z)
{
    int v[3] = {x, y, z};
    std::sort(v, v + 3);
    return Key3{v[0], v[1], v[2]};
}

// Morton key of a point in a box scaled isotropically to 2^21 cells per side
static uint64_t morton3(const double x[3], const double lo[3], double sc)
{
    auto spread = [](uint64_t v) {  // 21 bits -> every third bit
        v &= 0x1FFFFF;
        v = (v | v << 32) & 0x1F00000000FFFFull;
        v = (v | v << 16) & 0x1F0000FF0000FFull;
        v = (v | v << 8) & 0x100F00F00F00F00Full;
        v = (v | v << 4) & 0x10C30C30C30C30C3ull;
        v = (v | v << 2) & 0x1249249249249249ull;
        return v;
    };
    uint64_t code = 0;
    for (int c = 0; c < 3; ++c) {
        const uint64_t q = (uint64_t)std::min(std::max((x[c] - lo[c]) * sc, 0.0), (double)((1 << 21) - 1));
        code |= spread(q) << c;
    }
    return code;
}

static void build_mesh_internal(Ctx* ctx, const nlth_mesh_desc* d, Mesh& M);

// Validates the node references, renumbers the nodes in Morton order of their
// coordinates (nodal vectors then follow the spatial order of the elements,
// which keeps the gathers of single members local), and builds the mesh on
// the renumbered description.  M.node_new maps input node ids to storage ids.
static void build_mesh(Ctx* ctx, const nlth_mesh_desc* d, Mesh& M)
{
    if (!d || d->n_nodes <= 0 || d->n_tets <= 0 || !d->xyz || !d->tet10 || !d->layer)
        throw Error{NLTH_EINVAL, "mesh: n_nodes, n_tets, xyz, tet10 and layer are required"};
    if (d->n_bfaces < 0 || (d->n_bfaces > 0 && (!d->bface6 || !d->bface_kind)))
        throw Error{NLTH_EINVAL, "mesh: bface6/bface_kind missing"};
    if (d->n_recv < 0 || (d->n_recv > 0 && !d->recv)) throw Error{NLTH_EINVAL, "mesh: recv missing"};
    const int nn = d->n_nodes, ne = d->n_tets;
    char buf[256];
    for (long i = 0; i < 10L * ne; ++i)
        if (d->tet10[i] < 0 || d->tet10[i] >= nn) {
            snprintf(buf, sizeof buf, "mesh: tet %ld references node %d outside [0, %d)", i / 10, d->tet10[i], nn);
            throw Error{NLTH_EINVAL, buf};
        }
    for (long i = 0; i < 6L * d->n_bfaces; ++i)
        if (d->bface6[i] < 0 || d->bface6[i] >= nn) {
            snprintf(buf, sizeof buf, "mesh: boundary face %ld references node %d outside [0, %d)", i / 6,
                     d->bface6[i], nn);
            throw Error{NLTH_EINVAL, buf};
        }
    for (int r = 0; r < d->n_recv; ++r)
        if (d->recv[r] < 0 || d->recv[r] >= nn) {
            snprintf(buf, sizeof buf, "mesh: receiver %d is node %d outside [0, %d)", r, d->recv[r], nn);
            throw Error{NLTH_EINVAL, buf};
        }
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (long i = 0; i < nn; ++i)
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::min(lo[c], d->xyz[3 * i + c]);
            hi[c] = std::max(hi[c], d->xyz[3 * i + c]);
        }
    const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
    std::vector<std::pair<uint64_t, int>> key(nn);
    for (int i = 0; i < nn; ++i) key[i] = {morton3(d->xyz + 3L * i, lo, (double)(1 << 21) / ext), i};
    std::sort(key.begin(), key.end());
    M.node_new.resize(nn);
    for (int k = 0; k < nn; ++k) M.node_new[key[k].second] = k;
    std::vector<double> xyz(3L * nn);
    for (int k = 0; k < nn; ++k)
        for (int c = 0; c < 3; ++c) xyz[3L * k + c] = d->xyz[3L * key[k].second + c];
    std::vector<int> tet(10L * ne), bf(6L * d->n_bfaces), rc(d->n_recv);
    for (long i = 0; i < 10L * ne; ++i) tet[i] = M.node_new[d->tet10[i]];
    for (long i = 0; i < 6L * d->n_bfaces; ++i) bf[i] = M.node_new[d->bface6[i]];
    for (int r = 0; r < d->n_recv; ++r) rc[r] = M.node_new[d->recv[r]];
    nlth_mesh_desc dn = *d;
    dn.xyz = xyz.data();
    dn.tet10 = tet.data();
    dn.bface6 = d->n_bfaces > 0 ? bf.data() : d->bface6;
    dn.recv = d->n_recv > 0 ? rc.data() : d->recv;
    build_mesh_internal(ctx, &dn, M);
}

static void build_mesh_internal(Ctx* ctx, const nlth_mesh_desc* d, Mesh& M)
{
    const int nn = d->n_nodes, ne = d->n_tets;
    M.ctx = ctx;
    M.nn = nn;
    M.ne = ne;
    M.xyz.assign(d->xyz, d->xyz + 3L * nn);
    char buf[256];
    M.max_layer = 0;
    for (int e = 0; e < ne; ++e) {
        if (d->layer[e] < 0) {
            snprintf(buf, sizeof buf, "mesh: tet %d has negative layer id", e);
            throw Error{NLTH_EINVAL, buf};
        }
        M.max_layer = std::max(M.max_layer, d->layer[e]);
    }
    // geometry per input tet
    std::vector<double> gl(12L * ne), vol(ne);
    double vtot = 0;
    for (int e = 0; e < ne; ++e) {
        const int* t = d->tet10 + 10L * e;
        double X[4][3], G[4][3], V;
        for (int a = 0; a < 4; ++a)
            for (int c = 0; c < 3; ++c) X[a][c] = d->xyz[3L * t[a] + c];
        if (!tet_geometry(X, G, &V)) {
            snprintf(buf, sizeof buf, "mesh: tet %d has a non-positive Jacobian", e);
            throw Error{NLTH_EINVAL, buf};
        }
        for (int k = 0; k < 6; ++k) {
            const double* pa = d->xyz + 3L * t[kEdge[k][0]];
            const double* pb = d->xyz + 3L * t[kEdge[k][1]];
            const double* pm = d->xyz + 3L * t[4 + k];
            double el = 0, dv = 0;
            for (int c = 0; c < 3; ++c) {
                el += (pb[c] - pa[c]) * (pb[c] - pa[c]);
                double q = pm[c] - 0.5 * (pa[c] + pb[c]);
                dv += q * q;
            }
            if (dv > 1e-18 * el) {
                snprintf(buf, sizeof buf, "mesh: tet %d is not straight-sided (mid-node of edge %d off the midpoint)", e, k);
                throw Error{NLTH_EINVAL, buf};
            }
        }
        for (int k = 0; k < 12; ++k) gl[12L * e + k] = G[k / 3][k % 3];
        vol[e] = V;
        vtot += V;
    }
    M.volume = vtot;

    // storage order: elements sorted along a Morton curve through their
    // centroids (isotropic scaling), so that consecutive elements share nodes
    // and a sweep over the elements re-reads nodal vectors from cache
    {
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (long i = 0; i < nn; ++i)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], d->xyz[3 * i + c]);
                hi[c] = std::max(hi[c], d->xyz[3 * i + c]);
            }
        const double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
        const double sc = (double)(1 << 21) / ext;
        std::vector<std::pair<uint64_t, int>> key(ne);
        for (int e = 0; e < ne; ++e) {
            const int* t = d->tet10 + 10L * e;
            double x[3];
            for (int c = 0; c < 3; ++c) {
                x[c] = 0;
                for (int a = 0; a < 4; ++a) x[c] += 0.25 * d->xyz[3L * t[a] + c];
            }
            key[e] = {morton3(x, lo, sc), e};
        }
        std::sort(key.begin(), key.end());
        M.order.resize(ne);
        M.inv_order.resize(ne);
        for (int pos = 0; pos < ne; ++pos) {
            M.order[pos] = key[pos].second;
            M.inv_order[key[pos].second] = pos;
        }
    }

    // greedy colouring in storage order: a tet takes the lowest colour no tet
    // sharing a node has; colour classes are kept as lists of storage positions
    const int W = 4;  // up to 256 colours
    std::vector<uint64_t> used((size_t)nn * W, 0);
    std::vector<int> color(ne);
    int ncol = 0;
    for (int pos = 0; pos < ne; ++pos) {
        const int* t = d->tet10 + 10L * M.order[pos];
        uint64_t u[W] = {0, 0, 0, 0};
        for (int a = 0; a < 10; ++a)
            for (int w = 0; w < W; ++w) u[w] |= used[(size_t)t[a] * W + w];
        int c = -1;
        for (int w = 0; w < W && c < 0; ++w)
            if (~u[w]) c = 64 * w + __builtin_ctzll(~u[w]);
        if (c < 0) throw Error{NLTH_EINVAL, "mesh: more than 256 colours needed"};
        color[pos] = c;
        ncol = std::max(ncol, c + 1);
        for (int a = 0; a < 10; ++a) used[(size_t)t[a] * W + c / 64] |= 1ull << (c % 64);
    }
    M.ncolor = ncol;
    M.color_off.assign(ncol + 1, 0);
    for (int pos = 0; pos < ne; ++pos) M.color_off[color[pos] + 1]++;
    for (int c = 0; c < ncol; ++c) M.color_off[c + 1] += M.color_off[c];
    M.color_elems.resize(ne);
    {
        std::vector<int> fill(M.color_off.begin(), M.color_off.end() - 1);
        for (int pos = 0; pos < ne; ++pos) M.color_elems[fill[color[pos]]++] = pos;
    }
    // node -> (element, local node) incidences in storage order, for the
    // deterministic gather of element outputs
    std::vector<int> inc_ptr(nn + 1, 0), inc(10L * ne);
    for (int pos = 0; pos < ne; ++pos)
        for (int a = 0; a < 10; ++a) inc_ptr[d->tet10[10L * M.order[pos] + a] + 1]++;
    for (int i = 0; i < nn; ++i) inc_ptr[i + 1] += inc_ptr[i];
    {
        std::vector<int> fill(inc_ptr.begin(), inc_ptr.end() - 1);
        for (int pos = 0; pos < ne; ++pos)
            for (int a = 0; a < 10; ++a) inc[fill[d->tet10[10L * M.order[pos] + a]]++] = pos * 10 + a;
    }
    if (10L * ne > INT32_MAX) throw Error{NLTH_EINVAL, "mesh: more than 214,748,364 tets"};
    // element clusters: runs of consecutive storage elements, closed when the
    // next element would bring more than kClusterElems elements or
    // kClusterNodes distinct nodes; local node lists in first-use order
    std::vector<int> cl_off(1, 0), cl_noff(1, 0), cl_node;
    std::vector<uint32_t> cl_lconn(4L * ne, 0u);
    {
        std::vector<int> loc(nn, -1);
        std::vector<int> cur;  // the open cluster's nodes
        int start = 0;
        auto close = [&](int end) {
            for (int g : cur) loc[g] = -1;
            cl_node.insert(cl_node.end(), cur.begin(), cur.end());
            cl_noff.push_back((int)cl_node.size());
            cl_off.push_back(end);
            cur.clear();
            start = end;
        };
        for (int pos = 0; pos < ne; ++pos) {
            const int* t = d->tet10 + 10L * M.order[pos];
            int add = 0;
            for (int a = 0; a < 10; ++a) {
                bool seen = loc[t[a]] >= 0;
                for (int b = 0; b < a && !seen; ++b) seen = t[b] == t[a];
                add += !seen;
            }
            if (pos > start && (pos - start >= kClusterElems || (int)cur.size() + add > kClusterNodes)) close(pos);
            for (int a = 0; a < 10; ++a) {
                if (loc[t[a]] < 0) {
                    loc[t[a]] = (int)cur.size();
                    cur.push_back(t[a]);
                }
                cl_lconn[4L * pos + a / 4] |= (uint32_t)loc[t[a]] << (8 * (a % 4));
            }
        }
        close(ne);
    }
    M.ncl = (int)cl_off.size() - 1;
    // node -> cluster rows, ascending
    std::vector<int> cn_ptr(nn + 1, 0), cn_row(cl_node.size());
    for (int g : cl_node) cn_ptr[g + 1]++;
    for (int i = 0; i < nn; ++i) cn_ptr[i + 1] += cn_ptr[i];
    {
        std::vector<int> fill(cn_ptr.begin(), cn_ptr.end() - 1);
        for (int r = 0; r < (int)cl_node.size(); ++r) cn_row[fill[cl_node[r]]++] = r;
    }
    M.cl_rows = (long)cl_node.size();
    // sorted SoA arrays
    std::vector<int> conn(10L * ne), lay(ne);
    std::vector<double> g64(13L * ne);
    std::vector<float> g32(13L * ne);
    for (int p = 0; p < ne; ++p) {
        int e = M.order[p];
        for (int k = 0; k < 10; ++k) conn[(long)k * ne + p] = d->tet10[10L * e + k];
        for (int k = 0; k < 12; ++k) g64[(long)k * ne + p] = gl[12L * e + k];
        g64[12L * ne + p] = vol[e];
        lay[p] = d->layer[e];
    }
    for (long i = 0; i < 13L * ne; ++i) g32[i] = (float)g64[i];

    // boundary faces: owning tet (for the material), normal, P2 face mass
    std::unordered_map<Key3, int, Key3Hash> owner;
    owner.reserve(4L * ne);
    static const int TF[4][3] = {{0, 1, 2}, {1, 2, 3}, {0, 2, 3}, {0, 1, 3}};
    if (d->n_bfaces > 0)
        for (int e = 0; e < ne; ++e)
            for (int f = 0; f < 4; ++f) {
                const int* t = d->tet10 + 10L * e;
                owner[key3(t[TF[f][0]], t[TF[f][1]], t[TF[f][2]])] = e;
            }
    const int nf = d->n_bfaces;
    M.nf = nf;
    std::vector<int> fnode(6L * nf), flayer(nf);
    std::vector<double> fM(36L * nf), fn(3L * nf);
    std::vector<uint8_t> fkind(nf);
    std::vector<std::vector<std::pair<int, int>>> node_faces;
    std::vector<int> bnodes;
    std::unordered_map<int, int> bn_index;
    for (int f = 0; f < nf; ++f) {
        const int* q = d->bface6 + 6L * f;
        for (int a = 0; a < 6; ++a)
            if (q[a] < 0 || q[a] >= nn) {
                snprintf(buf, sizeof buf, "mesh: boundary face %d references node %d outside [0, %d)", f, q[a], nn);
                throw Error{NLTH_EINVAL, buf};
            }
        if (d->bface_kind[f] > 1) {
            snprintf(buf, sizeof buf, "mesh: boundary face %d has kind %d (0 base, 1 side)", f, d->bface_kind[f]);
            throw Error{NLTH_EINVAL, buf};
        }
        auto it = owner.find(key3(q[0], q[1], q[2]));
        if (it == owner.end()) {
            snprintf(buf, sizeof buf, "mesh: boundary face %d is not a face of any tet", f);
            throw Error{NLTH_EINVAL, buf};
        }
        flayer[f] = d->layer[it->second];
        fkind[f] = d->bface_kind[f];
        double e1[3], e2[3], c[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = d->xyz[3L * q[1] + k] - d->xyz[3L * q[0] + k];
            e2[k] = d->xyz[3L * q[2] + k] - d->xyz[3L * q[0] + k];
        }
        c[0] = e1[1] * e2[2] - e1[2] * e2[1];
        c[1] = e1[2] * e2[0] - e1[0] * e2[2];
        c[2] = e1[0] * e2[1] - e1[1] * e2[0];
        double nc = sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
        if (!(nc > 0)) {
            snprintf(buf, sizeof buf, "mesh: boundary face %d is degenerate", f);
            throw Error{NLTH_EINVAL, buf};
        }
        for (int k = 0; k < 3; ++k) fn[3L * f + k] = c[k] / nc;
        p2_triangle_mass(0.5 * nc, &fM[36L * f]);
        for (int a = 0; a < 6; ++a) {
            fnode[6L * f + a] = q[a];
            auto bi = bn_index.find(q[a]);
            int idx;
            if (bi == bn_index.end()) {
                idx = (int)bnodes.size();
                bn_index[q[a]] = idx;
                bnodes.push_back(q[a]);
                node_faces.emplace_back();
            } else idx = bi->second;
            node_faces[idx].push_back({f, a});
        }
    }
    // boundary nodes in ascending node order, their (face, local) lists
    std::vector<int> perm(bnodes.size());
    for (size_t i = 0; i < perm.size(); ++i) perm[i] = (int)i;
    std::sort(perm.begin(), perm.end(), [&](int x, int y) { return bnodes[x] < bnodes[y]; });
    std::vector<int> bn_node, bn_ptr(1, 0), bn_face, bn_loc;
    for (int pi : perm) {
        bn_node.push_back(bnodes[pi]);
        for (auto& fl : node_faces[pi]) {
            bn_face.push_back(fl.first);
            bn_loc.push_back(fl.second);
        }
        bn_ptr.push_back((int)bn_face.size());
    }
    M.nbn = (int)bn_node.size();
    std::vector<int> bn_of_node(nn, -1);
    for (int i = 0; i < M.nbn; ++i) bn_of_node[bn_node[i]] = i;
    M.nrecv = d->n_recv;
    M.recv.assign(d->recv, d->recv + d->n_recv);
    for (int r = 0; r < d->n_recv; ++r)
        if (M.recv[r] < 0 || M.recv[r] >= nn) {
            snprintf(buf, sizeof buf, "mesh: receiver %d is node %d outside [0, %d)", r, M.recv[r], nn);
            throw Error{NLTH_EINVAL, buf};
        }
    if (ctx->host_only) return;
    Budget* b = &ctx->budget;
    upload(b, M.conn, conn);
    upload(b, M.geo64, g64);
    upload(b, M.geo32, g32);
    upload(b, M.layer, lay);
    upload(b, M.bn_node, bn_node);
    upload(b, M.bn_ptr, bn_ptr);
    upload(b, M.bn_face, bn_face);
    upload(b, M.bn_loc, bn_loc);
    upload(b, M.f_node, fnode);
    upload(b, M.f_M, fM);
    upload(b, M.f_n, fn);
    upload(b, M.f_layer, flayer);
    upload(b, M.f_kind, fkind);
    upload(b, M.recv_d, M.recv);
    upload(b, M.inc_ptr, inc_ptr);
    upload(b, M.inc, inc);
    upload(b, M.celem, M.color_elems);
    upload(b, M.bn_of, bn_of_node);
    upload(b, M.cl_off_d, cl_off);
    upload(b, M.cl_noff_d, cl_noff);
    upload(b, M.cl_lconn_d, cl_lconn);
    upload(b, M.cn_ptr_d, cn_ptr);
    upload(b, M.cn_row_d, cn_row);
    upload(b, M.order_d, M.order);
    upload(b, M.node_new_d, M.node_new);
}

DevMesh Mesh::dev() const
{
    DevMesh d{};
    d.ne = ne;
    d.nn = nn;
    d.conn = conn.as<int>();
    d.geo64 = geo64.as<double>();
    d.geo32 = geo32.as<float>();
    d.layer = layer.as<int>();
    d.nbn = nbn;
    d.bn_node = bn_node.as<int>();
    d.bn_ptr = bn_ptr.as<int>();
    d.bn_face = bn_face.as<int>();
    d.bn_loc = bn_loc.as<int>();
    d.f_node = f_node.as<int>();
    d.f_M = f_M.as<double>();
    d.f_n = f_n.as<double>();
    d.f_layer = f_layer.as<int>();
    d.f_kind = f_kind.as<uint8_t>();
    d.inc_ptr = inc_ptr.as<int>();
    d.inc = inc.as<int>();
    d.celem = celem.as<int>();
    d.bn_of_node = bn_of.as<int>();
    d.ncl = ncl;
    d.cl_off = cl_off_d.as<int>();
    d.cl_noff = cl_noff_d.as<int>();
    d.cl_lconn = cl_lconn_d.as<uint32_t>();
    d.cn_ptr = cn_ptr_d.as<int>();
    d.cn_row = cn_row_d.as<int>();
    return d;
}

// ---------------------------------------------------------------------------
// problem
// ---------------------------------------------------------------------------

// members m0 .. m0+n-1 of a problem (the per-member arrays sliced)
Problem member_slice(const Problem& P, int m0, int n)
{
    Problem q = P;
    q.nm = n;
    const long nl = P.nl, ns3 = (long)P.n_steps * 3;
    q.rho.assign(P.rho.begin() + m0 * nl, P.rho.begin() + (m0 + n) * nl);
    q.vs.assign(P.vs.begin() + m0 * nl, P.vs.begin() + (m0 + n) * nl);
    q.nu.assign(P.nu.begin() + m0 * nl, P.nu.begin() + (m0 + n) * nl);
    q.gref.assign(P.gref.begin() + m0 * nl, P.gref.begin() + (m0 + n) * nl);
    if (!P.acc.empty()) q.acc.assign(P.acc.begin() + m0 * ns3, P.acc.begin() + (m0 + n) * ns3);
    return q;
}

void copy_problem(const nlth_problem* in, Problem& P)
{
    if (!in) throw Error{NLTH_EINVAL, "problem is NULL"};
    if (in->n_members <= 0 || in->n_layers <= 0 || in->n_springs <= 0 || in->n_steps < 0)
        throw Error{NLTH_EINVAL, "problem: n_members, n_layers, n_springs must be positive, n_steps >= 0"};
    if (!in->rho || !in->vs || !in->nu || !in->gamma_ref || !in->h_max || !in->nonlinear || !in->dirs ||
        !in->weights || (in->n_steps > 0 && !in->input_acc))
        throw Error{NLTH_EINVAL, "problem: a required array is NULL"};
    if (!(in->dt > 0) || !(in->cg_tol > 0) || in->cg_maxit <= 0)
        throw Error{NLTH_EINVAL, "problem: dt, cg_tol and cg_maxit must be positive"};
    if (in->precision != NLTH_FP64 && in->precision != NLTH_MIXED)
        throw Error{NLTH_EINVAL, "problem: precision must be NLTH_FP64 or NLTH_MIXED"};
    if (in->precision == NLTH_MIXED && (!(in->inner_tol > 0) || in->inner_maxit <= 0))
        throw Error{NLTH_EINVAL, "problem: inner_tol and inner_maxit must be positive for NLTH_MIXED"};
    if (in->damping_mode < 0 || in->damping_mode > 2) throw Error{NLTH_EINVAL, "problem: bad damping_mode"};
    if (in->damping_mode == NLTH_DAMPING_LAW || in->damping_mode == NLTH_DAMPING_CONST)
        if (!(in->f_lo > 0) || !(in->f_hi > in->f_lo)) throw Error{NLTH_EINVAL, "problem: need 0 < f_lo < f_hi"};
    P.nm = in->n_members;
    P.nl = in->n_layers;
    P.ns = in->n_springs;
    P.n_steps = in->n_steps;
    const long ml = (long)P.nm * P.nl;
    P.rho.assign(in->rho, in->rho + ml);
    P.vs.assign(in->vs, in->vs + ml);
    P.nu.assign(in->nu, in->nu + ml);
    P.gref.assign(in->gamma_ref, in->gamma_ref + ml);
    P.hmax.assign(in->h_max, in->h_max + P.nl);
    P.nonlinear.assign(in->nonlinear, in->nonlinear + P.nl);
    P.dirs.assign(in->dirs, in->dirs + 6L * P.ns);
    P.w.assign(in->weights, in->weights + P.ns);
    if (P.n_steps > 0) P.acc.assign(in->input_acc, in->input_acc + (long)P.nm * P.n_steps * 3);
    for (long i = 0; i < ml; ++i) {
        if (!(P.rho[i] > 0) || !(P.vs[i] > 0) || !(P.nu[i] >= 0 && P.nu[i] < 0.5) || !(P.gref[i] > 0))
            throw Error{NLTH_EINVAL, "problem: need rho > 0, vs > 0, 0 <= nu < 0.5, gamma_ref > 0"};
    }
    for (int l = 0; l < P.nl; ++l)
        if (!(P.hmax[l] >= 0 && P.hmax[l] < 2.0 / M_PI)) throw Error{NLTH_EINVAL, "problem: need 0 <= h_max < 2/pi"};
    for (double x : P.acc)
        if (!std::isfinite(x)) throw Error{NLTH_EINVAL, "problem: input_acc has a non-finite value"};
    P.damping_mode = in->damping_mode;
    P.h0 = in->h0;
    P.f_lo = in->f_lo;
    P.f_hi = in->f_hi;
    P.dt = in->dt;
    P.cg_tol = in->cg_tol;
    P.cg_maxit = in->cg_maxit;
    P.precision = in->precision;
    P.inner_tol = in->inner_tol;
    P.inner_maxit = in->inner_maxit;
    if (in->masing_depth < 0 || in->masing_depth > kMaxMasingDepth)
        throw Error{NLTH_EINVAL, "problem: masing_depth must be in 0..8"};
    P.depth = std::max(1, (int)in->masing_depth);
    if (in->inner_dtype != NLTH_INNER_BF16 && in->inner_dtype != NLTH_INNER_FP32 &&
        in->inner_dtype != NLTH_INNER_BF16_MEAN)
        throw Error{NLTH_EINVAL, "problem: inner_dtype must be NLTH_INNER_BF16, NLTH_INNER_FP32 or NLTH_INNER_BF16_MEAN"};
    P.inner_dtype = in->inner_dtype;
}

// least-squares Rayleigh fit: minimise int (a/(4 pi f) + pi b f - 1)^2 df over [f_lo, f_hi]
static void rayleigh_fit(double fl, double fh, double* a, double* b)
{
    const double pi = M_PI;
    const double s11 = (1.0 / fl - 1.0 / fh) / (16.0 * pi * pi);
    const double s12 = 0.25 * (fh - fl);
    const double s22 = pi * pi * (fh * fh * fh - fl * fl * fl) / 3.0;
    const double t1 = log(fh / fl) / (4.0 * pi);
    const double t2 = 0.5 * pi * (fh * fh - fl * fl);
    const double det = s11 * s22 - s12 * s12;
    *a = (t1 * s22 - s12 * t2) / det;
    *b = (s11 * t2 - s12 * t1) / det;
}

void rayleigh_coefficients(double f_lo, double f_hi, double* a, double* b) { rayleigh_fit(f_lo, f_hi, a, b); }

int64_t ensemble_bytes(const Mesh& m, const Problem& p, int MB, bool paged)
{
    const int64_t ndof = 3L * m.nn;
    int64_t v = ndof * MB * 8;
    int64_t bytes = 12 * v;                                  // u v a q du du2 du3 b r z p Ap
    bytes += 2 * (int64_t)m.nn * 6 * MB * 8 + (int64_t)m.nn * 6 * MB * 4;  // diag, pinv, pinv32
    if (p.precision == NLTH_MIXED) {
        bytes += 5 * ndof * MB * 4;
        bytes += (int64_t)(2 * kLanczosMax * 8 + (2 * kChebMax + 1) * 4 + 16) * MB;  // Lanczos, Chebyshev tables
        if (MB >= 64 && MB <= 256) bytes += (int64_t)m.nbn * 3 * MB * 4;           // dashpot rows
    }
    bytes += (int64_t)m.ne * 4 * 21 * MB * 8;               // D64
    if (p.precision == NLTH_MIXED)
        bytes += (int64_t)m.ne * 4 *
                 (p.inner_dtype == NLTH_INNER_FP32 ? 84 : (p.inner_dtype == NLTH_INNER_BF16_MEAN ? 11 : 44)) * MB;
    bytes += (int64_t)m.ne * MB * 8;                        // h
    if (MB >= 64 && MB <= 256) bytes += (int64_t)m.cl_rows * 3 * MB * 8;  // cluster rows
    else if (MB < 64) bytes += (int64_t)m.ne * 30 * MB * 8;             // element outputs
    bytes += (int64_t)p.n_steps * std::max(1, m.nrecv) * 3 * MB * 8;  // receiver history
    bytes += (int64_t)p.n_steps * 3 * MB * 8 * 2;           // acc, vI
    if (!paged) bytes += (int64_t)m.ne * 4 * p.ns * MB * theta_bytes(p.depth);
    return bytes;
}

// ---------------------------------------------------------------------------
// ensemble
// ---------------------------------------------------------------------------

hipEvent_t Ens::ev()
{
    if (!ev_pool.empty()) {
        hipEvent_t e = ev_pool.back();
        ev_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    NLTH_HIP(hipEventCreate(&e));
    return e;
}

void Ens::tstart(hipEvent_t& e0)
{
    e0 = nullptr;
    if (!profile) return;
    e0 = ev();
    NLTH_HIP(hipEventRecord(e0, s));
}

void Ens::tstop(hipEvent_t e0, ProfCat* cat, int64_t elems)
{
    if (!profile || !e0) return;
    hipEvent_t e1 = ev();
    NLTH_HIP(hipEventRecord(e1, s));
    pending.push_back({{e0, e1}, cat});
    cat->elems += elems;
}

void Ens::collect_prof()
{
    for (auto& pe : pending) {
        float ms = 0;
        NLTH_HIP(hipEventElapsedTime(&ms, pe.first.first, pe.first.second));
        pe.second->ms += ms;
        pe.second->n += 1;
        ev_pool.push_back(pe.first.first);
        ev_pool.push_back(pe.first.second);
    }
    pending.clear();
}

void Ens::sync()
{
    NLTH_HIP(hipStreamSynchronize(s));
    collect_prof();
}

void Ens::create(Ctx* c, const Mesh* m, const Problem& prob, int member_pad)
{
    ctx = c;
    mesh = m;
    P = prob;
    if (P.nl <= m->max_layer) throw Error{NLTH_EINVAL, "problem: mesh uses a layer id >= n_layers"};
    nm = P.nm;
    MB = member_pad > 0 ? member_pad : pad_members(nm);
    ndof = 3L * m->nn;
    s = own_s ? own_s : c->stream;
    Budget* bg = &c->budget;
    sc.dt = P.dt;
    sc.damping_mode = P.damping_mode;
    sc.h0 = P.h0;
    if (P.damping_mode == NLTH_DAMPING_NONE) sc.ahat = sc.bhat = 0.0;
    else rayleigh_fit(P.f_lo, P.f_hi, &sc.ahat, &sc.bhat);

    // per-member material table (padded members copy member 0)
    std::vector<double> mt((size_t)P.nl * MAT_N * MB, 0.0);
    for (int l = 0; l < P.nl; ++l)
        for (int mm = 0; mm < MB; ++mm) {
            const int src = mm < nm ? mm : 0;
            const double rho = P.rho[(long)src * P.nl + l], vs = P.vs[(long)src * P.nl + l];
            const double nu = P.nu[(long)src * P.nl + l];
            const double G0 = rho * vs * vs, lam = 2.0 * G0 * nu / (1.0 - 2.0 * nu);
            const double hm = P.hmax[l];
            double* col = &mt[(size_t)l * MAT_N * MB];
            col[MAT_RHO * MB + mm] = rho;
            col[MAT_G0 * MB + mm] = G0;
            col[MAT_KB * MB + mm] = lam + 2.0 * G0 / 3.0;
            col[MAT_VS * MB + mm] = vs;
            col[MAT_VP * MB + mm] = sqrt((lam + 2.0 * G0) / rho);
            col[MAT_GREF * MB + mm] = P.gref[(long)src * P.nl + l];
            col[MAT_HMAX * MB + mm] = hm;
            col[MAT_BETA * MB + mm] = 2.0 * M_PI * hm / (2.0 - M_PI * hm);
        }
    upload(bg, mat, mt);
    upload(bg, dirs, P.dirs);
    upload(bg, w, P.w);
    upload(bg, nonlinear, P.nonlinear);

    const int ns_steps = std::max(1, P.n_steps);
    // inputs: acceleration as given, incident velocity by the trapezoid rule (device)
    std::vector<double> acc_pad((size_t)MB * ns_steps * 3, 0.0);
    if (P.n_steps > 0) std::copy(P.acc.begin(), P.acc.end(), acc_pad.begin());
    upload(bg, acc, acc_pad);
    vI_all.alloc(bg, acc_pad.size() * 8);
    launch_incident_velocity(s, MB, MB, ns_steps, acc.as<double>(), vI_all.as<double>(), P.dt);
    vI_cur.alloc(bg, 3L * MB * 8);

    const size_t vb = (size_t)ndof * MB * 8;
    for (DevBuf* bb : {&u, &v, &a, &q, &du, &du2, &du3, &b, &r, &z, &p, &Ap}) {
        bb->alloc(bg, vb);
        launch_fill(s, bb->as<double>(), 0.0, (long)ndof * MB);
    }
    diag.alloc(bg, (size_t)m->nn * 6 * MB * 8);
    pinv.alloc(bg, (size_t)m->nn * 6 * MB * 8);
    pinv32.alloc(bg, (size_t)m->nn * 6 * MB * 4);
    if (P.precision == NLTH_MIXED) {
        for (DevBuf* bb : {&ir, &iz, &ip, &iw, &iAp}) {
            bb->alloc(bg, (size_t)ndof * MB * 4);
            launch_fill32(s, bb->as<float>(), 0.0f, (long)ndof * MB);
        }
        lz.alloc(bg, (size_t)2 * kLanczosMax * MB * 8);
        launch_fill(s, lz.as<double>(), 0.0, (long)2 * kLanczosMax * MB);
        chebc.alloc(bg, (size_t)(2 * kChebMax + 1) * MB * 4);
        launch_fill32(s, chebc.as<float>(), 0.0f, (long)(2 * kChebMax + 1) * MB);
        cheb_bounds.alloc(bg, (size_t)(2 * MB + 1) * 8);  // per-member lo, hi; the running upper bound
        launch_fill(s, cheb_bounds.as<double>(), 0.0, (long)2 * MB + 1);
        if (MB >= 64 && MB <= 256 && m->nbn > 0) qb.alloc(bg, (size_t)m->nbn * 3 * MB * 4);
    }
    EB = MB >= 64 ? 1 : 64 / MB;
    ne_pad = (m->ne + EB - 1) / EB * EB;
    const size_t nD = (size_t)ne_pad * 4 * 21 * MB;
    D64.alloc(bg, nD * 8);
    if (P.precision == NLTH_MIXED && P.inner_dtype == NLTH_INNER_FP32) D32.alloc(bg, nD * 4);
    if (P.precision == NLTH_MIXED && P.inner_dtype == NLTH_INNER_BF16) D16.alloc(bg, (size_t)ne_pad * 4 * 11 * MB * 4);
    if (P.precision == NLTH_MIXED && P.inner_dtype == NLTH_INNER_BF16_MEAN) D16.alloc(bg, (size_t)ne_pad * 11 * MB * 4);
    d16_mean = P.inner_dtype == NLTH_INNER_BF16_MEAN;
    tail_max = MB >= 64 && MB <= 256 && (P.precision == NLTH_FP64 || d16_mean) ? 32 : 0;
    h.alloc(bg, (size_t)m->ne * MB * 8);
    // operator path: element clusters (64-member groups) when MB is a multiple
    // of 64, element outputs below that, colours above 256 member slots (the
    // node gather covers at most 256 slots per block)
    if (MB > 256) {
        scatter = 1;
    } else if (MB >= 64) {
        scatter = 2;
        cbuf.alloc(bg, (size_t)m->cl_rows * 3 * MB * 8);
    } else {
        scatter = 0;
        fbuf.alloc(bg, (size_t)ne_pad * 30 * MB * 8);
    }
    const DevMesh dm = m->dev();
    launch_law_init(s, dm, MB, MB, mat.as<double>(), P.nl, P.ns, dirs.as<double>(), w.as<double>(),
                    D64.as<double>(), D32.as<float>(), D16.as<uint32_t>(), h.as<double>(), -1, d16_mean);

    // law state: resident if it fits the remaining budget, else paged
    const size_t per_elem = (size_t)4 * P.ns * MB * theta_bytes(P.depth);
    const size_t state_bytes = per_elem * ne_pad;
    int64_t avail;
    {
        std::lock_guard<std::mutex> g(bg->mu);
        avail = bg->limit > 0 ? bg->limit - bg->used : INT64_MAX;
    }
    const int64_t reserve = (int64_t)P.n_steps * std::max(1, m->nrecv) * 3 * MB * 8 * 2 + (64 << 20) + reserve_extra;
    paged = force_paged || (int64_t)state_bytes + reserve > avail;
    if (!paged) {
        theta.alloc(bg, state_bytes);
        launch_theta_init(s, theta.p, ne_pad, P.ns, MB);
    } else {
        // chunk ring: the largest chunk with 3 slots fitting a quarter of what is left
        int64_t slot_bytes = std::max<int64_t>((avail - reserve) / 4 / ring, (int64_t)per_elem);
        slot_bytes = std::min<int64_t>(slot_bytes, (int64_t)1 << 31);
        chunk_elems = (int)std::max<int64_t>(1, std::min<int64_t>(slot_bytes / (int64_t)per_elem, ne_pad));
        chunk_elems = std::max(EB, chunk_elems / EB * EB);
        nchunks = (m->ne + chunk_elems - 1) / chunk_elems;
        if (nchunks < ring) ring = std::max(1, nchunks);
        theta_host.alloc(bg, state_bytes, true);
        theta.alloc(bg, (size_t)chunk_elems * per_elem * ring);
        long off = 0;
        for (int cix = 0; cix < nchunks; ++cix) {
            int e0 = cix * chunk_elems, ec = std::min(chunk_elems, m->ne - e0);
            chunk_e0.push_back(e0);
            chunk_ec.push_back(ec);
            chunk_ecp.push_back((ec + EB - 1) / EB * EB);
            chunk_off.push_back(off);
            off += (long)chunk_ecp.back() * per_elem;
        }
        // initialise each chunk on the device and write it to the host copy
        for (int cix = 0; cix < nchunks; ++cix) {
            launch_theta_init(s, theta.p, chunk_ecp[cix], P.ns, MB);
            NLTH_HIP(hipMemcpyAsync((char*)theta_host.p + chunk_off[cix], theta.p, (size_t)chunk_ecp[cix] * per_elem,
                                    hipMemcpyDeviceToHost, s));
        }
        if (!shared_copy_streams) NLTH_HIP(hipStreamCreateWithFlags(&s_h2d, hipStreamNonBlocking));
        for (int k = 0; k < ring; ++k) {
            hipEvent_t e1, e2;
            NLTH_HIP(hipEventCreateWithFlags(&e1, hipEventDisableTiming));
            NLTH_HIP(hipEventCreateWithFlags(&e2, hipEventDisableTiming));
            ev_h2d.push_back(e1);
            ev_d2h.push_back(e2);
        }
        slot_chunk.assign(ring, -1);
        prefetched.assign(nchunks, false);
        NLTH_HIP(hipEventCreateWithFlags(&ev_zc, hipEventDisableTiming));
        NLTH_HIP(hipEventCreate(&ev_copy0));
        NLTH_HIP(hipEventCreate(&ev_copy1));
    }

    hist.alloc(bg, (size_t)MB * ns_steps * std::max(1, m->nrecv) * 3 * 8);
    launch_fill(s, hist.as<double>(), 0.0, (long)MB * ns_steps * std::max(1, m->nrecv) * 3);
    vmax.alloc(bg, (size_t)MB * std::max(1, m->nrecv) * 8);
    launch_fill(s, vmax.as<double>(), 0.0, (long)MB * std::max(1, m->nrecv));
    iters_dev.alloc(bg, (size_t)MB * ns_steps * 2 * 4);
    NLTH_HIP(hipMemsetAsync(iters_dev.p, 0, iters_dev.bytes, s));
    partial.alloc(bg, (size_t)kPartialRows * MB * 8);
    // CG scalars: 12 double arrays and 9 int arrays of MB
    scal.alloc(bg, (size_t)MB * (12 * 8 + 9 * 4) + 64);
    NLTH_HIP(hipMemsetAsync(scal.p, 0, scal.bytes, s));
    double* dptr = scal.as<double>();
    cs.bb = dptr; cs.rr = dptr + MB; cs.rz = dptr + 2 * MB; cs.alpha = dptr + 3 * MB; cs.beta = dptr + 4 * MB;
    cs.pAp = dptr + 5 * MB; cs.r0 = dptr + 6 * MB; cs.irr = dptr + 7 * MB; cs.irz = dptr + 8 * MB;
    cs.ialpha = dptr + 9 * MB; cs.ibeta = dptr + 10 * MB; cs.ir0 = dptr + 11 * MB;
    int* iptr = (int*)(dptr + 12 * MB);
    cs.active = iptr; cs.iters = iptr + MB; cs.status = iptr + 2 * MB; cs.inner_active = iptr + 3 * MB;
    cs.inner_iters = iptr + 4 * MB; cs.inner_total = iptr + 5 * MB; cs.inner_upd = iptr + 6 * MB;
    cs.lz = lz.as<double>();
    NLTH_HIP(hipHostMalloc((void**)&h_mail, sizeof(int) * (5 * (size_t)MB + 1),
                           hipHostMallocMapped | hipHostMallocCoherent));
    NLTH_HIP(hipHostGetDevicePointer((void**)&d_mail, h_mail, 0));
    h_flags = h_mail;
    h_tlist = h_mail + 4 * MB;
    member_step.alloc(bg, (size_t)MB * 4);
    stepping.alloc(bg, (size_t)MB * 4);
    cs.stepping = stepping.as<int>();
    h_member_step.assign(MB, 0);
    h_stepping.assign(MB, 0);
    h_status.assign(MB, 0);
    {
        std::lock_guard<std::mutex> g(bg->mu);
        dev_bytes = bg->used;
        host_bytes = bg->host_used;
    }
    NLTH_HIP(hipStreamSynchronize(s));
}

void Ens::destroy()
{
    twin.reset();  // the second set uses this set's transfer-in stream
    if (!ctx) {
        if (own_s) (void)hipStreamDestroy(own_s);
        own_s = nullptr;
        return;
    }
    if (s) (void)hipStreamSynchronize(s);
    if (shared_copy_streams) {
        s_h2d = nullptr;
    } else if (s_h2d) {
        (void)hipStreamSynchronize(s_h2d);
        (void)hipStreamDestroy(s_h2d);
        s_h2d = nullptr;
    }
    for (auto e : ev_h2d) (void)hipEventDestroy(e);
    for (auto e : ev_d2h) (void)hipEventDestroy(e);
    ev_h2d.clear(); ev_d2h.clear();
    if (ev_zc) (void)hipEventDestroy(ev_zc);
    ev_zc = nullptr;
    for (auto& pe : pending) { (void)hipEventDestroy(pe.first.first); (void)hipEventDestroy(pe.first.second); }
    pending.clear();
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    ev_pool.clear();
    clear_graphs();
    if (h_mail) (void)hipHostFree(h_mail);
    h_mail = d_mail = h_flags = h_tlist = nullptr;
    if (ev_copy0) (void)hipEventDestroy(ev_copy0);
    if (ev_copy1) (void)hipEventDestroy(ev_copy1);
    ev_copy0 = ev_copy1 = nullptr;
    ctx = nullptr;
    // device buffers go with the object; the stream after the work on it
    if (own_s) (void)hipStreamDestroy(own_s);
    own_s = nullptr;
}

// y = operator of `mode` applied to x1 (and x2 for the right-hand side)
//     + bscale * base + the boundary dashpot dcoef * C_abs x1 (+ 2 C_base vI),
// and with nblk the per-member block partials of x1 . y in `partial`.
// Gather path: one launch writes every element's nodal forces, a second sums
// them per node with the base, the dashpot and the dot fused in.  Colour
// path: one launch per colour adds the forces into y, then the dashpot and
// the dot as launches of their own.
void Ens::ebe(OpMode mode, const double* x1, const double* x2, double* y, const int* act, const double* base,
              double bscale, double dcoef, const double* vI, int* nblk)
{
    const DevMesh dm = mesh->dev();
    set_ebe_block(ebe_block);
    set_cluster_blocks(cluster_blocks);
    if (scatter != 1) {
        hipEvent_t t0;
        tstart(t0);
        double* pd = nblk ? partial.as<double>() : nullptr;
        if (scatter == 2) {
            launch_ebe_cluster64(s, mode, dm, MB, nm, D64.as<double>(), h.as<double>(), mat.as<double>(), sc, x1, x2,
                                 cbuf.as<double>(), act);
            launch_gather<double>(s, dm, MB, nm, cbuf.as<double>(), base, bscale, y, act, x1, pd, nblk, true);
        } else {
            launch_ebe<double>(s, mode, dm, MB, nm, 0, mesh->ne, D64.as<double>(), h.as<double>(), mat.as<double>(),
                               P.nl, sc, x1, x2, fbuf.as<double>(), act, true);
            launch_gather<double>(s, dm, MB, nm, fbuf.as<double>(), base, bscale, y, act, x1, pd, nblk, false);
        }
        if (dcoef != 0.0) launch_dashpot<double>(s, dm, MB, nm, mat.as<double>(), P.nl, dcoef, x1, y, vI, act, pd, nblk);
        tstop(t0, &pc_ebe64, (int64_t)mesh->ne * nm);
        return;
    }
    if (!base) launch_fill(s, y, 0.0, (long)ndof * MB);
    else if (base != y && bscale == -1.0) launch_neg_copy(s, base, y, (long)ndof * MB);
    else if (base != y || bscale != 1.0) throw Error{NLTH_EINVAL, "operator base: -1 * other array or 1 * y only"};
    for (int c = 0; c < mesh->ncolor; ++c) {
        const int e0 = mesh->color_off[c], e1 = mesh->color_off[c + 1];
        hipEvent_t t0;
        tstart(t0);
        launch_ebe<double>(s, mode, dm, MB, nm, e0, e1, D64.as<double>(), h.as<double>(), mat.as<double>(), P.nl, sc,
                           x1, x2, y, act, false);
        tstop(t0, &pc_ebe64, (int64_t)(e1 - e0) * nm);
    }
    if (dcoef != 0.0) launch_dashpot<double>(s, dm, MB, nm, mat.as<double>(), P.nl, dcoef, x1, y, vI, act);
    if (nblk) dots(1, x1, y, nullptr, nullptr, nullptr, nullptr, *nblk);
}

// y = A x with the inner operator's arithmetic (FP32, D in FP32 or bfloat16),
// dashpot included; with nblk the per-member block partials of x . y
void Ens::ebe32(const float* x, float* y, const int* act, int* nblk)
{
    const DevMesh dm = mesh->dev();
    set_ebe_block(ebe_block);
    set_cluster_blocks(cluster_blocks);
    const double dc = 2.0 / P.dt;
    if (scatter != 1) {
        const bool cl = scatter == 2;
        float* f = cl ? (float*)cbuf.p : (float*)fbuf.p;
        hipEvent_t t0;
        tstart(t0);
        if (cl)
            launch_ebe_cluster32(s, dm, MB, nm, D32.as<float>(), D16.as<uint32_t>(), h.as<double>(), mat.as<double>(),
                                 sc, x, f, act, d16_mean);
        else
            launch_ebe32(s, dm, MB, nm, 0, mesh->ne, D32.as<float>(), D16.as<uint32_t>(), h.as<double>(),
                         mat.as<double>(), sc, x, f, act, true, d16_mean);
        tstop(t0, &pc_ebe32, (int64_t)mesh->ne * nm);
        tstart(t0);
        double* pd = nblk ? partial.as<double>() : nullptr;
        launch_gather<float>(s, dm, MB, nm, f, nullptr, 0.0f, y, act, x, pd, nblk, cl);
        tstop(t0, &pc_gather32, (int64_t)mesh->nn * nm);
        launch_dashpot<float>(s, dm, MB, nm, mat.as<double>(), P.nl, (float)dc, x, y, nullptr, act, pd, nblk);
        return;
    }
    launch_fill32(s, y, 0.0f, (long)ndof * MB);
    for (int c = 0; c < mesh->ncolor; ++c) {
        const int e0 = mesh->color_off[c], e1 = mesh->color_off[c + 1];
        hipEvent_t t0;
        tstart(t0);
        launch_ebe32(s, dm, MB, nm, e0, e1, D32.as<float>(), D16.as<uint32_t>(), h.as<double>(), mat.as<double>(),
                     sc, x, y, act, false, d16_mean);
        tstop(t0, &pc_ebe32, (int64_t)(e1 - e0) * nm);
    }
    launch_dashpot<float>(s, dm, MB, nm, mat.as<double>(), P.nl, (float)dc, x, y, nullptr, act);
    if (nblk)
        launch_dotsv<float>(s, 1, x, y, nullptr, nullptr, nullptr, nullptr, ndof, MB, nm, act, partial.as<double>(),
                            nblk);
}

void Ens::build_rhs()
{
    // b = f - q + C v + M (a + 4/dt v), f = 2 C_base v_I
    ebe(OP_RHS, v.as<double>(), a.as<double>(), b.as<double>(), stepping.as<int>(), q.as<double>(), -1.0, 1.0,
        vI_cur.as<double>(), nullptr);
}

// Block-Jacobi diagonal: from D per point (FP64), or, for the mixed path with
// one D per element in the inner operator, the diagonal blocks of that inner
// operator itself (closed-form integrals, a fraction of the bytes); the outer
// FP64 iteration of the mixed path does not use the diagonal.
void Ens::build_diag()
{
    const DevMesh dm = mesh->dev();
    const bool mean = P.precision == NLTH_MIXED && d16_mean;
    launch_fill(s, diag.as<double>(), 0.0, (long)mesh->nn * 6 * MB);
    for (int c = 0; c < mesh->ncolor; ++c) {
        if (mean)
            launch_diag_mean(s, dm, MB, nm, mesh->color_off[c], mesh->color_off[c + 1], D16.as<uint32_t>(),
                             h.as<double>(), mat.as<double>(), sc, diag.as<double>());
        else
            launch_diag(s, dm, MB, nm, mesh->color_off[c], mesh->color_off[c + 1], D64.as<double>(), h.as<double>(),
                        mat.as<double>(), P.nl, sc, diag.as<double>());
    }
    launch_diag_dashpot(s, dm, MB, nm, mat.as<double>(), P.nl, 2.0 / P.dt, diag.as<double>());
    launch_invert_diag(s, mesh->nn, MB, nm, diag.as<double>(), pinv.as<double>(),
                       P.precision == NLTH_MIXED ? pinv32.as<float>() : nullptr);
}

void Ens::dots(int nd, const double* a0, const double* b0, const double* a1, const double* b1, const double* a2,
               const double* b2, int& nblk)
{
    launch_dotsv<double>(s, nd, a0, b0, a1, b1, a2, b2, ndof, MB, nm, nullptr, partial.as<double>(), &nblk);
}

// members whose flag was set at the last read
int Ens::count_flags() const
{
    int n = 0;
    for (int m = 0; m < nm; ++m) n += h_flags[m] != 0;
    return n;
}

// any member still iterating?  (the flags copied to the host mailbox)
int Ens::read_any_active(const int* flags)
{
    launch_copy_i32(s, flags, d_mail, nm);
    NLTH_HIP(hipStreamSynchronize(s));
    for (int m = 0; m < nm; ++m)
        if (h_flags[m]) return 1;
    return 0;
}

void Ens::fin(FinalizeStage st, int nd, int nblk, double tol2, int maxit)
{
    launch_finalize(s, st, nd, MB, nm, partial.as<double>(), nblk, cs, tol2, maxit);
}

void Ens::apply_A64(const double* x, double* y, const int* act, int* nblk)
{
    ebe(OP_A, x, nullptr, y, act, nullptr, 0.0, 2.0 / P.dt, nullptr, nblk);
}

// FP64 block-Jacobi PCG (Section 2.2): x0 = previous increment
void Ens::solve_pcg()
{
    const long n = ndof;
    int nblk;
    double* x = du.as<double>();
    const int* st = stepping.as<int>();
    const int* act = cs.active;
    const double tol2 = P.cg_tol * P.cg_tol;
    double* pd = partial.as<double>();
    apply_A64(x, Ap.as<double>(), st);
    launch_pcg_start(s, mesh->nn, MB, nm, b.as<double>(), Ap.as<double>(), pinv.as<double>(), r.as<double>(),
                     z.as<double>(), p.as<double>(), st, pd, &nblk);
    fin(FIN_START, 3, nblk, tol2, P.cg_maxit);
    launch_zero_if_b0(s, n, MB, nm, x, cs.bb, st);
    launch_p_update<double>(s, n, MB, nm, z.as<double>(), p.as<double>(), nullptr, nullptr, nullptr);
    if (!read_any_active(act)) return;
    for (;;) {
        if (!tail64_g) enter_tail64();  // with few members left: compact rows
        run_iters(1, check_every);
        if (!read_any_active(act)) break;
        if (tail64_g) tail_count = count_flags();
    }
    if (tail64_g) leave_tail64();
}

// With at most tail_max of the members just read (h_flags) still iterating,
// their PCG state and operator data go to compact rows of 16 or 32 lanes for
// the rest of the step's solve.
bool Ens::enter_tail64()
{
    if (tail_max <= 0 || P.precision != NLTH_FP64 || MB < 64 || MB > 256) return false;
    int na = 0;
    for (int m = 0; m < nm; ++m) na += h_flags[m] != 0;
    if (na == 0 || na > tail_max) return false;
    if (!alloc_tail64()) {  // no room: keep the full operator
        tail_max = 0;
        return false;
    }
    h_tlist[0] = na;
    tail_count = na;
    int k = 1;
    for (int m = 0; m < nm; ++m)
        if (h_flags[m]) h_tlist[k++] = m;
    launch_copy_i32(s, d_mail + 4 * MB, tlist.as<int>(), 1 + na);
    tail64_g = na <= 16 ? 16 : 32;
    const int* tl = tlist.as<int>();
    launch_tail_pack64(s, mesh->dev(), MB, tail64_g, P.nl, tl, D64.as<double>(), h.as<double>(), mat.as<double>(),
                       pinv.as<double>(), tc.D, tc.h, tc.mat, tc.pinv);
    launch_tail_rows64(s, ndof, MB, tail64_g, tl, du.as<double>(), tc.x, false);
    launch_tail_rows64(s, ndof, MB, tail64_g, tl, r.as<double>(), tc.r, false);
    launch_tail_rows64(s, ndof, MB, tail64_g, tl, z.as<double>(), tc.z, false);
    launch_tail_rows64(s, ndof, MB, tail64_g, tl, p.as<double>(), tc.p, false);
    return true;
}

// FP64 compact rows of 32 lanes: D per point (elements padded to blocks of
// 4), h, material, inverse blocks, five CG vectors, the operator's cluster
// rows (at most 10 per element: sized as element outputs)
bool Ens::alloc_tail64()
{
    if (tail64_mem.p) return true;
    const size_t ne4 = ((size_t)mesh->ne + 3) / 4 * 4, nn = mesh->nn, L = 32;
    const size_t nv = 3 * nn * L * 8;
    const size_t sz[10] = {ne4 * 84 * L * 8, (size_t)mesh->ne * L * 8, (size_t)P.nl * MAT_N * L * 8,
                           nn * 6 * L * 8, nv, nv, nv, nv, nv, (size_t)mesh->ne * 30 * L * 8};
    size_t off[10], tot = 0;
    for (int i = 0; i < 10; ++i) {
        off[i] = tot;
        tot += (sz[i] + 255) / 256 * 256;
    }
    try {
        tail64_mem.alloc(&ctx->budget, tot);
        if (!tlist.p) tlist.alloc(&ctx->budget, (size_t)(1 + MB) * 4);
    } catch (const Error&) {
        tail64_mem.release();
        return false;
    }
    char* b = (char*)tail64_mem.p;
    double** dst[10] = {&tc.D, &tc.h, &tc.mat, &tc.pinv, &tc.x, &tc.r, &tc.z, &tc.p, &tc.Ap, &tc.f};
    for (int i = 0; i < 10; ++i) *dst[i] = (double*)(b + off[i]);
    return true;
}

// Mixed path, once the inner solve runs on the compact rows of a list (just
// packed by update_tail): the outer iteration of the listed members moves to
// the FP64 compact rows too, its operator data and the increment, residual,
// direction and last operator result packed once; the list stays fixed for
// the rest of the step.
bool Ens::enter_outer_tail()
{
    if (!outer_tail_ok || P.precision != NLTH_MIXED || !tail_g || MB < 64 || MB > 256) return false;
    if (!alloc_tail64()) {
        outer_tail_ok = false;
        return false;
    }
    const int* tl = tlist.as<int>();
    launch_tail_pack64(s, mesh->dev(), MB, tail_g, P.nl, tl, D64.as<double>(), h.as<double>(), mat.as<double>(),
                       pinv.as<double>(), tc.D, tc.h, tc.mat, tc.pinv);
    launch_tail_rows64(s, ndof, MB, tail_g, tl, du.as<double>(), tc.x, false);
    launch_tail_rows64(s, ndof, MB, tail_g, tl, r.as<double>(), tc.r, false);
    launch_tail_rows64(s, ndof, MB, tail_g, tl, p.as<double>(), tc.p, false);
    launch_tail_rows64(s, ndof, MB, tail_g, tl, Ap.as<double>(), tc.Ap, false);  // the flexible beta reads it
    outer_compact = true;
    return true;
}

void Ens::leave_tail64()
{
    launch_tail_rows64(s, ndof, MB, tail64_g, tlist.as<int>(), tc.x, du.as<double>(), true);
    tail64_g = 0;
}

// one FP64 PCG iteration of the listed members on the compact rows, with the
// stage logic of the full path
void Ens::tail64_iter()
{
    const DevMesh dm = mesh->dev();
    const int* tl = tlist.as<int>();
    const int* act = cs.active;
    const double tol2 = P.cg_tol * P.cg_tol;
    double* pd = partial.as<double>();
    int nblk;
    hipEvent_t t0;
    tstart(t0);
    launch_ebe64_ctail(s, dm, tail64_g, tl, tc.D, tc.h, tc.mat, sc, tc.p, tc.f);
    launch_gather_tail<double>(s, dm, MB, nm, tail64_g, tl, tc.f, tc.Ap, act, tc.p, pd, &nblk, true);
    launch_dashpot_tail<double>(s, dm, MB, nm, tail64_g, tl, tc.mat, 2.0 / P.dt, tc.p, tc.Ap, act, pd, &nblk);
    tstop(t0, &pc_tail32, (int64_t)mesh->ne * tail_count);
    fin(FIN_ALPHA, 1, nblk, tol2, P.cg_maxit);
    launch_tail_pcg_update(s, mesh->nn, MB, nm, tail64_g, tl, tc.x, tc.r, tc.z, tc.p, tc.Ap, tc.pinv, cs.alpha, act,
                           pd, &nblk);
    fin(FIN_BETA, 2, nblk, tol2, P.cg_maxit);
    launch_tail_p_update(s, ndof, nm, tail64_g, tl, tc.z, tc.p, cs.beta, act);
}

// inner FP32 block-Jacobi PCG: z ~ A^-1 r to inner_tol relative (preconditioner)
void Ens::inner_solve()
{
    const long n = ndof;
    int nblk;
    const int* act = cs.active;
    const int* iact = cs.inner_active;
    const double tol2 = P.inner_tol * P.inner_tol;
    double* pd = partial.as<double>();
    if (tail_g)
        launch_tail_start(s, mesh->nn, MB, nm, tail_g, tlist.as<int>(), outer_compact ? tc.r : r.as<double>(),
                          outer_compact, tb.pinv, tb.ir, tb.iz, tb.ip, act, pd, &nblk);
    else
        launch_inner_start(s, mesh->nn, MB, nm, r.as<double>(), pinv32.as<float>(), ir.as<float>(), iz.as<float>(),
                           ip.as<float>(), iw.as<float>(), iAp.as<float>(), act, pd, &nblk);
    fin(FIN_IN_START, 2, nblk, tol2, P.inner_maxit);
    int done_iters = 0;
    while (done_iters < P.inner_maxit) {
        const int chunk = std::min(check_every, P.inner_maxit - done_iters);
        run_iters(0, chunk);
        done_iters += chunk;
        if (!read_any_active(iact)) break;
    }
    // the listed members' result back to the full rows (the others are not
    // outer-active: the output step writes zero for them); with the outer
    // iteration on the compact rows it stays there
    if (tail_g && !outer_compact) launch_tail_unpack(s, n, MB, tail_g, tlist.as<int>(), tb.iz, iz.as<float>());
}

// Choose the inner operator for the next preconditioner calls from the
// outer-active flags just read into h_flags: with at most tail_max of them,
// the list goes to the device (count first) and the tail path runs on it.
void Ens::update_tail()
{
    tail_g = 0;
    if (tail_max <= 0 || inner_method == 1) return;
    int na = 0;
    for (int m = 0; m < nm; ++m) na += h_flags[m] != 0;
    if (na == 0 || na > tail_max) return;
    if (!tail_mem.p) {
        // compact rows of 32 lanes: D (elements padded to blocks of 4), h,
        // material, inverse blocks, five CG vectors, the operator's cluster
        // rows (at most 10 per element: sized as element outputs)
        const size_t ne4 = ((size_t)mesh->ne + 3) / 4 * 4, nn = mesh->nn, L = 32;
        const size_t sz[10] = {ne4 * 11 * L * 4, (size_t)mesh->ne * L * 8, (size_t)P.nl * MAT_N * L * 8,
                               nn * 6 * L * 4, nn * 3 * L * 4, nn * 3 * L * 4, nn * 3 * L * 4, nn * 3 * L * 4,
                               nn * 3 * L * 4, (size_t)mesh->ne * 30 * L * 4};
        size_t off[10], tot = 0;
        for (int i = 0; i < 10; ++i) {
            off[i] = tot;
            tot += (sz[i] + 255) / 256 * 256;
        }
        try {
            tail_mem.alloc(&ctx->budget, tot);
            tlist.alloc(&ctx->budget, (size_t)(1 + MB) * 4);
        } catch (const Error&) {  // no room: keep the full operator
            tail_mem.release();
            tlist.release();
            tail_max = 0;
            return;
        }
        char* b = (char*)tail_mem.p;
        tb.D = (uint32_t*)(b + off[0]);
        tb.h = (double*)(b + off[1]);
        tb.mat = (double*)(b + off[2]);
        tb.pinv = (float*)(b + off[3]);
        tb.ir = (float*)(b + off[4]);
        tb.iz = (float*)(b + off[5]);
        tb.ip = (float*)(b + off[6]);
        tb.w = (float*)(b + off[7]);
        tb.Ap = (float*)(b + off[8]);
        tb.f = (float*)(b + off[9]);
    }
    h_tlist[0] = na;
    tail_count = na;
    int k = 1;
    for (int m = 0; m < nm; ++m)
        if (h_flags[m]) h_tlist[k++] = m;
    // the previous list copy has completed: the caller synchronised to read h_flags
    launch_copy_i32(s, d_mail + 4 * MB, tlist.as<int>(), 1 + na);
    tail_g = na <= 16 ? 16 : 32;
    launch_tail_pack(s, mesh->dev(), MB, tail_g, P.nl, tlist.as<int>(), D16.as<uint32_t>(), h.as<double>(),
                     mat.as<double>(), pinv32.as<float>(), tb.D, tb.h, tb.mat, tb.pinv);
}

// one inner CG iteration of the listed members on the compact rows: the
// operator (cluster rows, node sums, dashpot), then the updates of the
// full path with the same per-member stage logic
void Ens::tail_iter()
{
    const DevMesh dm = mesh->dev();
    const int* tl = tlist.as<int>();
    const int* iact = cs.inner_active;
    const double tol2 = P.inner_tol * P.inner_tol;
    double* pd = partial.as<double>();
    int nblk;
    hipEvent_t t0;
    tstart(t0);
    launch_ebe32_ctail(s, dm, tail_g, tl, tb.D, tb.h, tb.mat, sc, tb.ip, tb.f);
    launch_gather_tail(s, dm, MB, nm, tail_g, tl, tb.f, tb.Ap, iact, tb.ip, pd, &nblk, true);
    launch_dashpot_tail(s, dm, MB, nm, tail_g, tl, tb.mat, (float)(2.0 / P.dt), tb.ip, tb.Ap, iact, pd, &nblk);
    tstop(t0, &pc_tail32, (int64_t)mesh->ne * tail_count);
    fin(FIN_IN_ALPHA, 1, nblk, tol2, P.inner_maxit);
    launch_tail_update(s, mesh->nn, MB, nm, tail_g, tl, tb.ir, tb.w, tb.Ap, tb.pinv, cs.ialpha, iact, pd, &nblk);
    fin(FIN_IN_BETA, 2, nblk, tol2, P.inner_maxit);
    launch_tail_pz(s, ndof, nm, tail_g, tl, tb.iz, tb.ip, tb.w, cs.ialpha, cs.ibeta, cs.inner_upd);
}

// Chebyshev inner solve of degree inner_maxit for the outer-active members,
// with the coefficient table of the step (from the first inner CG solve).
// The whole solve has fixed launches, so it is captured once into a hipGraph.
void Ens::cheb_body()
{
    const int n = std::min(P.inner_maxit, kChebMax);
    const int* act = cs.active;
    const DevMesh dm = mesh->dev();
    const float* cheb = chebc.as<float>();
    const float* pv = pinv32.as<float>();
    launch_cheb_start(s, mesh->nn, MB, nm, r.as<double>(), pv, cheb, ir.as<float>(), iz.as<float>(), ip.as<float>(),
                      act);
    float* d = ip.as<float>();
    float* dn = iw.as<float>();
    const bool fused = scatter == 2 && (qb.p || dm.nbn == 0);
    for (int k = 0; k < n; ++k) {
        const bool last = k + 1 == n;
        if (fused) {
            set_cluster_blocks(cluster_blocks);
            hipEvent_t t0;
            tstart(t0);
            launch_ebe_cluster32(s, dm, MB, nm, D32.as<float>(), D16.as<uint32_t>(), h.as<double>(),
                                 mat.as<double>(), sc, d, (float*)cbuf.p, act, d16_mean);
            tstop(t0, &pc_ebe32, (int64_t)mesh->ne * nm);
            launch_dashpot_rows(s, dm, MB, nm, mat.as<double>(), (float)(2.0 / P.dt), d, qb.as<float>(), act);
            tstart(t0);
            launch_gather_cheb(s, dm, MB, nm, k, last, (const float*)cbuf.p, qb.as<float>(), iz.as<float>(),
                               ir.as<float>(), d, dn, pv, cheb, act);
            tstop(t0, &pc_gather32, (int64_t)mesh->nn * nm);
        } else {
            ebe32(d, iAp.as<float>(), act, nullptr);
            launch_cheb_update(s, mesh->nn, MB, nm, k, last, iz.as<float>(), ir.as<float>(), d, iAp.as<float>(), dn,
                               pv, cheb, act);
        }
        std::swap(d, dn);
    }
    launch_finalize(s, FIN_CHEB_COUNT, 0, MB, nm, partial.as<double>(), 0, cs, 0.0, n);
}

// Largest eigenvalue of the block-Jacobi preconditioned inner operator, from
// cheb_est_iters inner CG iterations on a random right-hand side for the
// members of this step (z serves as that vector: the outer solve overwrites
// it before reading it).  Raises the running upper bound of the Chebyshev
// interval; runs before the step's solve every cheb_est_every steps.
void Ens::cheb_estimate()
{
    const long n = ndof;
    int nblk;
    launch_fill_random(s, z.as<double>(), n * MB, 0x5851F42D4C957F2Dull + (uint64_t)steps_done);
    launch_inner_start(s, mesh->nn, MB, nm, z.as<double>(), pinv32.as<float>(), ir.as<float>(), iz.as<float>(),
                       ip.as<float>(), iw.as<float>(), iAp.as<float>(), stepping.as<int>(), partial.as<double>(),
                       &nblk);
    fin(FIN_EST_START, 2, nblk, 0.0, 0);
    const int keep_it = P.inner_maxit;
    const double keep_tol = P.inner_tol;
    P.inner_maxit = std::min(cheb_est_iters, kLanczosMax);
    P.inner_tol = 0.0;
    est_iters = P.inner_maxit;
    try {
        for (int i = 0; i < P.inner_maxit; ++i) inner_iter();
    } catch (...) {
        P.inner_maxit = keep_it;
        P.inner_tol = keep_tol;
        throw;
    }
    P.inner_maxit = keep_it;
    P.inner_tol = keep_tol;
    launch_cheb_hi_estimate(s, MB, nm, cs, cheb_est_scale, cheb_bounds.as<double>());
}

void Ens::cheb_solve()
{
    if (!use_graph || profile) {
        cheb_body();
        return;
    }
    if (!g_cheb) {
        hipGraph_t g = nullptr;
        NLTH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            cheb_body();
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        NLTH_HIP(hipStreamEndCapture(s, &g));
        hipError_t e = hipGraphInstantiate(&g_cheb, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            g_cheb = nullptr;
            use_graph = false;
            cheb_body();
            return;
        }
    }
    NLTH_HIP(hipGraphLaunch(g_cheb, s));
}

// one inner FP32 PCG iteration (every launch reads its scalars on the device)
void Ens::inner_iter()
{
    if (tail_g) {
        tail_iter();
        return;
    }
    const long n = ndof;
    int nblk;
    const int* iact = cs.inner_active;
    const double tol2 = P.inner_tol * P.inner_tol;
    double* pd = partial.as<double>();
    ebe32(ip.as<float>(), iAp.as<float>(), iact, &nblk);
    fin(FIN_IN_ALPHA, 1, nblk, tol2, P.inner_maxit);
    launch_inner_update(s, mesh->nn, MB, nm, ir.as<float>(), iw.as<float>(), iAp.as<float>(), pinv32.as<float>(),
                        cs.ialpha, iact, pd, &nblk);
    fin(FIN_IN_BETA, 2, nblk, tol2, P.inner_maxit);
    launch_inner_pz(s, n, MB, nm, iz.as<float>(), ip.as<float>(), iw.as<float>(), cs.ialpha, cs.ibeta, cs.inner_upd);
}

// one FP64 block-Jacobi PCG iteration
void Ens::pcg_iter()
{
    if (tail64_g) {
        tail64_iter();
        return;
    }
    const long n = ndof;
    int nblk;
    double* x = du.as<double>();
    const int* act = cs.active;
    const double tol2 = P.cg_tol * P.cg_tol;
    double* pd = partial.as<double>();
    apply_A64(p.as<double>(), Ap.as<double>(), act, &nblk);
    fin(FIN_ALPHA, 1, nblk, tol2, P.cg_maxit);
    launch_pcg_update(s, mesh->nn, MB, nm, x, r.as<double>(), z.as<double>(), p.as<double>(), Ap.as<double>(),
                      pinv.as<double>(), cs.alpha, act, pd, &nblk);
    fin(FIN_BETA, 2, nblk, tol2, P.cg_maxit);
    launch_p_update<double>(s, n, MB, nm, z.as<double>(), p.as<double>(), cs.beta, act, nullptr);
}

void Ens::clear_graphs()
{
    for (auto& kv : g_chunks)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    g_chunks.clear();
    if (g_cheb) (void)hipGraphExecDestroy(g_cheb);
    g_cheb = nullptr;
}

// k iterations of kind 0 (inner) or 1 (FP64 PCG); a chunk of k iterations is
// captured once into a hipGraph per (kind, compact-row width, k) and replayed
// (the launches and their arguments are the same every chunk: scalars are
// read on the device), which removes per-launch host overhead
void Ens::run_iters(int kind, int k)
{
    if (!use_graph || profile || k <= 0 || k > 64) {
        for (int i = 0; i < k; ++i) kind == 0 ? inner_iter() : pcg_iter();
        return;
    }
    const int g = kind == 1 ? tail64_g : tail_g;
    hipGraphExec_t& ge = g_chunks[(kind * 64 + g) * 128 + k];
    if (!ge) {
        hipGraph_t g = nullptr;
        NLTH_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        try {
            for (int i = 0; i < k; ++i) kind == 0 ? inner_iter() : pcg_iter();
        } catch (...) {
            (void)hipStreamEndCapture(s, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        NLTH_HIP(hipStreamEndCapture(s, &g));
        hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            ge = nullptr;
            use_graph = false;  // fall back to direct launches of the same kernels
            for (int i = 0; i < k; ++i) kind == 0 ? inner_iter() : pcg_iter();
            return;
        }
    }
    NLTH_HIP(hipGraphLaunch(ge, s));
}

// FP64 flexible CG (Polak-Ribiere beta) preconditioned by the inner FP32 PCG
void Ens::solve_fcg()
{
    const long n = ndof;
    int nblk;
    double* x = du.as<double>();
    const int* st = stepping.as<int>();
    const int* act = cs.active;
    const double tol2 = P.cg_tol * P.cg_tol;
    double* pd = partial.as<double>();
    tail_g = 0;
    apply_A64(x, Ap.as<double>(), st);
    launch_pcg_start(s, mesh->nn, MB, nm, b.as<double>(), Ap.as<double>(), pinv.as<double>(), r.as<double>(),
                     z.as<double>(), p.as<double>(), st, pd, &nblk);
    fin(FIN_FCG_START, 2, nblk, tol2, P.cg_maxit);
    if (est_iters) {  // the spectrum estimate of this step counts as inner iterations
        fin(FIN_CHEB_COUNT, 0, 0, 0.0, est_iters);
        est_iters = 0;
    }
    launch_zero_if_b0(s, n, MB, nm, x, cs.bb, st);
    if (!read_any_active(act)) return;
    update_tail();
    inner_solve();
    // Chebyshev for the later preconditioner calls of this step: spectrum
    // bounds of each member from the Lanczos matrix of the CG solve just done
    const bool cheb = inner_method == 1 && P.inner_maxit >= 1;
    if (cheb)
        launch_cheb_bounds(s, MB, nm, cs, std::min(P.inner_maxit, kChebMax), cheb_lo, cheb_hi, chebc.as<float>(),
                           cheb_bounds.as<double>());
    launch_inner_out(s, n, MB, nm, iz.as<float>(), z.as<double>(), Ap.as<double>(), r.as<double>(), act, pd, &nblk);
    fin(FIN_FCG_RZ, 2, nblk, tol2, P.cg_maxit);
    launch_p_update<double>(s, n, MB, nm, z.as<double>(), p.as<double>(), nullptr, act, nullptr);
    outer_compact = false;
    const DevMesh dm = mesh->dev();
    for (;;) {
        if (outer_compact) {
            const int* tl = tlist.as<int>();
            hipEvent_t t0;
            tstart(t0);
            launch_ebe64_ctail(s, dm, tail_g, tl, tc.D, tc.h, tc.mat, sc, tc.p, tc.f);
            launch_gather_tail<double>(s, dm, MB, nm, tail_g, tl, tc.f, tc.Ap, act, tc.p, pd, &nblk, true);
            launch_dashpot_tail<double>(s, dm, MB, nm, tail_g, tl, tc.mat, 2.0 / P.dt, tc.p, tc.Ap, act, pd, &nblk);
            tstop(t0, &pc_ebe64, (int64_t)mesh->ne * tail_count);  // an FP64 operator application
            fin(FIN_ALPHA, 1, nblk, tol2, P.cg_maxit);
            launch_tail_xr_update(s, n, MB, nm, tail_g, tl, tc.x, tc.r, tc.p, tc.Ap, cs.alpha, act, pd, &nblk);
        } else {
            apply_A64(p.as<double>(), Ap.as<double>(), act, &nblk);
            fin(FIN_ALPHA, 1, nblk, tol2, P.cg_maxit);
            launch_xr_update(s, n, MB, nm, x, r.as<double>(), p.as<double>(), Ap.as<double>(), cs.alpha, act, pd,
                             &nblk);
        }
        fin(FIN_FCG_RR, 1, nblk, tol2, P.cg_maxit);
        if (!read_any_active(act)) break;
        if (!outer_compact) {
            update_tail();
            enter_outer_tail();
        } else {
            tail_count = count_flags();  // the listed members still iterating
        }
        if (cheb) cheb_solve();
        else inner_solve();
        if (outer_compact) {
            const int* tl = tlist.as<int>();
            launch_tail_inner_out(s, n, MB, nm, tail_g, tl, tb.iz, tc.z, tc.Ap, tc.r, act, pd, &nblk);
            fin(FIN_FCG_BETA, 2, nblk, tol2, P.cg_maxit);
            launch_tail_p_update(s, n, nm, tail_g, tl, tc.z, tc.p, cs.beta, act);
        } else {
            launch_inner_out(s, n, MB, nm, iz.as<float>(), z.as<double>(), Ap.as<double>(), r.as<double>(), act, pd,
                             &nblk);
            fin(FIN_FCG_BETA, 2, nblk, tol2, P.cg_maxit);
            launch_p_update<double>(s, n, MB, nm, z.as<double>(), p.as<double>(), cs.beta, act, nullptr);
        }
    }
    if (outer_compact) launch_tail_rows64(s, n, MB, tail_g, tlist.as<int>(), tc.x, x, true);
    outer_compact = false;
    tail_g = 0;
}

void Ens::law_phase()
{
    const DevMesh dm = mesh->dev();
    const size_t per_elem = (size_t)4 * P.ns * MB * theta_bytes(P.depth);
    if (!paged) {
        hipEvent_t t0;
        tstart(t0);
        launch_law(s, dm, MB, nm, 0, mesh->ne, ne_pad, mat.as<double>(), P.nl, nonlinear.as<int>(), P.ns, P.depth, dirs.as<double>(),
                   w.as<double>(), du.as<double>(), theta.p, D64.as<double>(), D32.as<float>(), D16.as<uint32_t>(), h.as<double>(),
                   stepping.as<int>(), d16_mean);
        tstop(t0, &pc_law, (int64_t)mesh->ne * nm);
        return;
    }
    if (zero_copy) {
        // ablation of the pipeline: the kernel reads and writes the pinned
        // host state over the host link itself, chunk by chunk (the footnote
        // of Section 2.3 measures this form on GH200).  Earlier write-backs of
        // the pipelined form must have landed first.
        for (int slot = 0; slot < ring; ++slot) NLTH_HIP(hipStreamWaitEvent(s, ev_d2h[slot], 0));
        for (int cix = 0; cix < nchunks; ++cix) {
            hipEvent_t t0;
            tstart(t0);
            launch_law(s, dm, MB, nm, chunk_e0[cix], chunk_ec[cix], chunk_ecp[cix], mat.as<double>(), P.nl,
                       nonlinear.as<int>(), P.ns, P.depth, dirs.as<double>(), w.as<double>(), du.as<double>(),
                       (char*)theta_host.p + chunk_off[cix], D64.as<double>(), D32.as<float>(), D16.as<uint32_t>(),
                       h.as<double>(), stepping.as<int>(), d16_mean);
            tstop(t0, &pc_law, (int64_t)chunk_ec[cix] * nm);
            prefetched[cix] = false;
        }
        NLTH_HIP(hipEventRecord(ev_zc, s));
        return;
    }
    // Algorithm 3 pipeline over a ring of device slots: chunk c goes back to
    // the host (after its law kernel, on the compute stream) while chunk c+1
    // comes in on the copy stream
    for (int cix = 0; cix < nchunks; ++cix) {
        const int slot = cix % ring;
        char* dslot = (char*)theta.p + (size_t)slot * chunk_elems * per_elem;
        const size_t bytes = (size_t)chunk_ecp[cix] * per_elem;
        if (!prefetched[cix]) {
            if (slot_chunk[slot] >= 0) NLTH_HIP(hipStreamWaitEvent(s_h2d, ev_d2h[slot], 0));
            NLTH_HIP(hipStreamWaitEvent(s_h2d, ev_zc, 0));  // host state written by a zero-copy pass
            NLTH_HIP(hipMemcpyAsync(dslot, (char*)theta_host.p + chunk_off[cix], bytes, hipMemcpyHostToDevice, s_h2d));
            NLTH_HIP(hipEventRecord(ev_h2d[slot], s_h2d));
            h2d_bytes += bytes;
        }
        prefetched[cix] = false;
        slot_chunk[slot] = cix;
        NLTH_HIP(hipStreamWaitEvent(s, ev_h2d[slot], 0));
        hipEvent_t t0;
        tstart(t0);
        launch_law(s, dm, MB, nm, chunk_e0[cix], chunk_ec[cix], chunk_ecp[cix], mat.as<double>(), P.nl, nonlinear.as<int>(), P.ns, P.depth,
                   dirs.as<double>(), w.as<double>(), du.as<double>(), dslot, D64.as<double>(), D32.as<float>(), D16.as<uint32_t>(),
                   h.as<double>(), stepping.as<int>(), d16_mean);
        tstop(t0, &pc_law, (int64_t)chunk_ec[cix] * nm);
        // the write-back follows the law kernel on the compute stream (the
        // runtime copies to pinned host memory with a blit kernel, which on a
        // stream of its own could share a hardware queue with the other member
        // set's solve and hold it back); the next chunk's transfer in runs
        // meanwhile on the copy stream
        NLTH_HIP(hipMemcpyAsync((char*)theta_host.p + chunk_off[cix], dslot, bytes, hipMemcpyDeviceToHost, s));
        NLTH_HIP(hipEventRecord(ev_d2h[slot], s));
        d2h_bytes += bytes;
    }
    // the next step's first chunks are prefetched now so their transfer
    // overlaps the next solve (each waits for its slot's write-back)
    prefetch_next();
}

void Ens::prefetch_next()
{
    const size_t per_elem = (size_t)4 * P.ns * MB * theta_bytes(P.depth);
    for (int cix = 0; cix < std::min(ring - 1, nchunks); ++cix) {
        const int slot = cix % ring;
        char* dslot = (char*)theta.p + (size_t)slot * chunk_elems * per_elem;
        const size_t bytes = (size_t)chunk_ecp[cix] * per_elem;
        // the slot's previous chunk must be back on the host; chunk cix's own
        // write-back precedes that one on the D2H stream
        NLTH_HIP(hipStreamWaitEvent(s_h2d, ev_d2h[slot], 0));
        NLTH_HIP(hipMemcpyAsync(dslot, (char*)theta_host.p + chunk_off[cix], bytes, hipMemcpyHostToDevice, s_h2d));
        NLTH_HIP(hipEventRecord(ev_h2d[slot], s_h2d));
        h2d_bytes += bytes;
        prefetched[cix] = true;
    }
}

void Ens::one_step()
{
    enqueue_step();
    read_status();
}

// wait for the stream, then the member status from the mailbox
void Ens::read_status()
{
    launch_copy_i32(s, cs.status, d_mail + MB, MB);
    sync();
    std::copy(h_mail + MB, h_mail + 2 * MB, h_status.begin());
}

void Ens::enqueue_step()
{
    const DevMesh dm = mesh->dev();
    // the previous step has completed (its status was read), so the mailbox is free
    std::copy(h_member_step.begin(), h_member_step.end(), h_mail + 2 * MB);
    std::copy(h_stepping.begin(), h_stepping.end(), h_mail + 3 * MB);
    launch_copy_i32(s, d_mail + 2 * MB, member_step.as<int>(), MB);
    launch_copy_i32(s, d_mail + 3 * MB, stepping.as<int>(), MB);
    const int ns_steps = std::max(1, P.n_steps);
    launch_pick_vI(s, MB, nm, ns_steps, vI_all.as<double>(), member_step.as<int>(), vI_cur.as<double>());
    hipEvent_t t0;
    tstart(t0);
    build_rhs();
    build_diag();
    tstop(t0, &pc_other, 0);
    if (P.precision == NLTH_MIXED && inner_method == 1 &&
        (cheb_est_age < 0 || cheb_est_age >= cheb_est_every)) {
        cheb_estimate();
        cheb_est_age = 0;
    }
    if (cheb_est_age >= 0) ++cheb_est_age;
    // CG initial guess: the last increment, or its extrapolation in time
    launch_predict(s, ndof, MB, nm, predictor, du.as<double>(), du2.as<double>(), du3.as<double>(),
                   stepping.as<int>());
    if (P.precision == NLTH_FP64) solve_pcg();
    else solve_fcg();
    tstart(t0);
    ebe(OP_K, du.as<double>(), nullptr, q.as<double>(), stepping.as<int>(), q.as<double>(), 1.0, 0.0, nullptr,
        nullptr);
    launch_newmark(s, ndof, MB, nm, du.as<double>(), u.as<double>(), v.as<double>(), a.as<double>(), P.dt,
                   stepping.as<int>());
    tstop(t0, &pc_other, 0);
    law_phase();
    launch_receivers(s, mesh->nrecv, mesh->recv_d.as<int>(), MB, nm, v.as<double>(), hist.as<double>(),
                     member_step.as<int>(), ns_steps, vmax.as<double>(), stepping.as<int>());
    launch_record_iters(s, MB, nm, ns_steps, member_step.as<int>(), stepping.as<int>(), cs.iters, cs.inner_total,
                        iters_dev.as<int>());
}

void Ens::step_begin()
{
    for (int m = 0; m < MB; ++m) {
        h_member_step[m] = steps_done;
        h_stepping[m] = (m < nm && h_status[m] == 0) ? 1 : 0;
    }
    enqueue_step();
}

void Ens::step_end()
{
    read_status();  // after the step's law phase
    ++steps_done;
}

// Two member sets A (this) and B (twin): A's solve of step k runs while B's
// law state of step k-1 streams, then B's solve of step k while A's law state
// of step k streams.  Each set's solve waits on its own stream only.  (The
// chunk pipeline of Alg. 3 overlaps the transfers with the law kernels alone,
// which take a tenth of the link time here; Alg. 4 runs its two sets' solves
// together and then their law updates.)
void Ens::step_pair(int n_steps)
{
    auto t0 = std::chrono::steady_clock::now();
    Ens& A = *this;
    Ens& B = *twin;
    const int n = std::min(n_steps, P.n_steps - steps_done);
    if (n > 0) A.step_begin();
    for (int k = 0; k < n; ++k) {
        B.step_begin();
        A.step_end();
        if (k + 1 < n) A.step_begin();
        B.step_end();
    }
    NLTH_HIP(hipStreamSynchronize(s_h2d));
    ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void Ens::step_all(int n_steps)
{
    auto t0 = std::chrono::steady_clock::now();
    for (int k = 0; k < n_steps && steps_done < P.n_steps; ++k) {
        for (int m = 0; m < MB; ++m) {
            h_member_step[m] = steps_done;
            h_stepping[m] = (m < nm && h_status[m] == 0) ? 1 : 0;
        }
        one_step();
        ++steps_done;
    }
    if (paged) {
        NLTH_HIP(hipStreamSynchronize(s_h2d));
    }
    ms_total += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void Ens::read(nlth_result* res) const
{
    if (!res) return;
    const int ns_steps = std::max(1, P.n_steps);
    const int nr = std::max(1, mesh->nrecv);
    if (res->vel && P.n_steps > 0 && mesh->nrecv > 0)
        NLTH_HIP(hipMemcpy(res->vel, hist.p, (size_t)nm * ns_steps * nr * 3 * 8, hipMemcpyDeviceToHost));
    if (res->iters && P.n_steps > 0)
        NLTH_HIP(hipMemcpy(res->iters, iters_dev.p, (size_t)nm * ns_steps * 2 * 4, hipMemcpyDeviceToHost));
    if (res->vmax && mesh->nrecv > 0)
        NLTH_HIP(hipMemcpy(res->vmax, vmax.p, (size_t)nm * nr * 8, hipMemcpyDeviceToHost));
    if (res->member_status)
        for (int m = 0; m < nm; ++m) res->member_status[m] = h_status[m];
}

Ctx::~Ctx()
{
    {
        std::lock_guard<std::mutex> g(smu);
        stop = true;
    }
    scv.notify_all();
    if (worker.joinable()) worker.join();
    serve_shutdown(this);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
}

}  // namespace nlth

using namespace nlth;

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

#define API_BEGIN(ctxp) \
    Ctx* ctx_ = (ctxp);  \
    try {
#define API_END                                 \
    }                                           \
    catch (const Error& e) {                    \
        set_error(ctx_, e);                     \
        return e.code;                          \
    }                                           \
    catch (const std::bad_alloc&) {             \
        set_error(ctx_, Error{NLTH_ENOMEM_HOST, "host allocation failed"}); \
        return NLTH_ENOMEM_HOST;                \
    }                                           \
    return NLTH_OK;

struct nlth_ctx : Ctx {};
struct nlth_mesh : Mesh {};
struct nlth_ens : Ens {};

extern "C" {

int nlth_version(void) { return NLTH_VERSION; }

const char* nlth_last_error(const nlth_ctx* ctx)
{
    if (ctx) return ctx->last_error.c_str();
    std::lock_guard<std::mutex> g(g_err_mu);
    static thread_local std::string copy;
    copy = g_err;
    return copy.c_str();
}

int nlth_ctx_create(int device, const nlth_ctx_opts* opts, nlth_ctx** out)
{
    API_BEGIN(nullptr)
    if (!out) throw Error{NLTH_EINVAL, "out is NULL"};
    *out = nullptr;
    std::unique_ptr<nlth_ctx> c(new nlth_ctx());
    c->device = device;
    c->host_only = device == NLTH_DEVICE_NONE;
    if (opts) {
        c->log_level = opts->log_level;
        if (opts->max_batch > 0) c->max_batch = opts->max_batch;
        if (opts->paging_sets < 0 || opts->paging_sets > 2) throw Error{NLTH_EINVAL, "paging_sets must be 0, 1 or 2"};
        c->paging_sets = opts->paging_sets == 1 ? 1 : 2;
    }
    c->budget.host_limit = (opts && opts->host_budget > 0) ? opts->host_budget : (int64_t)64 << 30;
    if (!c->host_only) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n)
            throw Error{NLTH_EDEVICE, "no such HIP device"};
        NLTH_HIP(hipSetDevice(device));
        scratch_setup(device);
        size_t fr = 0, tot = 0;
        NLTH_HIP(hipMemGetInfo(&fr, &tot));
        c->budget.limit = (opts && opts->hbm_budget > 0) ? opts->hbm_budget : (int64_t)(0.9 * fr);
        if (opts && opts->stream) {
            c->stream = (hipStream_t)opts->stream;
        } else {
            NLTH_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->own_stream = true;
        }
    }
    *out = c.release();
    API_END
}

int nlth_ctx_destroy(nlth_ctx* ctx)
{
    if (!ctx) return NLTH_OK;
    {
        std::lock_guard<std::mutex> g(ctx->smu);
        for (auto& kv : ctx->requests)
            if (kv.second->state.load() < 2) {
                set_error(ctx, Error{NLTH_EBUSY, "context has unfinished requests"});
                return NLTH_EBUSY;
            }
    }
    if (ctx->live_meshes.load() > 0) {
        set_error(ctx, Error{NLTH_EBUSY, "context still has meshes"});
        return NLTH_EBUSY;
    }
    delete ctx;
    return NLTH_OK;
}

int nlth_mesh_create(nlth_ctx* ctx, const nlth_mesh_desc* d, nlth_mesh** out)
{
    API_BEGIN(ctx)
    if (!ctx || !out) throw Error{NLTH_EINVAL, "ctx/out is NULL"};
    *out = nullptr;
    std::lock_guard<std::mutex> g(ctx->mu);
    if (!ctx->host_only) NLTH_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<nlth_mesh> m(new nlth_mesh());
    build_mesh(ctx, d, *m);
    ctx->live_meshes++;
    *out = m.release();
    API_END
}

int nlth_mesh_destroy(nlth_mesh* mesh)
{
    if (!mesh) return NLTH_OK;
    Ctx* c = mesh->ctx;
    if (mesh->refs.load() > 0) {
        set_error(c, Error{NLTH_EBUSY, "mesh is referenced by a pending request"});
        return NLTH_EBUSY;
    }
    {
        std::lock_guard<std::mutex> g(c->mu);
        delete mesh;
    }
    c->live_meshes--;
    return NLTH_OK;
}

int nlth_mesh_query(const nlth_mesh* mesh, nlth_mesh_info* info, int32_t* elem_order, int32_t* color_offsets)
{
    API_BEGIN(mesh ? mesh->ctx : nullptr)
    if (!mesh) throw Error{NLTH_EINVAL, "mesh is NULL"};
    if (info) {
        info->n_nodes = mesh->nn;
        info->n_tets = mesh->ne;
        info->n_colors = mesh->ncolor;
        info->n_clusters = mesh->ncl;
        info->cluster_rows = mesh->cl_rows;
        info->n_bnodes = mesh->nbn;
        info->volume = mesh->volume;
    }
    if (elem_order)
        for (int i = 0; i < mesh->ne; ++i) elem_order[i] = mesh->order[mesh->color_elems[i]];
    if (color_offsets) std::copy(mesh->color_off.begin(), mesh->color_off.end(), color_offsets);
    API_END
}

int nlth_ens_create(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, nlth_ens** out)
{
    API_BEGIN(ctx)
    if (!ctx || !mesh || !out) throw Error{NLTH_EINVAL, "ctx/mesh/out is NULL"};
    if (mesh->ctx != ctx) throw Error{NLTH_EINVAL, "mesh belongs to another context"};
    *out = nullptr;
    Problem P;
    copy_problem(prob, P);
    if (P.nl <= mesh->max_layer) throw Error{NLTH_EINVAL, "problem: mesh uses a layer id >= n_layers"};
    if (ctx->host_only) throw Error{NLTH_EDEVICE, "host-only context cannot run solves"};
    std::lock_guard<std::mutex> g(ctx->mu);
    NLTH_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<nlth_ens> e(new nlth_ens());
    int64_t avail;
    {
        std::lock_guard<std::mutex> gb(ctx->budget.mu);
        avail = ctx->budget.limit > 0 ? ctx->budget.limit - ctx->budget.used : INT64_MAX;
    }
    if (ctx->paging_sets == 2 && P.nm >= 2 && ensemble_bytes(*mesh, P, pad_members(P.nm), false) > avail) {
        // the law state will not stay resident: two member sets, so that the
        // transfers of one overlap the solve of the other
        const int nA = (P.nm + 1) / 2;
        const Problem PA = member_slice(P, 0, nA), PB = member_slice(P, nA, P.nm - nA);
        e->force_paged = true;
        e->reserve_extra = ensemble_bytes(*mesh, PB, pad_members(PB.nm), true);
        e->create(ctx, mesh, PA);
        std::unique_ptr<Ens> b(new Ens());
        b->force_paged = true;
        b->member_base = nA;
        b->shared_copy_streams = true;
        b->s_h2d = e->s_h2d;
        NLTH_HIP(hipStreamCreateWithFlags(&b->own_s, hipStreamNonBlocking));
        b->create(ctx, mesh, PB);
        e->twin = std::move(b);
    } else {
        e->create(ctx, mesh, P);
    }
    *out = e.release();
    API_END
}

int nlth_ens_step(nlth_ens* ens, int32_t n_steps)
{
    API_BEGIN(ens ? ens->ctx : nullptr)
    if (!ens || n_steps < 0) throw Error{NLTH_EINVAL, "ens is NULL or n_steps < 0"};
    std::lock_guard<std::mutex> g(ens->ctx->mu);
    NLTH_HIP(hipSetDevice(ens->ctx->device));
    if (ens->twin) ens->step_pair(n_steps);
    else ens->step_all(n_steps);
    for (const Ens* e = ens; e; e = e->twin.get())
        for (int m = 0; m < e->nm; ++m)
            if (e->h_status[m] != 0) {
                char buf[128];
                snprintf(buf, sizeof buf, "member %d: CG did not converge within cg_maxit", e->member_base + m);
                throw Error{NLTH_ENOCONV, buf};
            }
    API_END
}

int nlth_ens_read(nlth_ens* ens, nlth_result* res)
{
    API_BEGIN(ens ? ens->ctx : nullptr)
    if (!ens) throw Error{NLTH_EINVAL, "ens is NULL"};
    std::lock_guard<std::mutex> g(ens->ctx->mu);
    NLTH_HIP(hipSetDevice(ens->ctx->device));
    ens->read(res);
    if (const Ens* b = ens->twin.get()) {  // the second set's members follow the first's
        const long ns_steps = std::max(1, ens->P.n_steps), nr = std::max(1, ens->mesh->nrecv), m0 = b->member_base;
        nlth_result rb{};
        rb.vel = res->vel ? res->vel + m0 * ns_steps * nr * 3 : nullptr;
        rb.iters = res->iters ? res->iters + m0 * ns_steps * 2 : nullptr;
        rb.member_status = res->member_status ? res->member_status + m0 : nullptr;
        rb.vmax = res->vmax ? res->vmax + m0 * nr : nullptr;
        b->read(&rb);
    }
    API_END
}

int nlth_ens_destroy(nlth_ens* ens)
{
    if (!ens) return NLTH_OK;
    Ctx* c = ens->ctx;
    std::lock_guard<std::mutex> g(c->mu);
    (void)hipSetDevice(c->device);
    delete ens;
    return NLTH_OK;
}

int nlth_ens_set_profile(nlth_ens* ens, int32_t profile)
{
    if (!ens) return NLTH_EINVAL;
    for (Ens* e = ens; e; e = e->twin.get()) e->profile = profile != 0;
    return NLTH_OK;
}

static void apply_tuning(Ens* ens, const nlth_tuning* t);

int nlth_ens_set_tuning(nlth_ens* ens, const nlth_tuning* t)
{
    API_BEGIN(ens ? ens->ctx : nullptr)
    if (!ens || !t) throw Error{NLTH_EINVAL, "ens/tuning is NULL"};
    if (t->ebe_block != 0 && t->ebe_block != 64 && t->ebe_block != 128 && t->ebe_block != 256)
        throw Error{NLTH_EINVAL, "ebe_block must be 0, 64, 128 or 256"};
    if (t->check_every < 0 || t->check_every > 64) throw Error{NLTH_EINVAL, "check_every must be in [0, 64]"};
    if (t->inner_maxit < 0 || t->inner_maxit > 100000 || !(t->inner_tol >= 0) || t->inner_tol >= 1)
        throw Error{NLTH_EINVAL, "inner_maxit must be in [0, 100000] and inner_tol in [0, 1)"};
    if (t->scatter < -1 || t->scatter > 2) throw Error{NLTH_EINVAL, "scatter must be -1, 0, 1 or 2"};
    if (t->cluster_blocks != 0 && (t->cluster_blocks < 2 || t->cluster_blocks > 4))
        throw Error{NLTH_EINVAL, "cluster_blocks must be 0, 2, 3 or 4"};
    if ((t->scatter == 0 && !ens->fbuf.p) || (t->scatter == 2 && !ens->cbuf.p))
        throw Error{NLTH_EINVAL, "scatter: element outputs need fewer than 64 member slots, clusters 64..256"};
    if (t->inner_method < -1 || t->inner_method > 1) throw Error{NLTH_EINVAL, "inner_method must be -1, 0 or 1"};
    if (t->zero_copy < -1 || t->zero_copy > 1) throw Error{NLTH_EINVAL, "zero_copy must be -1, 0 or 1"};
    if (t->tail_members != -1 && t->tail_members != 0 && t->tail_members != 16 && t->tail_members != 32)
        throw Error{NLTH_EINVAL, "tail_members must be -1, 0, 16 or 32"};
    if (t->tail_members > 0 &&
        (ens->MB < 64 || ens->MB > 256 || (ens->P.precision == NLTH_MIXED && !ens->d16_mean)))
        throw Error{NLTH_EINVAL, "tail_members needs an ensemble of 64..256 member slots (FP64, or mixed with the "
                                 "element-mean inner D)"};
    if (t->zero_copy == 1 && !ens->paged) throw Error{NLTH_EINVAL, "zero_copy needs an ensemble whose law state is paged"};
    if (t->predictor < -1 || t->predictor > 2) throw Error{NLTH_EINVAL, "predictor must be -1, 0, 1 or 2"};
    if ((t->inner_method == 1 || (t->inner_method == -1 && ens->inner_method == 1)) &&
        (t->inner_maxit ? t->inner_maxit : ens->P.inner_maxit) > kChebMax)
        throw Error{NLTH_EINVAL, "the Chebyshev degree (inner_maxit) must be at most 64"};
    std::lock_guard<std::mutex> g(ens->ctx->mu);
    for (Ens* e = ens; e; e = e->twin.get()) apply_tuning(e, t);
    return NLTH_OK;
    API_END
}

static void apply_tuning(Ens* ens, const nlth_tuning* t)
{
    if (t->ebe_block) ens->ebe_block = t->ebe_block;
    if (t->check_every) ens->check_every = t->check_every;
    if (t->use_graph >= 0) ens->use_graph = t->use_graph != 0;
    if (t->inner_maxit) ens->P.inner_maxit = t->inner_maxit;
    if (t->inner_tol > 0) ens->P.inner_tol = t->inner_tol;
    if (t->scatter >= 0) ens->scatter = t->scatter;
    if (t->cluster_blocks > 0) ens->cluster_blocks = t->cluster_blocks;
    if (t->inner_method >= 0) ens->inner_method = t->inner_method;
    if (t->zero_copy >= 0) ens->zero_copy = t->zero_copy != 0;
    if (t->tail_members >= 0) ens->tail_max = t->tail_members;
    if (t->predictor >= 0) ens->predictor = t->predictor;
    ens->tail_g = 0;
    ens->clear_graphs();  // captured chunks hold the old launch shapes
}

int nlth_ens_reset_stats(nlth_ens* ens)
{
    if (!ens) return NLTH_EINVAL;
    for (Ens* e = ens; e; e = e->twin.get()) {
        e->pc_ebe64 = e->pc_ebe32 = e->pc_gather32 = e->pc_vec = e->pc_law = e->pc_other = e->pc_tail32 = ProfCat{};
        e->ms_total = e->ms_copy = 0;
        e->h2d_bytes = e->d2h_bytes = 0;
    }
    return NLTH_OK;
}

int nlth_ens_stats(const nlth_ens* ens, nlth_stats* st)
{
    API_BEGIN(ens ? ens->ctx : nullptr)
    if (!ens || !st) throw Error{NLTH_EINVAL, "ens/st is NULL"};
    memset(st, 0, sizeof *st);
    st->steps_done = ens->steps_done;
    st->paged = ens->paged;
    st->ms_total = ens->ms_total;
    st->n_colors = ens->mesh->ncolor;
    // counters and timers summed over the member sets; the budget figures are
    // those after the last set was created
    for (const Ens* e = ens; e; e = e->twin.get()) {
        const int ns_steps = std::max(1, e->P.n_steps);
        std::vector<int> it((size_t)e->nm * ns_steps * 2);
        NLTH_HIP(hipMemcpy(it.data(), e->iters_dev.p, it.size() * 4, hipMemcpyDeviceToHost));
        for (size_t i = 0; i < it.size(); i += 2) {
            st->outer_iters += it[i];
            st->inner_iters += it[i + 1];
        }
        st->ms_ebe64 += e->pc_ebe64.ms;
        st->ms_ebe32 += e->pc_ebe32.ms;
        st->ms_vec += e->pc_vec.ms;
        st->ms_law += e->pc_law.ms;
        st->ms_other += e->pc_other.ms;
        st->n_ebe64 += e->pc_ebe64.n;
        st->n_ebe32 += e->pc_ebe32.n;
        st->n_law += e->pc_law.n;
        st->elems_ebe64 += e->pc_ebe64.elems;
        st->elems_ebe32 += e->pc_ebe32.elems;
        st->h2d_bytes += e->h2d_bytes;
        st->d2h_bytes += e->d2h_bytes;
        st->ms_copy += e->ms_copy;
        st->n_members += e->nm;
        st->members_padded += e->MB;
        st->device_bytes = e->dev_bytes;
        st->host_bytes = e->host_bytes;
        st->ms_gather32 += e->pc_gather32.ms;
        st->n_gather32 += e->pc_gather32.n;
        st->ms_tail32 += e->pc_tail32.ms;
        st->n_tail32 += e->pc_tail32.n;
        st->elems_tail32 += e->pc_tail32.elems;
    }
    st->member_sets = ens->twin ? 2 : 1;
    if (ens->cheb_bounds.p && ens->inner_method == 1) {
        std::vector<double> bd((size_t)2 * ens->MB);
        NLTH_HIP(hipMemcpy(bd.data(), ens->cheb_bounds.p, bd.size() * 8, hipMemcpyDeviceToHost));
        st->cheb_lo_min = 1e300;
        for (int m = 0; m < ens->nm; ++m) {
            st->cheb_lo_min = std::min(st->cheb_lo_min, bd[m]);
            st->cheb_hi_max = std::max(st->cheb_hi_max, bd[ens->MB + m]);
        }
    }
    API_END
}

int nlth_solve(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, nlth_result* res)
{
    nlth_ens* e = nullptr;
    int rc = nlth_ens_create(ctx, mesh, prob, &e);
    if (rc != NLTH_OK) return rc;
    int rs = nlth_ens_step(e, prob->n_steps);
    std::string msg = rs != NLTH_OK ? ctx->last_error : std::string();
    int rr = nlth_ens_read(e, res);
    nlth_ens_destroy(e);
    if (rs != NLTH_OK) {
        set_error(ctx, Error{rs, msg});
        return rs;
    }
    return rr;
}

int nlth_response_spectra(nlth_ctx* ctx, const double* vel, int32_t n_series, int32_t n_steps, double dt,
                          const double* periods, int32_t n_periods, double h, int32_t kind, double* out)
{
    API_BEGIN(ctx)
    if (!ctx || !vel || !periods || !out) throw Error{NLTH_EINVAL, "NULL argument"};
    if (n_series <= 0 || n_steps <= 0 || n_periods <= 0) throw Error{NLTH_EINVAL, "empty series, steps or periods"};
    if (!(dt > 0.0) || !(h >= 0.0 && h < 1.0)) throw Error{NLTH_EINVAL, "dt must be > 0 and h in [0, 1)"};
    if (kind != NLTH_SPEC_VELOCITY && kind != NLTH_SPEC_PSEUDO_VELOCITY)
        throw Error{NLTH_EINVAL, "kind must be NLTH_SPEC_VELOCITY or NLTH_SPEC_PSEUDO_VELOCITY"};
    for (int k = 0; k < n_periods; ++k)
        if (!(periods[k] > 0.0)) throw Error{NLTH_EINVAL, "periods must be > 0"};
    if (ctx->host_only) throw Error{NLTH_EDEVICE, "host-only context"};
    std::lock_guard<std::mutex> g(ctx->mu);
    NLTH_HIP(hipSetDevice(ctx->device));
    const size_t nv = (size_t)n_series * n_steps, no = (size_t)n_series * n_periods;
    DevBuf dv, dp, dout;
    dv.alloc(nullptr, nv * 8);
    dp.alloc(nullptr, (size_t)n_periods * 8);
    dout.alloc(nullptr, no * 8);
    hipStream_t s = ctx->stream;
    NLTH_HIP(hipMemcpyAsync(dv.p, vel, nv * 8, hipMemcpyHostToDevice, s));
    NLTH_HIP(hipMemcpyAsync(dp.p, periods, (size_t)n_periods * 8, hipMemcpyHostToDevice, s));
    launch_response_spectra(s, dv.as<double>(), n_series, n_steps, dt, dp.as<double>(), n_periods, h, kind,
                            dout.as<double>());
    NLTH_HIP(hipGetLastError());
    NLTH_HIP(hipMemcpyAsync(out, dout.p, no * 8, hipMemcpyDeviceToHost, s));
    NLTH_HIP(hipStreamSynchronize(s));
    return NLTH_OK;
    API_END
}

int nlth_apply_operator(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, int32_t which,
                        int32_t precision, const double* D_ip, const double* hh, const double* x, double* y)
{
    API_BEGIN(ctx)
    if (!ctx || !mesh || !prob || !D_ip || !x || !y) throw Error{NLTH_EINVAL, "NULL argument"};
    if (ctx->host_only) throw Error{NLTH_EDEVICE, "host-only context"};
    if (which < NLTH_OP_A || which > NLTH_OP_DIAG) throw Error{NLTH_EINVAL, "which must be NLTH_OP_A/K/M/DIAG"};
    if (precision == NLTH_MIXED && which != NLTH_OP_A && which != NLTH_OP_DIAG)
        throw Error{NLTH_EINVAL, "FP32 apply supports NLTH_OP_A and NLTH_OP_DIAG"};
    std::lock_guard<std::mutex> g(ctx->mu);
    NLTH_HIP(hipSetDevice(ctx->device));
    Problem P;
    nlth_problem p1 = *prob;
    p1.n_members = 1;
    p1.n_steps = 0;
    p1.precision = precision;  // allocates the inner operator's D storage for NLTH_MIXED
    if (precision == NLTH_MIXED) {
        if (!(p1.inner_tol > 0)) p1.inner_tol = 0.1;
        if (p1.inner_maxit <= 0) p1.inner_maxit = 1;
    }
    copy_problem(&p1, P);
    std::unique_ptr<nlth_ens> e(new nlth_ens());
    e->create(ctx, mesh, P);
    const int ne = mesh->ne, nn = mesh->nn;
    // D and h into the sorted, member-innermost layout (MB = 1)
    const int EB = e->EB;  // MB = 1
    std::vector<double> Dd((size_t)e->ne_pad * 84, 0.0), hd(ne, 0.0);
    for (int pos = 0; pos < ne; ++pos) {
        int e0 = mesh->order[pos];
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 21; ++k)
                Dd[((size_t)(pos / EB) * 84 + j * 21 + k) * EB + pos % EB] = D_ip[(size_t)e0 * 84 + j * 21 + k];
        if (hh) hd[pos] = hh[e0];
    }
    NLTH_HIP(hipMemcpy(e->D64.p, Dd.data(), Dd.size() * 8, hipMemcpyHostToDevice));
    if (e->D32.p) {
        std::vector<float> Df(Dd.begin(), Dd.end());
        NLTH_HIP(hipMemcpy(e->D32.p, Df.data(), Df.size() * 4, hipMemcpyHostToDevice));
    }
    if (e->D16.p) {  // bfloat16 pairs, round to nearest even on the FP32 bits
        auto bf = [](double x) {
            float f = (float)x;
            uint32_t u;
            memcpy(&u, &f, 4);
            return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
        };
        const bool mean = e->d16_mean;  // one D per element: the mean over its points
        std::vector<uint32_t> Dh((size_t)e->ne_pad * (mean ? 11 : 44), 0u);
        for (int pos = 0; pos < ne; ++pos) {
            const size_t base = (size_t)(pos / EB) * 84 * EB + pos % EB;
            if (mean) {
                double dmean[21];
                for (int k = 0; k < 21; ++k) {
                    dmean[k] = 0.0;
                    for (int j = 0; j < 4; ++j) dmean[k] += Dd[base + (size_t)(j * 21 + k) * EB];
                    dmean[k] *= 0.25;
                }
                for (int q = 0; q < 11; ++q) {
                    const uint32_t lo = bf(dmean[2 * q]), hi = (2 * q + 1 < 21) ? bf(dmean[2 * q + 1]) : 0u;
                    Dh[((size_t)(pos / EB) * 11 + q) * EB + pos % EB] = lo | (hi << 16);
                }
                continue;
            }
            for (int j = 0; j < 4; ++j)
                for (int q = 0; q < 11; ++q) {
                    const size_t src = base + (size_t)(j * 21) * EB;
                    const uint32_t lo = bf(Dd[src + (size_t)(2 * q) * EB]);
                    const uint32_t hi = (2 * q + 1 < 21) ? bf(Dd[src + (size_t)(2 * q + 1) * EB]) : 0u;
                    Dh[((size_t)(pos / EB) * 44 + j * 11 + q) * EB + pos % EB] = lo | (hi << 16);
                }
        }
        NLTH_HIP(hipMemcpy(e->D16.p, Dh.data(), Dh.size() * 4, hipMemcpyHostToDevice));
    }
    NLTH_HIP(hipMemcpy(e->h.p, hd.data(), hd.size() * 8, hipMemcpyHostToDevice));
    const long n = 3L * nn;
    int one = 1;
    NLTH_HIP(hipMemcpy(e->stepping.p, &one, 4, hipMemcpyHostToDevice));
    hipStream_t s = e->s;
    // x and y are in input node order; the library stores nodes in Morton order
    std::vector<double> xs(n), ys(n);
    for (int i = 0; i < nn; ++i)
        for (int c = 0; c < 3; ++c) xs[3L * mesh->node_new[i] + c] = x[3L * i + c];
    x = xs.data();
    double* y_user = y;
    y = ys.data();
    if (which == NLTH_OP_DIAG) {
        // the block-Jacobi preconditioner's 3x3 diagonal blocks applied to x
        e->build_diag();
        std::vector<double> dg((size_t)nn * 6);
        NLTH_HIP(hipStreamSynchronize(s));
        NLTH_HIP(hipMemcpy(dg.data(), e->diag.p, dg.size() * 8, hipMemcpyDeviceToHost));
        for (int i = 0; i < nn; ++i) {
            const double* b = &dg[(size_t)i * 6];  // 00 01 02 11 12 22
            const double* xv = x + 3L * i;
            y[3L * i] = b[0] * xv[0] + b[1] * xv[1] + b[2] * xv[2];
            y[3L * i + 1] = b[1] * xv[0] + b[3] * xv[1] + b[4] * xv[2];
            y[3L * i + 2] = b[2] * xv[0] + b[4] * xv[1] + b[5] * xv[2];
        }
    } else if (precision == NLTH_FP64) {
        NLTH_HIP(hipMemcpy(e->p.p, x, n * 8, hipMemcpyHostToDevice));
        launch_fill(s, e->Ap.as<double>(), 0.0, n);
        e->ebe((OpMode)which, e->p.as<double>(), nullptr, e->Ap.as<double>(), e->stepping.as<int>(), nullptr, 0.0,
               which == NLTH_OP_A ? 2.0 / P.dt : 0.0, nullptr, nullptr);
        NLTH_HIP(hipStreamSynchronize(s));
        NLTH_HIP(hipMemcpy(y, e->Ap.p, n * 8, hipMemcpyDeviceToHost));
    } else {
        std::vector<float> xf(x, x + n), yf(n);
        DevBuf xd, yd;
        xd.alloc(&ctx->budget, n * 4);
        yd.alloc(&ctx->budget, n * 4);
        NLTH_HIP(hipMemcpy(xd.p, xf.data(), n * 4, hipMemcpyHostToDevice));
        launch_fill32(s, yd.as<float>(), 0.0f, n);
        e->ebe32(xd.as<float>(), yd.as<float>(), e->stepping.as<int>());
        NLTH_HIP(hipStreamSynchronize(s));
        NLTH_HIP(hipMemcpy(yf.data(), yd.p, n * 4, hipMemcpyDeviceToHost));
        for (long i = 0; i < n; ++i) y[i] = yf[i];
    }
    for (int i = 0; i < nn; ++i)
        for (int c = 0; c < 3; ++c) y_user[3L * i + c] = ys[3L * mesh->node_new[i] + c];
    API_END
}

}  // extern "C"
