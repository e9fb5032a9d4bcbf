// Host runtime of libnlth: contexts, meshes, ensembles (the per-step driver),
// paging of the law state and the serving loop.  Internal to the library.
#pragma once

#include <atomic>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/nlth.h"
#include "nlth_impl.hpp"

namespace nlth {

struct Error {
    int code;
    std::string msg;
};

#define NLTH_HIP(expr)                                                                  \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::nlth::Error{NLTH_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
    } while (0)

// device allocation with a byte budget shared by a context
struct Budget {
    std::mutex mu;
    int64_t limit = 0, used = 0;
    int64_t host_limit = 0, host_used = 0;
};

struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    Budget* budget = nullptr;
    bool host = false;  // pinned host memory
    size_t base_off = 0;  // p = the allocation + base_off (device buffers are staggered)
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void alloc(Budget* b, size_t n, bool pinned_host = false);
    void release();
    template <typename T> T* as() const { return (T*)p; }
};

struct Ctx;

struct Mesh {
    Ctx* ctx = nullptr;
    int nn = 0, ne = 0, nf = 0, nrecv = 0, ncolor = 0, max_layer = 0;
    double volume = 0.0;
    // host copies / analysis
    std::vector<double> xyz;
    std::vector<int> node_new;     // input node -> storage node (Morton order)
    std::vector<int> order;        // storage position -> input tet (Morton order)
    std::vector<int> inv_order;    // input tet -> storage position
    std::vector<int> color_off;    // [ncolor+1] into color_elems
    std::vector<int> color_elems;  // storage positions grouped by colour
    std::vector<int> recv;
    // device
    DevBuf conn, geo64, geo32, layer, bn_node, bn_ptr, bn_face, bn_loc, f_node, f_M, f_n, f_layer, f_kind, recv_d;
    DevBuf inc_ptr, inc, celem, bn_of;
    DevBuf cl_off_d, cl_noff_d, cl_lconn_d, cn_ptr_d, cn_row_d;
    DevBuf order_d, node_new_d;    // storage position -> input tet; input node -> storage node
    int ncl = 0;
    long cl_rows = 0;  // total rows of the clusters' node lists
    int nbn = 0;
    mutable std::atomic<int> refs{0};  // pending requests using the mesh
    DevMesh dev() const;
};

struct Problem {  // host copy of an nlth_problem
    int nm = 0, nl = 0, ns = 0, n_steps = 0;
    std::vector<double> rho, vs, nu, gref, hmax, dirs, w, acc;
    std::vector<int> nonlinear;
    int damping_mode = 0;
    double h0 = 0, f_lo = 0.1, f_hi = 10, dt = 1e-3, cg_tol = 1e-8, inner_tol = 0.1;
    int cg_maxit = 1000, precision = 0, inner_maxit = 50, inner_dtype = 0;
    int depth = 1;  // reversal points the law remembers (1: the three-rule law)
};

struct ProfCat { double ms = 0; int64_t n = 0; int64_t elems = 0; };

struct Ens {
    Ctx* ctx = nullptr;
    const Mesh* mesh = nullptr;
    Problem P;
    int MB = 1, nm = 0, EB = 1, ne_pad = 0;  // EB: elements per layout block
    long ndof = 0;
    StepConst sc{};
    hipStream_t s = nullptr;
    // device state
    DevBuf mat, dirs, w, nonlinear, acc, vI_all, vI_cur;
    DevBuf u, v, a, q, du, b, r, z, p, Ap, diag, pinv, pinv32;
    DevBuf du2, du3;                    // increments of the two steps before the last (CG initial guess)
    int predictor = 0;                  // degree of the extrapolation of the increments giving x0 (0..2)
    DevBuf ir, iz, ip, iw, iAp;
    DevBuf lz, chebc, cheb_bounds, qb;  // inner CG coefficients, Chebyshev table and bounds, dashpot rows
    int inner_method = 0;               // 0: inner CG; 1: Chebyshev after one inner CG per step
    // convergence tail: with at most tail_max (16 or 32; 0 off) members still
    // active, the inner operator runs on their list only (tail_g lanes per element)
    int tail_max = 0, tail_g = 0;      // tail_max: 32 for mixed ensembles of 64..256 slots
    DevBuf tlist, tail_mem;             // [1 + MB] count then member indices; compact copies
    struct {                            // in tail_mem, G <= 32 lanes per row
        uint32_t* D;                    // element-mean D, element blocks of 64 / G
        double *h, *mat;
        float *pinv, *ir, *iz, *ip, *w, *Ap, *f;
    } tb{};
    int* h_tlist = nullptr;             // the list in the host mailbox
    int tail_count = 0;                 // listed members still iterating (profile counts)
    int count_flags() const;            // flags set at the last read_any_active
    // the same for the plain FP64 PCG: once at most tail_max members are still
    // iterating, their PCG moves to compact rows for the rest of the step
    int tail64_g = 0;
    DevBuf tail64_mem;
    struct {
        double *D, *h, *mat, *pinv, *x, *r, *z, *p, *Ap, *f;
    } tc{};
    bool enter_tail64();                // from h_flags: pack the listed members' rows
    void leave_tail64();                // their increment back to the full rows
    void tail64_iter();                 // one PCG iteration on the compact rows
    bool alloc_tail64();                // the FP64 compact rows (32 lanes), at first use
    // the mixed path's outer flexible CG moves to the same compact rows (the
    // inner tail's list) for the rest of the step
    bool outer_tail_ok = true;          // false once the compact rows could not be allocated
    bool outer_compact = false;
    bool enter_outer_tail();
    void update_tail();                 // from h_flags (the outer-active members just read)
    void tail_iter();                   // one inner CG iteration on the compact rows
    double cheb_lo = 1.0, cheb_hi = 1.05;  // scales of the Lanczos extreme eigenvalues of a step's first inner CG
    double cheb_est_scale = 1.1;           // scale of the random-start estimate of the largest eigenvalue
    int cheb_est_iters = 20, cheb_est_every = 32, cheb_est_age = -1;  // -1: no estimate yet
    int est_iters = 0;                  // estimate iterations of this step, not yet counted
    DevBuf D64, D32, D16, h;             // D16: bfloat16 pairs for the inner operator
    bool d16_mean = false;              // inner D: one bfloat16 D per element (the mean over its points)
    DevBuf fbuf;                        // element outputs of the gather path (FP64 or FP32)
    DevBuf cbuf;                        // cluster node rows of the cluster path (FP64 or FP32)
    int scatter = 0;                    // 0: element outputs + gather; 1: colour launches; 2: clusters + gather
    DevBuf theta;                       // resident law state (or the device chunk ring)
    DevBuf theta_host;                  // pinned host state when paged
    DevBuf hist, vmax, iters_dev;
    DevBuf partial, scal;               // CG scalars block
    DevBuf member_step, stepping, status;
    CgScalars cs{};
    // paging
    bool paged = false;
    bool zero_copy = false;             // paged state: the law kernel works on the pinned host copy directly
    int chunk_elems = 0, nchunks = 0, ring = 3;
    std::vector<long> chunk_off;        // byte offset of each chunk in theta_host
    std::vector<int> chunk_e0, chunk_ec, chunk_ecp;
    hipStream_t s_h2d = nullptr;        // transfers in; the write-backs run on the compute stream
    std::vector<hipEvent_t> ev_h2d, ev_d2h;
    hipEvent_t ev_zc = nullptr;         // end of the last zero-copy law pass (the copies wait for it)
    std::vector<int> slot_chunk;        // chunk currently held by each slot (-1 none)
    std::vector<bool> prefetched;
    // host bookkeeping
    std::vector<int> h_member_step, h_stepping, h_status;
    int steps_done = 0;
    int check_every = 8;
    // profiling
    bool profile = false;
    ProfCat pc_ebe64, pc_ebe32, pc_gather32, pc_vec, pc_law, pc_other, pc_tail32;
    std::vector<std::pair<std::pair<hipEvent_t, hipEvent_t>, ProfCat*>> pending;
    std::vector<hipEvent_t> ev_pool;
    double ms_total = 0, ms_copy = 0;
    int64_t outer_total = 0, inner_total = 0, h2d_bytes = 0, d2h_bytes = 0;
    int64_t dev_bytes = 0, host_bytes = 0;
    hipEvent_t ev_copy0 = nullptr, ev_copy1 = nullptr;

    // A paged ensemble runs as two member sets, each with its own compute
    // stream; the solve of one set runs while the law state of the other
    // streams over the host link.  `twin` is the second set (members
    // member_base.. of the caller's numbering); the transfer-in stream is shared.
    std::unique_ptr<Ens> twin;
    int member_base = 0;
    bool force_paged = false;           // page the law state even if it fits (a set of a pair)
    int64_t reserve_extra = 0;          // device bytes left for the second set when sizing the ring
    hipStream_t own_s = nullptr;        // compute stream of a second set (else the context's)
    bool shared_copy_streams = false;   // s_h2d belongs to the first set

    void create(Ctx* c, const Mesh* m, const Problem& p, int member_pad = 0);
    void destroy();
    ~Ens() { destroy(); }
    void step_all(int n_steps);        // lockstep members
    void step_pair(int n_steps);       // two member sets, alternating solves and law phases
    void step_begin();                  // member flags, then one step enqueued up to its receivers
    void step_end();                    // wait for the step, read the member status
    void one_step();                    // uses h_member_step / h_stepping
    void enqueue_step();                // one_step without the final wait
    void read_status();                 // wait for the stream; h_status from the device
    void read(nlth_result* res) const;
    // pieces
    void ebe(OpMode mode, const double* x1, const double* x2, double* y, const int* active, const double* base,
             double bscale, double dcoef, const double* vI, int* nblk);
    void ebe32(const float* x, float* y, const int* active, int* nblk = nullptr);
    void build_rhs();
    void build_diag();
    void solve_pcg();
    void solve_fcg();
    void inner_solve();                 // the preconditioner: z ~ A^-1 r
    void cheb_solve();
    void cheb_estimate();
    void cheb_body();
    void law_phase();
    void prefetch_next();
    // helpers
    void dots(int nd, const double* a0, const double* b0, const double* a1, const double* b1,
              const double* a2, const double* b2, int& nblk);
    int read_any_active(const int* flags);
    void inner_iter();
    void pcg_iter();
    void run_iters(int kind, int k);
    bool use_graph = true;
    // captured CG chunks, by (kind, compact-row width, iterations); the Chebyshev solve
    std::map<int, hipGraphExec_t> g_chunks;
    hipGraphExec_t g_cheb = nullptr;
    void clear_graphs();
    int ebe_block = 256;
    int cluster_blocks = 3;             // co-resident cluster blocks per CU
    void fin(FinalizeStage st, int nd, int nblk, double tol2, int maxit);
    void apply_A64(const double* x, double* y, const int* act, int* nblk = nullptr);
    // Host mailbox: pinned, device-mapped and coherent, written and read by
    // small copy kernels on the compute stream (not by the copy engines, which
    // a paged member set keeps busy with large transfers): per-member flags,
    // status, step index and stepping flag, then the tail list [1 + MB].
    int* h_mail = nullptr;
    int* d_mail = nullptr;              // device address of h_mail
    int* h_flags = nullptr;             // = h_mail: per-member flags just read
    hipEvent_t ev();
    void tstart(hipEvent_t& e0);
    void tstop(hipEvent_t e0, ProfCat* cat, int64_t elems);
    void collect_prof();
    void sync();
    // member slot management (serving)
    void reset_member(int m);
};

struct Request;

struct Ctx {
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    Budget budget;
    std::mutex mu;  // serialises API calls on the context
    int paging_sets = 2;  // member sets of a paged ensemble (1 or 2)
    std::string last_error;
    int log_level = 0;
    int max_batch = 64;
    std::atomic<int> live_meshes{0};
    // serving
    std::mutex smu;
    std::condition_variable scv;
    std::thread worker;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::map<uint64_t, std::shared_ptr<Request>> requests;
    std::deque<std::shared_ptr<Request>> queue;
    void ensure_worker();
    void worker_loop();
    ~Ctx();
};

struct Request {
    uint64_t ticket = 0;
    const Mesh* mesh = nullptr;
    Problem P;  // one member
    nlth_result res{};
    std::atomic<int> state{0};  // 0 queued, 1 running, 2 done, 3 cancelled
    std::atomic<int> cancel{0};
    int status = 0;
    int members_left = 0;  // guarded by the context's request lock
    int64_t host_bytes = 0;  // input copy charged to the host budget while queued
};

void serve_shutdown(Ctx* c);
// device address of the allocation-free entry point's scratch array on
// `device` (current), taken once per device
void scratch_setup(int device);
// least-squares Rayleigh fit of alpha/(4 pi f) + pi beta f to 1 over [f_lo, f_hi]
void rayleigh_coefficients(double f_lo, double f_hi, double* a, double* b);

void set_error(Ctx* c, const Error& e);
int64_t ensemble_bytes(const Mesh& m, const Problem& p, int MB, bool paged);
void copy_problem(const nlth_problem* in, Problem& out);
int pad_members(int nm);

}  // namespace nlth
