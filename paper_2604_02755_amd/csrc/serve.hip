// Continuous-batching request loop of libnlth.
//
// Requests (one or more members each) are admitted into member slots of a
// batch: an ensemble whose members share the mesh and every non-member
// parameter.  A worker thread steps each busy batch; at every step boundary
// finished members leave (their results are copied to the caller's buffers)
// and queued requests take the free slots, so requests that arrive while
// others run overlap with them in the same launches.  Members of a batch run
// at their own step index (their own input wave position); all per-member
// arithmetic is independent of the other slots' values, except that when few
// members of a batch of 64 or more slots are still iterating, they finish on
// compact rows (the same arithmetic, its sums in another order).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cstdio>

#include "runtime.hpp"

namespace nlth {

struct Slot {
    std::shared_ptr<Request> req;
    int member = -1;  // member index within the request
    int step = 0;
    int n_steps = 0;
};

// Host memory of the serving loop, charged against the context's host budget
// beside the pinned law state of paged ensembles: the input copy of every
// queued request (from submission until its members take slots) and each
// batch's own copy of its members' inputs.
static int64_t problem_host_bytes(const Problem& p)
{
    return (int64_t)(p.rho.size() + p.vs.size() + p.nu.size() + p.gref.size() + p.hmax.size() + p.dirs.size() +
                     p.w.size() + p.acc.size()) * 8 + (int64_t)p.nonlinear.size() * 4;
}

static bool host_charge(Budget& b, int64_t n, int64_t* used = nullptr)
{
    std::lock_guard<std::mutex> g(b.mu);
    if (used) *used = b.host_used;
    if (b.host_limit > 0 && b.host_used + n > b.host_limit) return false;
    b.host_used += n;
    return true;
}

static void host_uncharge(Budget& b, int64_t& n)
{
    if (n == 0) return;
    std::lock_guard<std::mutex> g(b.mu);
    b.host_used -= n;
    n = 0;
}

struct Batch {
    const Mesh* mesh = nullptr;
    Problem key;  // shared parameters (per-member arrays unused)
    std::unique_ptr<Ens> ens;
    std::vector<Slot> slots;
    int cap_steps = 0;
    Budget* budget = nullptr;  // host bytes of the batch's input copy, charged while it lives
    int64_t host_bytes = 0;
    ~Batch()
    {
        if (budget) host_uncharge(*budget, host_bytes);
    }
    int busy() const
    {
        int n = 0;
        for (auto& s : slots) n += s.req != nullptr;
        return n;
    }
    int free_slots() const { return (int)slots.size() - busy(); }
};

static bool same_shared(const Problem& a, const Problem& b)
{
    return a.nl == b.nl && a.ns == b.ns && a.dirs == b.dirs && a.w == b.w && a.hmax == b.hmax &&
           a.nonlinear == b.nonlinear && a.damping_mode == b.damping_mode && a.h0 == b.h0 && a.f_lo == b.f_lo &&
           a.f_hi == b.f_hi && a.dt == b.dt && a.cg_tol == b.cg_tol && a.cg_maxit == b.cg_maxit &&
           a.precision == b.precision && a.inner_tol == b.inner_tol && a.inner_maxit == b.inner_maxit &&
           a.inner_dtype == b.inner_dtype && a.depth == b.depth;
}

struct ServeState {
    std::vector<std::unique_ptr<Batch>> batches;
};

static std::mutex g_serve_mu;
static std::map<Ctx*, std::unique_ptr<ServeState>> g_serve;

static ServeState& serve_state(Ctx* c)
{
    std::lock_guard<std::mutex> g(g_serve_mu);
    auto& p = g_serve[c];
    if (!p) p.reset(new ServeState());
    return *p;
}

// a new request takes slot m of this ensemble: member inputs and a fresh state
void Ens::reset_member(int m)
{
    const int ns_steps = std::max(1, P.n_steps);
    const DevMesh dm = mesh->dev();
    // material column m
    std::vector<double> mt((size_t)P.nl * MAT_N * MB);
    NLTH_HIP(hipMemcpy(mt.data(), mat.p, mt.size() * 8, hipMemcpyDeviceToHost));
    for (int l = 0; l < P.nl; ++l) {
        const double rho = P.rho[(long)m * P.nl + l], vs = P.vs[(long)m * P.nl + l], nu = P.nu[(long)m * P.nl + l];
        const double G0 = rho * vs * vs, lam = 2.0 * G0 * nu / (1.0 - 2.0 * nu), hm = P.hmax[l];
        double* col = &mt[(size_t)l * MAT_N * MB];
        col[MAT_RHO * MB + m] = rho;
        col[MAT_G0 * MB + m] = G0;
        col[MAT_KB * MB + m] = lam + 2.0 * G0 / 3.0;
        col[MAT_VS * MB + m] = vs;
        col[MAT_VP * MB + m] = sqrt((lam + 2.0 * G0) / rho);
        col[MAT_GREF * MB + m] = P.gref[(long)m * P.nl + l];
        col[MAT_HMAX * MB + m] = hm;
        col[MAT_BETA * MB + m] = 2.0 * M_PI * hm / (2.0 - M_PI * hm);
    }
    NLTH_HIP(hipMemcpyAsync(mat.p, mt.data(), mt.size() * 8, hipMemcpyHostToDevice, s));
    // input wave of slot m, incident velocity by the trapezoid rule
    NLTH_HIP(hipMemcpyAsync(acc.as<double>() + (size_t)m * ns_steps * 3, P.acc.data() + (size_t)m * ns_steps * 3,
                            (size_t)ns_steps * 3 * 8, hipMemcpyHostToDevice, s));
    launch_incident_velocity(s, MB, 1, ns_steps, acc.as<double>() + (size_t)m * ns_steps * 3,
                             vI_all.as<double>() + (size_t)m * ns_steps * 3, P.dt);
    for (DevBuf* bb : {&u, &v, &a, &q, &du, &du2, &du3}) launch_zero_member(s, bb->as<double>(), ndof, MB, m);
    launch_fill(s, vmax.as<double>() + (size_t)m * std::max(1, mesh->nrecv), 0.0, std::max(1, mesh->nrecv));
    launch_theta_reset_member(s, theta.p, ne_pad, P.ns, MB, m);
    launch_law_init(s, dm, MB, nm, mat.as<double>(), P.nl, P.ns, dirs.as<double>(), w.as<double>(), D64.as<double>(),
                    D32.as<float>(), D16.as<uint32_t>(), h.as<double>(), m, d16_mean);
    int zero = 0;
    NLTH_HIP(hipMemcpyAsync(cs.status + m, &zero, 4, hipMemcpyHostToDevice, s));
    h_status[m] = 0;
    NLTH_HIP(hipStreamSynchronize(s));
}

void Ctx::ensure_worker()
{
    if (!worker.joinable()) worker = std::thread([this] { worker_loop(); });
}

// copy member slot m's results into its request's buffers
static void copy_out(Ens& E, int m, Slot& sl)
{
    Request& R = *sl.req;
    const int nr = std::max(1, E.mesh->nrecv);
    const int cap = std::max(1, E.P.n_steps);
    const int rm = sl.member, ns = sl.n_steps;
    if (R.res.vel && E.mesh->nrecv > 0 && ns > 0)
        NLTH_HIP(hipMemcpy(R.res.vel + (size_t)rm * ns * nr * 3, E.hist.as<double>() + (size_t)m * cap * nr * 3,
                           (size_t)ns * nr * 3 * 8, hipMemcpyDeviceToHost));
    if (R.res.iters && ns > 0)
        NLTH_HIP(hipMemcpy(R.res.iters + (size_t)rm * ns * 2, E.iters_dev.as<int>() + (size_t)m * cap * 2,
                           (size_t)ns * 2 * 4, hipMemcpyDeviceToHost));
    if (R.res.vmax && E.mesh->nrecv > 0)
        NLTH_HIP(hipMemcpy(R.res.vmax + (size_t)rm * nr, E.vmax.as<double>() + (size_t)m * nr, (size_t)nr * 8,
                           hipMemcpyDeviceToHost));
    if (R.res.member_status) R.res.member_status[rm] = E.h_status[m];
}

void Ctx::worker_loop()
{
    (void)hipSetDevice(device);
    ServeState& S = serve_state(this);
    for (;;) {
        // ---- admission (under the request lock)
        {
            std::unique_lock<std::mutex> lk(smu);
            scv.wait(lk, [&] {
                if (stop) return true;
                if (!queue.empty()) return true;
                for (auto& b : S.batches)
                    if (b->busy()) return true;
                return false;
            });
            if (stop) break;
            std::deque<std::shared_ptr<Request>> keep;
            while (!queue.empty()) {
                auto r = queue.front();
                queue.pop_front();
                if (r->cancel.load()) {
                    host_uncharge(budget, r->host_bytes);
                    r->status = NLTH_ECANCELED;
                    r->state = 3;
                    r->mesh->refs--;
                    scv.notify_all();
                    continue;
                }
                const int need = r->P.nm;
                Batch* target = nullptr;
                for (auto& b : S.batches)
                    if (b->mesh == r->mesh && same_shared(b->key, r->P) && r->P.n_steps <= b->cap_steps &&
                        b->free_slots() >= need) {
                        target = b.get();
                        break;
                    }
                if (!target) {
                    // a new batch sized for the members now waiting for this mesh and
                    // these shared parameters (a step costs the same for every slot,
                    // busy or not), halved until it fits the budget
                    std::unique_ptr<Batch> nb(new Batch());
                    nb->mesh = r->mesh;
                    nb->key = r->P;
                    nb->cap_steps = std::max(r->P.n_steps, 2048);
                    int waiting = need;
                    for (auto& q : queue)
                        if (q->mesh == r->mesh && same_shared(q->P, r->P) && !q->cancel.load()) waiting += q->P.nm;
                    int slots = 1;
                    while (slots < std::min(waiting, max_batch)) slots *= 2;
                    slots = std::max(slots, need);
                    bool made = false;
                    std::string why;
                    int why_code = NLTH_ENOMEM_DEVICE;
                    while (!made && slots >= need) {
                        Problem tp = r->P;
                        tp.nm = slots;
                        tp.n_steps = nb->cap_steps;
                        tp.rho.assign((size_t)slots * tp.nl, r->P.rho[0]);
                        tp.vs.assign((size_t)slots * tp.nl, r->P.vs[0]);
                        tp.nu.assign((size_t)slots * tp.nl, r->P.nu[0]);
                        tp.gref.assign((size_t)slots * tp.nl, r->P.gref[0]);
                        for (int k = 0; k < slots; ++k)
                            for (int l = 0; l < tp.nl; ++l) {
                                tp.rho[(size_t)k * tp.nl + l] = r->P.rho[l];
                                tp.vs[(size_t)k * tp.nl + l] = r->P.vs[l];
                                tp.nu[(size_t)k * tp.nl + l] = r->P.nu[l];
                                tp.gref[(size_t)k * tp.nl + l] = r->P.gref[l];
                            }
                        tp.acc.assign((size_t)slots * tp.n_steps * 3, 0.0);
                        int64_t hb = problem_host_bytes(tp);
                        if (!host_charge(budget, hb)) {
                            char buf[160];
                            snprintf(buf, sizeof buf, "host budget: a batch of %d slots needs %.3f MB of inputs",
                                     slots, hb / 1e6);
                            why = buf;
                            why_code = NLTH_ENOMEM_HOST;
                            slots /= 2;
                            continue;
                        }
                        try {
                            std::lock_guard<std::mutex> g(mu);
                            std::unique_ptr<Ens> e(new Ens());
                            e->create(this, r->mesh, tp, pad_members(slots));
                            if (e->paged) throw Error{NLTH_ENOMEM_DEVICE, "serving batches keep their state resident"};
                            e->predictor = 2;  // fewer iterations per step; same results within tol
                            nb->ens = std::move(e);
                            nb->budget = &budget;
                            nb->host_bytes = hb;
                            made = true;
                        } catch (const Error& err) {
                            host_uncharge(budget, hb);
                            why = err.msg;
                            why_code = err.code == NLTH_ENOMEM_HOST ? NLTH_ENOMEM_HOST : NLTH_ENOMEM_DEVICE;
                            slots /= 2;
                        }
                    }
                    if (!made) {
                        bool busy = false;
                        for (auto& b : S.batches) busy |= b->busy() > 0;
                        if (busy) {  // wait for running batches to free memory
                            keep.push_back(r);
                        } else {     // nothing else holds memory: it cannot run
                            host_uncharge(budget, r->host_bytes);
                            r->status = why_code;
                            r->state = 2;
                            r->mesh->refs--;
                            set_error(this, Error{why_code, why});
                            scv.notify_all();
                        }
                        continue;
                    }
                    nb->slots.resize(nb->ens->nm);
                    S.batches.push_back(std::move(nb));
                    target = S.batches.back().get();
                }
                // place the request's members
                std::lock_guard<std::mutex> g(mu);
                Ens& E = *target->ens;
                int placed = 0;
                for (int m = 0; m < (int)target->slots.size() && placed < need; ++m) {
                    if (target->slots[m].req) continue;
                    for (int l = 0; l < E.P.nl; ++l) {
                        E.P.rho[(size_t)m * E.P.nl + l] = r->P.rho[(size_t)placed * r->P.nl + l];
                        E.P.vs[(size_t)m * E.P.nl + l] = r->P.vs[(size_t)placed * r->P.nl + l];
                        E.P.nu[(size_t)m * E.P.nl + l] = r->P.nu[(size_t)placed * r->P.nl + l];
                        E.P.gref[(size_t)m * E.P.nl + l] = r->P.gref[(size_t)placed * r->P.nl + l];
                    }
                    const int cap = std::max(1, E.P.n_steps);
                    std::fill(E.P.acc.begin() + (size_t)m * cap * 3, E.P.acc.begin() + (size_t)(m + 1) * cap * 3, 0.0);
                    std::copy(r->P.acc.begin() + (size_t)placed * r->P.n_steps * 3,
                              r->P.acc.begin() + (size_t)(placed + 1) * r->P.n_steps * 3,
                              E.P.acc.begin() + (size_t)m * cap * 3);
                    try {
                        E.reset_member(m);
                    } catch (const Error& err) {
                        set_error(this, err);
                    }
                    target->slots[m].req = r;
                    target->slots[m].member = placed;
                    target->slots[m].step = 0;
                    target->slots[m].n_steps = r->P.n_steps;
                    ++placed;
                }
                r->state = 1;
                std::vector<double>().swap(r->P.acc);  // the batch holds its own copy
                host_uncharge(budget, r->host_bytes);
            }
            for (auto& r : keep) queue.push_back(r);
        }

        // ---- one step of every busy batch
        bool any = false;
        for (auto& bp : S.batches) {
            Batch& B = *bp;
            if (!B.busy()) continue;
            any = true;
            Ens& E = *B.ens;
            std::lock_guard<std::mutex> g(mu);
            for (int m = 0; m < E.MB; ++m) {
                Slot* sl = m < (int)B.slots.size() ? &B.slots[m] : nullptr;
                const bool run = sl && sl->req && !sl->req->cancel.load() && sl->step < sl->n_steps &&
                                 E.h_status[m] == 0;
                E.h_member_step[m] = sl ? sl->step : 0;
                E.h_stepping[m] = run ? 1 : 0;
            }
            try {
                E.one_step();
            } catch (const Error& err) {
                set_error(this, err);
            }
            for (int m = 0; m < (int)B.slots.size(); ++m) {
                Slot& sl = B.slots[m];
                if (!sl.req) continue;
                if (E.h_stepping[m]) sl.step++;
                const bool cancelled = sl.req->cancel.load();
                const bool failed = E.h_status[m] != 0;
                if (sl.step >= sl.n_steps || cancelled || failed) {
                    if (!cancelled) {
                        try {
                            copy_out(E, m, sl);
                        } catch (const Error& err) {
                            set_error(this, err);
                        }
                    }
                    std::shared_ptr<Request> r = sl.req;
                    sl.req.reset();
                    std::lock_guard<std::mutex> lk(smu);
                    if (failed) r->status = NLTH_ENOCONV;
                    if (cancelled) r->status = NLTH_ECANCELED;
                    if (--r->members_left == 0) {
                        r->state = cancelled ? 3 : 2;
                        r->mesh->refs--;
                        scv.notify_all();
                    }
                }
            }
        }
        // release idle batches so their memory serves waiting requests
        {
            std::lock_guard<std::mutex> lk(smu);
            for (size_t i = 0; i < S.batches.size();) {
                if (!S.batches[i]->busy()) {
                    std::lock_guard<std::mutex> g(mu);
                    S.batches.erase(S.batches.begin() + i);
                } else {
                    ++i;
                }
            }
        }
        (void)any;
    }
    std::lock_guard<std::mutex> g(mu);
    S.batches.clear();
}

void serve_shutdown(Ctx* c)
{
    std::lock_guard<std::mutex> g(g_serve_mu);
    g_serve.erase(c);
}

}  // namespace nlth

using namespace nlth;

struct nlth_ctx : Ctx {};
struct nlth_mesh : Mesh {};

extern "C" {

int nlth_submit(nlth_ctx* ctx, const nlth_mesh* mesh, const nlth_problem* prob, nlth_result* res, uint64_t* ticket)
{
    try {
        if (!ctx || !mesh || !prob || !res || !ticket) throw Error{NLTH_EINVAL, "NULL argument"};
        if (ctx->host_only) throw Error{NLTH_EDEVICE, "host-only context"};
        if (mesh->ctx != ctx) throw Error{NLTH_EINVAL, "mesh belongs to another context"};
        auto r = std::make_shared<Request>();
        copy_problem(prob, r->P);
        if (r->P.nl <= mesh->max_layer) throw Error{NLTH_EINVAL, "problem: mesh uses a layer id >= n_layers"};
        if (r->P.n_steps <= 0) throw Error{NLTH_EINVAL, "problem: n_steps must be positive for a request"};
        // can a batch holding just this request ever fit the device budget?
        const int64_t need = ensemble_bytes(*mesh, r->P, pad_members(r->P.nm), false);
        if (ctx->budget.limit > 0 && need > ctx->budget.limit) {
            char buf[160];
            snprintf(buf, sizeof buf, "request needs %.2f GB of device memory, budget is %.2f GB", need / 1e9,
                     ctx->budget.limit / 1e9);
            throw Error{NLTH_EBUSY, buf};
        }
        // the host budget must hold the request's input copy until its members
        // take slots (and can it ever hold it?)
        const int64_t hb = problem_host_bytes(r->P);
        if (ctx->budget.host_limit > 0 && hb > ctx->budget.host_limit) {
            char buf[160];
            snprintf(buf, sizeof buf, "request inputs need %.3f MB of host memory, host budget is %.3f MB", hb / 1e6,
                     ctx->budget.host_limit / 1e6);
            throw Error{NLTH_EBUSY, buf};
        }
        int64_t held = 0;
        if (!host_charge(ctx->budget, hb, &held)) {
            char buf[200];
            snprintf(buf, sizeof buf,
                     "host budget: queued requests, batches and paged state hold %.3f of %.3f MB; "
                     "this request needs %.3f MB (submit again when requests finish)",
                     held / 1e6, ctx->budget.host_limit / 1e6, hb / 1e6);
            throw Error{NLTH_EBUSY, buf};
        }
        r->host_bytes = hb;
        r->mesh = mesh;
        r->res = *res;
        r->members_left = r->P.nm;
        {
            std::lock_guard<std::mutex> g(ctx->smu);
            r->ticket = ctx->next_ticket++;
            ctx->requests[r->ticket] = r;
            ctx->queue.push_back(r);
            const_cast<nlth_mesh*>(mesh)->refs++;
            *ticket = r->ticket;
            ctx->ensure_worker();
        }
        ctx->scv.notify_all();
        return NLTH_OK;
    } catch (const Error& e) {
        set_error(ctx, e);
        return e.code;
    }
}

int nlth_poll(nlth_ctx* ctx, uint64_t ticket, int32_t* done)
{
    if (!ctx || !done) return NLTH_EINVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) {
        set_error(ctx, Error{NLTH_ENOTFOUND, "unknown ticket"});
        return NLTH_ENOTFOUND;
    }
    const int st = it->second->state.load();
    *done = st >= 2;
    return st >= 2 ? it->second->status : NLTH_OK;
}

int nlth_wait(nlth_ctx* ctx, uint64_t ticket, double timeout_s)
{
    if (!ctx) return NLTH_EINVAL;
    std::unique_lock<std::mutex> lk(ctx->smu);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) {
        set_error(ctx, Error{NLTH_ENOTFOUND, "unknown ticket"});
        return NLTH_ENOTFOUND;
    }
    std::shared_ptr<Request> r = it->second;
    auto pred = [&] { return r->state.load() >= 2; };
    if (timeout_s < 0) ctx->scv.wait(lk, pred);
    else if (!ctx->scv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
        set_error(ctx, Error{NLTH_ETIMEDOUT, "request still running"});
        return NLTH_ETIMEDOUT;
    }
    return r->status;
}

int nlth_cancel(nlth_ctx* ctx, uint64_t ticket)
{
    if (!ctx) return NLTH_EINVAL;
    {
        std::lock_guard<std::mutex> g(ctx->smu);
        auto it = ctx->requests.find(ticket);
        if (it == ctx->requests.end()) {
            set_error(ctx, Error{NLTH_ENOTFOUND, "unknown ticket"});
            return NLTH_ENOTFOUND;
        }
        it->second->cancel = 1;
    }
    ctx->scv.notify_all();
    return NLTH_OK;
}

int nlth_release(nlth_ctx* ctx, uint64_t ticket)
{
    if (!ctx) return NLTH_EINVAL;
    std::lock_guard<std::mutex> g(ctx->smu);
    auto it = ctx->requests.find(ticket);
    if (it == ctx->requests.end()) {
        set_error(ctx, Error{NLTH_ENOTFOUND, "unknown ticket"});
        return NLTH_ENOTFOUND;
    }
    if (it->second->state.load() < 2) {
        set_error(ctx, Error{NLTH_EBUSY, "request still queued or running"});
        return NLTH_EBUSY;
    }
    ctx->requests.erase(it);
    return NLTH_OK;
}

}  // extern "C"
