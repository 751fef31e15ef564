// serve.cpp -- the request-serving runtime of hmm_serve.h.
//
// One worker thread per server.  Each pass of its loop
//   1. retires launches whose host callback has run (it is enqueued on the
//      launch's stream after the download and only sets a flag): copies every
//      request's path out of the pinned staging area into the caller's
//      buffer, records the completion and returns the launch's device and
//      host blocks to their pools;
//   2. while a launch slot (stream) is free, forms a batch from the oldest
//      pending request allowed to start and the pending requests of the same
//      model, kind and length class behind it (up to max_batch, as long as
//      the batch's bytes fit the free device budget and staging area),
//      uploads it, enqueues the decode and the download on the slot's stream
//      and records the slot's event;
//   3. sleeps until a submission arrives or, with launches in flight, for a
//      few microseconds.
// Device and pinned memory come from two areas allocated at creation and
// carved by a first-fit allocator, so the serving loop never allocates
// device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <atomic>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "hmm_gpu.h"
#include "hmm_internal.hpp"
#include "hmm_serve.h"

namespace {

using hmmk::fail_status;

size_t a256(size_t n) { return (n + 255) & ~(size_t)255; }

double now_s() {
    static const auto t0 = std::chrono::steady_clock::now();
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// first-fit allocator over [0, cap) with 256-byte granularity
struct Pool {
    size_t cap = 0, used = 0, peak = 0;
    std::map<size_t, size_t> free_;   // offset -> length
    void init(size_t c) {
        cap = c & ~(size_t)255;
        free_.clear();
        if (cap) free_[0] = cap;
        used = peak = 0;
    }
    bool alloc(size_t n, size_t *off) {
        n = a256(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < n) continue;
            const size_t o = it->first, rem = it->second - n;
            free_.erase(it);
            if (rem) free_[o + n] = rem;
            *off = o;
            used += n;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t n) {
        n = a256(n);
        used -= n;
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t largest() const {
        size_t m = 0;
        for (auto &f : free_) m = std::max(m, f.second);
        return m;
    }
};

struct Model {
    hmm_model m;          // resident device copies
    double *buf = nullptr;
    int D = 1;            // observation values per step
};

struct Req {
    uint64_t id;
    int model, kind;
    int64_t T;
    std::vector<char> obs;   // T * D values of the server's observation type
    int32_t *path_out;
    double t_submit;
};

// byte layout of one launch; the first four regions are mirrored in the
// pinned staging block so that one copy moves offsets + observations up and
// one moves paths + log-probabilities down
struct Layout {
    size_t off_b = 0, obs_b = 0, path_b = 0, logp_b = 0, ws_b = 0;
    size_t o_obs = 0, o_path = 0, o_logp = 0, o_ws = 0, dev_total = 0, host_total = 0;
    void finish() {
        o_obs = a256(off_b);
        o_path = o_obs + a256(obs_b);
        o_logp = o_path + a256(path_b);
        host_total = o_logp + a256(logp_b);
        o_ws = host_total;
        dev_total = o_ws + a256(ws_b);
    }
};

struct Flight {
    int slot = 0, cls = 0;
    Model md;                         // the resident model (copied: the list may grow)
    std::atomic<bool> ready{false};   // set by the stream's host callback after the download
    std::vector<Req> reqs;
    std::vector<int64_t> h_off;
    Layout lay;
    size_t dev_off = 0, host_off = 0;
    double t_launch = 0;
    hmm_status launch_status = HMM_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    bool busy = false;
    bool long_launch = false;   // holds requests of the longest length class
};

// Length class of a request: a launch lasts as long as its longest
// sequence, so requests are batched only with others of their class, and
// launches holding long requests may occupy at most half of the slots (a
// short request then always finds a slot within one short launch's time).
int len_class(int64_t T) { return T < 2048 ? 0 : (T < 16384 ? 1 : 2); }

}  // namespace

// Locking: `mu` guards the request queue, the completion queue, the
// counters and the wake-up state shared with submitters, pollers and the
// stream callbacks.  The pools, slots and launches in flight belong to the
// worker alone, and the worker never holds `mu` across a HIP call, so a
// callback (which takes `mu` briefly) can never wait on a HIP call.
struct hmm_server {
    hmm_server_opts opts;
    char *dev = nullptr;     // device budget area
    char *host = nullptr;    // pinned staging area
    size_t es = 4;           // bytes per observation value
    // worker-owned
    Pool dpool, hpool;
    std::vector<Slot> slots;
    std::list<Flight> flights;   // stable addresses: host callbacks point at them
    // shared, under mu
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::vector<Model> models;
    std::deque<Req> pending;
    std::deque<hmm_completion> done;
    std::thread worker;
    bool stop = false, wake = false;
    uint64_t next_id = 1, submits = 0;
    int64_t n_submitted = 0, n_completed = 0, n_launches = 0, n_in_flight = 0;
    size_t pool_used = 0, pool_peak = 0;

    struct CbArg {
        hmm_server *s;
        Flight *f;
    };
    static void on_done(void *p) {
        CbArg *a = (CbArg *)p;
        a->f->ready.store(true, std::memory_order_release);
        {
            std::lock_guard<std::mutex> lk(a->s->mu);
            a->s->wake = true;
        }
        a->s->cv_work.notify_one();
        delete a;
    }

    hmm_status plan(const Model &md, int kind, const std::vector<int64_t> &h_off, Layout *lay);
    bool select(Flight *f);
    void issue(Flight *f);
    void retire(Flight &f);
    void run();
};

namespace {

hmm_status server_fail(hmm_status st, const char *msg) { return fail_status(st, "%s", msg); }

}  // namespace

hmm_status hmm_server::plan(const Model &md, int kind, const std::vector<int64_t> &h_off,
                            Layout *lay) {
    const int64_t B = (int64_t)h_off.size() - 1, total = h_off.back();
    // sizing only: the planner reads the host offsets; device pointers are
    // placeholders that are never dereferenced
    hmm_batch b{B, (const int64_t *)dev, h_off.data(), dev, opts.precision == HMM_PREC_F64, 0};
    size_t ws = 0;
    const hmm_op op = kind == HMM_REQ_VITERBI ? HMM_OP_VITERBI : HMM_OP_POSTERIOR_DECODE;
    hmm_status st = hmm_workspace_size(op, &md.m, &b, (hmm_precision)opts.precision, &ws);
    if (st != HMM_OK) return st;
    lay->off_b = (size_t)(B + 1) * 8;
    lay->obs_b = (size_t)total * md.D * es;
    lay->path_b = (size_t)total * 4;
    lay->logp_b = (size_t)B * 8;
    lay->ws_b = ws;
    lay->finish();
    return HMM_OK;
}

// Worker: pick the next batch (called with mu held).  Returns false when no
// slot is free or nothing can start now.  A request that no launch can serve
// comes back as a one-request flight with launch_status set.
bool hmm_server::select(Flight *f) {
    int slot = -1, long_busy = 0;
    for (size_t i = 0; i < slots.size(); ++i) {
        if (!slots[i].busy && slot < 0) slot = (int)i;
        if (slots[i].busy && slots[i].long_launch) ++long_busy;
    }
    if (slot < 0 || pending.empty()) return false;
    const int long_cap = std::max(1, (int)slots.size() / 2);
    // the oldest request whose class may start now sets the batch key
    const size_t window = std::min<size_t>(pending.size(), 1024);
    size_t head = window;
    for (size_t i = 0; i < window; ++i)
        if (len_class(pending[i].T) < 2 || long_busy < long_cap) {
            head = i;
            break;
        }
    if (head == window) return false;
    const int model = pending[head].model, kind = pending[head].kind;
    const int cls = len_class(pending[head].T);
    const Model &md = models[(size_t)model];
    std::vector<size_t> pick;
    std::vector<int64_t> h_off{0};
    Layout lay;
    const size_t dfree = dpool.largest(), hfree = hpool.largest();
    for (size_t i = head; i < window && (int)pick.size() < opts.max_batch; ++i) {
        const Req &r = pending[i];
        if (r.model != model || r.kind != kind || len_class(r.T) != cls) continue;
        std::vector<int64_t> trial = h_off;
        trial.push_back(trial.back() + r.T);
        Layout l;
        const hmm_status st = plan(md, kind, trial, &l);
        if (st != HMM_OK) {
            if (!pick.empty()) break;
            f->reqs.push_back(std::move(pending[i]));
            pending.erase(pending.begin() + (std::ptrdiff_t)i);
            f->h_off = {0, f->reqs[0].T};
            f->launch_status = st;
            f->slot = -1;
            return true;
        }
        if (l.dev_total > dfree || l.host_total > hfree) break;
        pick.push_back(i);
        h_off.swap(trial);
        lay = l;
    }
    if (pick.empty()) return false;   // wait for memory to free up
    f->slot = slot;
    f->cls = cls;
    f->md = md;
    f->h_off = h_off;
    f->lay = lay;
    f->reqs.resize(pick.size());
    for (size_t k = pick.size(); k-- > 0;) {   // back to front keeps indices valid
        f->reqs[k] = std::move(pending[pick[k]]);
        pending.erase(pending.begin() + (std::ptrdiff_t)pick[k]);
    }
    dpool.alloc(lay.dev_total, &f->dev_off);
    hpool.alloc(lay.host_total, &f->host_off);
    slots[(size_t)slot].busy = true;
    slots[(size_t)slot].long_launch = cls == 2;
    pool_used = dpool.used;
    pool_peak = dpool.peak;
    ++n_launches;
    ++n_in_flight;
    return true;
}

// Worker, without mu: upload, decode, download, then the completion callback.
void hmm_server::issue(Flight *f) {
    const Layout &lay = f->lay;
    const Model &md = f->md;
    const int kind = f->reqs[0].kind;
    char *hb = host + f->host_off;
    char *db = dev + f->dev_off;
    std::memcpy(hb, f->h_off.data(), lay.off_b);
    for (size_t k = 0; k < f->reqs.size(); ++k)
        std::memcpy(hb + lay.o_obs + (size_t)f->h_off[k] * md.D * es, f->reqs[k].obs.data(),
                    f->reqs[k].obs.size());
    hipStream_t s = slots[(size_t)f->slot].stream;
    hmm_status st = HMM_OK;
    if (hipMemcpyAsync(db, hb, lay.o_path, hipMemcpyHostToDevice, s) != hipSuccess)
        st = HMM_ERR_DEVICE;
    const int64_t B = (int64_t)f->reqs.size();
    hmm_batch b{B, (const int64_t *)db, f->h_off.data(), db + lay.o_obs,
                opts.precision == HMM_PREC_F64, 0};
    int32_t *path = (int32_t *)(db + lay.o_path);
    double *logp = (double *)(db + lay.o_logp);
    if (st == HMM_OK) {
        if (kind == HMM_REQ_VITERBI)
            st = hmm_viterbi(&md.m, &b, (hmm_precision)opts.precision, path, logp, nullptr,
                             db + lay.o_ws, lay.ws_b, s);
        else
            st = hmm_posterior_decode(&md.m, &b, (hmm_precision)opts.precision, path, logp,
                                      db + lay.o_ws, lay.ws_b, s);
    }
    if (st == HMM_OK &&
        hipMemcpyAsync(hb + lay.o_path, db + lay.o_path, lay.host_total - lay.o_path,
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        st = HMM_ERR_DEVICE;
    f->launch_status = st;
    f->t_launch = now_s();
    if (hipLaunchHostFunc(s, &hmm_server::on_done, new CbArg{this, f}) != hipSuccess) {
        hipStreamSynchronize(s);   // no callback: finish the launch here
        f->ready.store(true, std::memory_order_release);
    }
}

// Worker, without mu: paths into the callers' buffers, then the records.
void hmm_server::retire(Flight &f) {
    const char *hb = host + f.host_off;
    const double *lp = (const double *)(hb + f.lay.o_logp);
    std::vector<hmm_completion> out(f.reqs.size());
    for (size_t k = 0; k < f.reqs.size(); ++k) {
        Req &r = f.reqs[k];
        hmm_completion &c = out[k];
        c = hmm_completion{};
        c.id = r.id;
        c.model = r.model;
        c.kind = r.kind;
        c.batch_size = (int32_t)f.reqs.size();
        c.T = r.T;
        c.t_submit = r.t_submit;
        c.t_launch = f.t_launch;
        if (f.launch_status != HMM_OK) {
            c.status = -(int32_t)f.launch_status;
            c.logp = std::nan("");
        } else {
            std::memcpy(r.path_out, hb + f.lay.o_path + (size_t)f.h_off[k] * 4, (size_t)r.T * 4);
            c.logp = lp[k];
            c.status = std::isnan(c.logp) ? 2 : (std::isinf(c.logp) && c.logp < 0 ? 1 : 0);
        }
        c.t_done = now_s();
    }
    if (f.slot >= 0) {
        dpool.release(f.dev_off, f.lay.dev_total);
        hpool.release(f.host_off, f.lay.host_total);
        slots[(size_t)f.slot].busy = false;
        slots[(size_t)f.slot].long_launch = false;
    }
    {
        std::lock_guard<std::mutex> lk(mu);
        for (auto &c : out) done.push_back(c);
        n_completed += (int64_t)out.size();
        if (f.slot >= 0) --n_in_flight;
        pool_used = dpool.used;
    }
    cv_done.notify_all();
}

void hmm_server::run() {
    hipSetDevice(opts.device);
    uint64_t seen = 0;
    for (;;) {
        for (auto it = flights.begin(); it != flights.end();) {
            if (it->ready.load(std::memory_order_acquire)) {
                retire(*it);
                it = flights.erase(it);
            } else {
                ++it;
            }
        }
        bool quit = false;
        for (;;) {
            flights.emplace_back();
            Flight *f = &flights.back();
            bool got;
            {
                std::lock_guard<std::mutex> lk(mu);
                quit = stop;
                seen = submits;
                got = !stop && select(f);
            }
            if (!got) {
                flights.pop_back();
                break;
            }
            if (f->slot < 0) {   // refused request: report at once
                retire(*f);
                flights.pop_back();
                continue;
            }
            issue(f);
        }
        bool any_ready = false;
        for (auto &f : flights) any_ready |= f.ready.load(std::memory_order_acquire);
        if (any_ready) continue;
        std::unique_lock<std::mutex> lk(mu);
        if ((quit || stop) && flights.empty()) break;
        // woken by a finished launch, a submission, or destroy
        cv_work.wait(lk, [&] {
            return wake || (stop ? flights.empty() : submits != seen);
        });
        wake = false;
    }
}

extern "C" {

void hmm_server_default_opts(hmm_server_opts *o) {
    if (!o) return;
    o->hbm_budget = (size_t)16 << 30;
    o->host_staging = (size_t)256 << 20;
    o->max_batch = 64;
    o->n_streams = 4;
    o->precision = HMM_PREC_F32;
    o->device = 0;
}

double hmm_server_now(void) { return now_s(); }

hmm_status hmm_server_create(const hmm_server_opts *opts, hmm_server **out) {
    if (!opts || !out) return server_fail(HMM_ERR_ARG, "opts / out is NULL");
    if (opts->max_batch < 1) return server_fail(HMM_ERR_ARG, "max_batch must be >= 1");
    if (opts->n_streams < 1 || opts->n_streams > 16)
        return server_fail(HMM_ERR_ARG, "n_streams must be in 1 .. 16");
    if (opts->precision != HMM_PREC_F32 && opts->precision != HMM_PREC_F64)
        return server_fail(HMM_ERR_ARG, "precision must be HMM_PREC_F32 or HMM_PREC_F64");
    if (opts->hbm_budget < 4096 || opts->host_staging < 4096)
        return server_fail(HMM_ERR_ARG, "budget and staging must be at least 4 KiB");
    *out = nullptr;
    if (hipSetDevice(opts->device) != hipSuccess)
        return server_fail(HMM_ERR_DEVICE, "hipSetDevice failed");
    hmm_server *s = new hmm_server();
    s->opts = *opts;
    s->es = opts->precision == HMM_PREC_F64 ? 8 : 4;
    if (hipMalloc((void **)&s->dev, opts->hbm_budget) != hipSuccess) {
        delete s;
        return server_fail(HMM_ERR_DEVICE, "device budget allocation failed");
    }
    if (hipHostMalloc((void **)&s->host, opts->host_staging, hipHostMallocDefault) != hipSuccess) {
        hipFree(s->dev);
        delete s;
        return server_fail(HMM_ERR_DEVICE, "pinned staging allocation failed");
    }
    s->dpool.init(opts->hbm_budget);
    s->hpool.init(opts->host_staging);
    s->slots.resize((size_t)opts->n_streams);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
            hmm_server_destroy(s);
            return server_fail(HMM_ERR_DEVICE, "stream creation failed");
        }
    }
    s->worker = std::thread([s] { s->run(); });
    *out = s;
    return HMM_OK;
}

hmm_status hmm_server_destroy(hmm_server *s) {
    if (!s) return server_fail(HMM_ERR_ARG, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable()) s->worker.join();
    for (auto &sl : s->slots) {
        if (sl.stream) hipStreamSynchronize(sl.stream);
        if (sl.stream) hipStreamDestroy(sl.stream);
    }
    for (auto &m : s->models) hipFree(m.buf);
    if (s->host) hipHostFree(s->host);
    if (s->dev) hipFree(s->dev);
    delete s;
    return HMM_OK;
}

hmm_status hmm_server_add_model(hmm_server *s, const hmm_model *model, int32_t *model_id) {
    if (!s || !model || !model_id) return server_fail(HMM_ERR_ARG, "server / model / id is NULL");
    size_t tl = 0;
    hmm_status st = hmmk::model_theta_len(model, &tl);
    if (st != HMM_OK) return st;
    const size_t N = (size_t)model->n_states;
    Model m;
    m.m = *model;
    m.D = model->family == HMM_TABLE ? model->n_states : model->dim;
    const size_t nd = N + N * N + tl;
    if (hipMalloc((void **)&m.buf, std::max<size_t>(nd, 1) * sizeof(double)) != hipSuccess)
        return server_fail(HMM_ERR_DEVICE, "model allocation failed");
    bool okc = hipMemcpy(m.buf, model->log_pi, N * 8, hipMemcpyDeviceToDevice) == hipSuccess &&
               hipMemcpy(m.buf + N, model->log_A, N * N * 8, hipMemcpyDeviceToDevice) == hipSuccess;
    if (okc && tl)
        okc = hipMemcpy(m.buf + N + N * N, model->theta, tl * 8, hipMemcpyDeviceToDevice) == hipSuccess;
    if (!okc) {
        hipFree(m.buf);
        return server_fail(HMM_ERR_DEVICE, "model copy failed");
    }
    m.m.log_pi = m.buf;
    m.m.log_A = m.buf + N;
    m.m.theta = tl ? m.buf + N + N * N : model->theta;
    std::lock_guard<std::mutex> lk(s->mu);
    s->models.push_back(m);
    *model_id = (int32_t)s->models.size() - 1;
    return HMM_OK;
}

hmm_status hmm_server_submit(hmm_server *s, int32_t model_id, int32_t kind, const void *obs,
                             int32_t obs_f64, int64_t T, int32_t *path_out, uint64_t *id) {
    if (!s || !obs || !path_out || !id)
        return server_fail(HMM_ERR_ARG, "server / obs / path_out / id is NULL");
    if (kind != HMM_REQ_VITERBI && kind != HMM_REQ_POSTERIOR_DECODE)
        return server_fail(HMM_ERR_ARG, "unknown request kind");
    if (T < 1) return server_fail(HMM_ERR_ARG, "T must be >= 1");
    if (obs_f64 != 0 && obs_f64 != 1) return server_fail(HMM_ERR_ARG, "obs_f64 must be 0 or 1");
    int D;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (model_id < 0 || (size_t)model_id >= s->models.size())
            return server_fail(HMM_ERR_ARG, "unknown model id");
        D = s->models[(size_t)model_id].D;
        Layout l;
        hmm_status st = s->plan(s->models[(size_t)model_id], kind, {0, T}, &l);
        if (st != HMM_OK) return st;
        if (l.dev_total > s->dpool.cap || l.host_total > s->hpool.cap)
            return server_fail(HMM_ERR_WORKSPACE, "request needs more than the server's budget");
    }
    Req r;
    r.model = model_id;
    r.kind = kind;
    r.T = T;
    r.path_out = path_out;
    const size_t n = (size_t)T * (size_t)D;
    r.obs.resize(n * s->es);
    if (s->es == 8) {
        double *d = (double *)r.obs.data();
        if (obs_f64) std::memcpy(d, obs, n * 8);
        else for (size_t i = 0; i < n; ++i) d[i] = ((const float *)obs)[i];
    } else {
        float *d = (float *)r.obs.data();
        if (!obs_f64) std::memcpy(d, obs, n * 4);
        else for (size_t i = 0; i < n; ++i) d[i] = (float)((const double *)obs)[i];
    }
    {
        std::lock_guard<std::mutex> lk(s->mu);
        r.id = s->next_id++;
        *id = r.id;
        r.t_submit = now_s();
        s->pending.push_back(std::move(r));
        ++s->n_submitted;
        ++s->submits;
    }
    s->cv_work.notify_one();
    return HMM_OK;
}

hmm_status hmm_server_poll(hmm_server *s, hmm_completion *out, int32_t max, int32_t timeout_us,
                           int32_t *n_out) {
    if (!s || !n_out || (max > 0 && !out)) return server_fail(HMM_ERR_ARG, "NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && timeout_us > 0)
        s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                            [&] { return !s->done.empty(); });
    int32_t n = 0;
    while (n < max && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return HMM_OK;
}

hmm_status hmm_server_get_info(hmm_server *s, hmm_server_info *info) {
    if (!s || !info) return server_fail(HMM_ERR_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    info->submitted = s->n_submitted;
    info->completed = s->n_completed;
    info->launches = s->n_launches;
    info->pending = (int64_t)s->pending.size();
    info->in_flight = s->n_in_flight;
    info->pool_bytes = s->opts.hbm_budget & ~(size_t)255;
    info->pool_used = s->pool_used;
    info->pool_peak = s->pool_peak;
    return HMM_OK;
}

}  // extern "C"
