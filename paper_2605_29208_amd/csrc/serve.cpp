// serve.cpp -- the request-serving runtime of hmm_serve.h.
//
// One worker thread per server.  Each pass of its loop
//   1. retires launches whose completion event has fired: copies every
//      request's path out of the pinned staging area into the caller's
//      buffer, records the completion and returns the launch's device and
//      host blocks to their pools;
//   2. while a launch slot (stream) is free, forms a batch from the oldest
//      pending request and the pending requests of the same model and kind
//      behind it (up to max_batch, as long as the batch's bytes fit the free
//      device budget and staging area), uploads it, enqueues the decode and
//      the download on the slot's stream and records the slot's event;
//   3. sleeps until a submission arrives or, with launches in flight, for a
//      few microseconds.
// Device and pinned memory come from two areas allocated at creation and
// carved by a first-fit allocator, so the serving loop never allocates
// device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
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
    int slot;
    std::vector<Req> reqs;
    std::vector<int64_t> h_off;
    Layout lay;
    size_t dev_off = 0, host_off = 0;
    double t_launch = 0;
    hmm_status launch_status = HMM_OK;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
};

}  // namespace

struct hmm_server {
    hmm_server_opts opts;
    char *dev = nullptr;     // device budget area
    char *host = nullptr;    // pinned staging area
    Pool dpool, hpool;
    std::vector<Slot> slots;
    std::vector<Model> models;
    std::deque<Req> pending;
    std::deque<Flight> flights;
    std::deque<hmm_completion> done;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint64_t next_id = 1;
    int64_t n_submitted = 0, n_completed = 0, n_launches = 0;
    size_t es = 4;           // bytes per observation value

    hmm_status plan(int model, int kind, const std::vector<int64_t> &h_off, Layout *lay);
    bool launch_one();
    void retire(Flight &f);
    void run();
};

namespace {

hmm_status server_fail(hmm_status st, const char *msg) { return fail_status(st, "%s", msg); }

}  // namespace

hmm_status hmm_server::plan(int model, int kind, const std::vector<int64_t> &h_off, Layout *lay) {
    const Model &md = models[(size_t)model];
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

void hmm_server::retire(Flight &f) {
    const char *hb = host + f.host_off;
    const double *lp = (const double *)(hb + f.lay.o_logp);
    for (size_t k = 0; k < f.reqs.size(); ++k) {
        Req &r = f.reqs[k];
        hmm_completion c{};
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
        done.push_back(c);
        ++n_completed;
    }
    if (f.lay.dev_total) dpool.release(f.dev_off, f.lay.dev_total);
    if (f.lay.host_total) hpool.release(f.host_off, f.lay.host_total);
    slots[(size_t)f.slot].busy = false;
    cv_done.notify_all();
}

bool hmm_server::launch_one() {
    int slot = -1;
    for (size_t i = 0; i < slots.size(); ++i)
        if (!slots[i].busy) {
            slot = (int)i;
            break;
        }
    if (slot < 0 || pending.empty()) return false;
    const int model = pending.front().model, kind = pending.front().kind;
    // gather same-key requests in arrival order while the batch fits
    std::vector<size_t> pick;
    std::vector<int64_t> h_off{0};
    Layout lay;
    const size_t dfree = dpool.largest(), hfree = hpool.largest();
    const size_t window = std::min<size_t>(pending.size(), 1024);
    for (size_t i = 0; i < window && (int)pick.size() < opts.max_batch; ++i) {
        const Req &r = pending[i];
        if (r.model != model || r.kind != kind) continue;
        std::vector<int64_t> trial = h_off;
        trial.push_back(trial.back() + r.T);
        Layout l;
        if (plan(model, kind, trial, &l) != HMM_OK) {
            if (pick.empty()) {
                // the head request cannot be served at all: report it
                Flight f;
                f.slot = slot;
                f.reqs.push_back(std::move(pending.front()));
                pending.pop_front();
                f.h_off = {0, f.reqs[0].T};
                f.launch_status = HMM_ERR_UNSUPPORTED;
                f.t_launch = now_s();
                slots[(size_t)slot].busy = true;
                retire(f);
                return true;
            }
            break;
        }
        if (l.dev_total > dfree || l.host_total > hfree) break;
        pick.push_back(i);
        h_off.swap(trial);
        lay = l;
    }
    if (pick.empty()) return false;   // wait for memory to free up
    Flight f;
    f.slot = slot;
    f.h_off = h_off;
    f.lay = lay;
    dpool.alloc(lay.dev_total, &f.dev_off);
    hpool.alloc(lay.host_total, &f.host_off);
    // move the picked requests out of the queue (back to front keeps indices valid)
    f.reqs.resize(pick.size());
    for (size_t k = pick.size(); k-- > 0;) {
        f.reqs[k] = std::move(pending[pick[k]]);
        pending.erase(pending.begin() + (std::ptrdiff_t)pick[k]);
    }
    char *hb = host + f.host_off;
    char *db = dev + f.dev_off;
    std::memcpy(hb, h_off.data(), lay.off_b);
    for (size_t k = 0; k < f.reqs.size(); ++k)
        std::memcpy(hb + lay.o_obs + (size_t)h_off[k] * models[(size_t)model].D * es,
                    f.reqs[k].obs.data(), f.reqs[k].obs.size());
    Slot &sl = slots[(size_t)slot];
    hipStream_t s = sl.stream;
    hmm_status st = HMM_OK;
    if (hipMemcpyAsync(db, hb, lay.o_path, hipMemcpyHostToDevice, s) != hipSuccess)
        st = HMM_ERR_DEVICE;
    const Model &md = models[(size_t)model];
    const int64_t B = (int64_t)f.reqs.size();
    hmm_batch b{B, (const int64_t *)db, h_off.data(), db + lay.o_obs,
                opts.precision == HMM_PREC_F64, 0};
    int32_t *path = (int32_t *)(db + lay.o_path);
    double *logp = (double *)(db + lay.o_logp);
    if (st == HMM_OK) {
        if (kind == HMM_REQ_VITERBI)
            st = hmm_viterbi(&md.m, &b, (hmm_precision)opts.precision, path, logp, db + lay.o_ws,
                             lay.ws_b, s);
        else
            st = hmm_posterior_decode(&md.m, &b, (hmm_precision)opts.precision, path, logp,
                                      db + lay.o_ws, lay.ws_b, s);
    }
    if (st == HMM_OK &&
        hipMemcpyAsync(hb + lay.o_path, db + lay.o_path, lay.host_total - lay.o_path,
                       hipMemcpyDeviceToHost, s) != hipSuccess)
        st = HMM_ERR_DEVICE;
    f.launch_status = st;
    f.t_launch = now_s();
    hipEventRecord(sl.done, s);
    sl.busy = true;
    ++n_launches;
    flights.push_back(std::move(f));
    return true;
}

void hmm_server::run() {
    hipSetDevice(opts.device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        bool progressed = false;
        for (auto it = flights.begin(); it != flights.end();) {
            if (hipEventQuery(slots[(size_t)it->slot].done) != hipErrorNotReady) {
                retire(*it);
                it = flights.erase(it);
                progressed = true;
            } else {
                ++it;
            }
        }
        if (stop && flights.empty()) break;
        while (!stop && launch_one()) progressed = true;
        if (progressed) continue;
        if (flights.empty())
            cv_work.wait(lk, [&] { return stop || !pending.empty(); });
        else
            cv_work.wait_for(lk, std::chrono::microseconds(20));
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
    if (opts->n_streams < 1 || opts->n_streams > 8)
        return server_fail(HMM_ERR_ARG, "n_streams must be in 1 .. 8");
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
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            hmm_server_destroy(s);
            return server_fail(HMM_ERR_DEVICE, "stream / event creation failed");
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
        if (sl.done) hipEventDestroy(sl.done);
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
        hmm_status st = s->plan(model_id, kind, {0, T}, &l);
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
    info->in_flight = (int64_t)s->flights.size();
    info->pool_bytes = s->dpool.cap;
    info->pool_used = s->dpool.used;
    info->pool_peak = s->dpool.peak;
    return HMM_OK;
}

}  // extern "C"
