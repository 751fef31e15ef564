// abi.cpp -- extern "C" entry points: argument validation on the host,
// workspace planning, parameter staging and dispatch to the kernels.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "hmm_internal.hpp"

using namespace hmmk;

namespace {

thread_local std::string g_err;
std::atomic<int> g_chunk_len{0};

hmm_status fail(hmm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hmm_status ok() {
    g_err.clear();
    return HMM_OK;
}

inline size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

int family_k(int family, int D) {
    switch (family) {
    case HMM_GAUSSIAN: return 2;
    case HMM_GAMMA: return 3;
    case HMM_STUDENT_T: return 4;
    case HMM_POISSON: return 1;
    case HMM_DIAG_GAUSSIAN: return 2 * D;
    case HMM_FULL_GAUSSIAN: return D + D * (D + 1) / 2;
    case HMM_TABLE: return 0;
    default: return -1;
    }
}

bool is_f64(hmm_precision p) { return p == HMM_PREC_F64 || p == HMM_PREC_PLAIN_F64; }
bool is_plain(hmm_precision p) { return p == HMM_PREC_PLAIN_F32 || p == HMM_PREC_PLAIN_F64; }

struct Checked {
    int N, D, fam;
    int64_t B, total, Tmax;
    const int64_t *h_off;
};

hmm_status check_model(const hmm_model *m) {
    if (!m) return fail(HMM_ERR_ARG, "model is NULL");
    if (m->n_states < 1 || m->n_states > 1024)
        return fail(HMM_ERR_ARG, "n_states %d outside [1, 1024]", m->n_states);
    if (m->family < HMM_GAUSSIAN || m->family > HMM_TABLE)
        return fail(HMM_ERR_ARG, "unknown family %d", m->family);
    if (m->reserved != 0) return fail(HMM_ERR_ARG, "model.reserved must be 0");
    const bool scalar = m->family <= HMM_POISSON;
    if (scalar && m->dim != 1) return fail(HMM_ERR_ARG, "scalar family needs dim == 1 (got %d)", m->dim);
    if (m->family == HMM_TABLE && m->dim != m->n_states)
        return fail(HMM_ERR_ARG, "table family needs dim == n_states");
    if ((m->family == HMM_DIAG_GAUSSIAN || m->family == HMM_FULL_GAUSSIAN) &&
        (m->dim < 1 || m->dim > 64))
        return fail(HMM_ERR_ARG, "multivariate dim %d outside [1, 64]", m->dim);
    if (!m->log_pi || !m->log_A) return fail(HMM_ERR_ARG, "log_pi / log_A is NULL");
    if (m->family != HMM_TABLE && !m->theta)
        return fail(HMM_ERR_PARAMS_UNSET, "emission parameters (theta) are not set");
    return HMM_OK;
}

hmm_status check_batch(const hmm_batch *b, const hmm_model *m, Checked *c) {
    hmm_status st = check_model(m);
    if (st != HMM_OK) return st;
    if (!b) return fail(HMM_ERR_ARG, "batch is NULL");
    if (b->n_seq < 0) return fail(HMM_ERR_ARG, "n_seq < 0");
    if (b->reserved != 0) return fail(HMM_ERR_ARG, "batch.reserved must be 0");
    if (b->obs_f64 != 0 && b->obs_f64 != 1) return fail(HMM_ERR_ARG, "obs_f64 must be 0 or 1");
    c->N = m->n_states;
    c->D = m->dim;
    c->fam = m->family;
    c->B = b->n_seq;
    c->total = 0;
    c->Tmax = 0;
    c->h_off = b->h_offsets;
    if (b->n_seq == 0) return HMM_OK;
    if (!b->offsets || !b->h_offsets || !b->obs)
        return fail(HMM_ERR_ARG, "offsets / h_offsets / obs is NULL");
    if (b->h_offsets[0] != 0) return fail(HMM_ERR_ARG, "offsets[0] must be 0");
    for (int64_t i = 0; i < b->n_seq; ++i) {
        int64_t T = b->h_offsets[i + 1] - b->h_offsets[i];
        if (T < 1) return fail(HMM_ERR_ARG, "sequence %lld has length %lld (must be >= 1)",
                                (long long)i, (long long)T);
        if (T > c->Tmax) c->Tmax = T;
    }
    c->total = b->h_offsets[b->n_seq];
    if (c->Tmax > (int64_t)1 << 30) return fail(HMM_ERR_ARG, "sequence longer than 2^30 steps");
    return HMM_OK;
}

// ---------------------------------------------------------------- planning
struct Plan {
    bool f64 = false, plain = false, chunked = false, wave = false, block = false;
    int mfma = 0;   // scaled low-precision sweeps: 1 bf16, 2 fp16
    int G = 0, L = 0, C = 0, nblk = 0;
    int64_t S = 0;
    size_t staged = 0, cbase = 0, rec = 0, F = 0, Gb = 0, partial = 0;
    int SS = 16, SC = 0;   // chunks per superchunk, number of superchunks
    size_t sbase = 0, srec = 0, Fs = 0, Gs = 0, cdesc = 0, sdesc = 0;
    size_t vpsi = 0, vJ = 0, vqlast = 0, vqend = 0;
    size_t ll = 0, st = 0, gam = 0;
    size_t logB = 0, alpha = 0, beta = 0, ps = 0;
    size_t red = 0;
    size_t etab = 0, mt = 0, balpha = 0, aexp = 0, bgam = 0, xi = 0, xisum = 0, g1 = 0, compact = 0;
    int xi_nsl = 1;
    bool mvw = false;   // multivariate family on the wave path (log-density table)
    int route = 0;      // ROUTE_* of the batched path taken
    int variant = 0;    // tuned variant of that route
    size_t lt = 0, fpart = 0, red2 = 0;
    size_t lsc = 0, segJ = 0, seginc = 0, segbad = 0, segver = 0, seglim = 0;
    size_t total = 0;
};

// ---------------------------------------------------------------- variants and the tuner
// Each batched route has a few runtime variants (a schedule choice that does
// not change the arithmetic's definition):
//   chunked N <= 8: chunk length 16, 32 or 64 steps (FP64: 16 or 32);
//   large-state:    slices of the transition contraction, nominal, half or
//                   double (the split of its row dimension over workgroups);
//   wave:           sweep segments of 1024 steps, whole sequences, 512 or
//                   2048 steps;
//   plain:          one variant.
// hmm_autotune times every variant of a call's route on the caller's data and
// keeps the fastest for the call's key; HMM_FORCE_VARIANT (environment) or
// hmm_set_variant forces one.  The key is the device architecture, family,
// N, D, precision, route and the batch's shape in powers of two (sequence
// count, mean and longest length).  HMM_TUNE_CACHE names a text file that
// keeps the choices across processes ("key variant" per line).
enum { ROUTE_PLAIN = 0, ROUTE_CHUNK = 1, ROUTE_WAVE = 2, ROUTE_BLOCK = 3 };

int route_variants(int route, bool f64) {
    if (route == ROUTE_CHUNK) return f64 ? 2 : 3;
    if (route == ROUTE_BLOCK) return 3;
    if (route == ROUTE_WAVE) return 4;
    return 1;
}

std::mutex g_tune_mu;
std::map<std::string, int> g_tune;
bool g_tune_loaded = false;
std::atomic<int> g_force_variant{-2};   // -2: environment not read yet, -1: none

int force_variant() {
    int v = g_force_variant.load();
    if (v == -2) {
        const char *e = getenv("HMM_FORCE_VARIANT");
        v = (e && *e) ? atoi(e) : -1;
        if (v < -1) v = -1;
        int expect = -2;
        g_force_variant.compare_exchange_strong(expect, v);
        v = g_force_variant.load();
    }
    return v;
}

const char *tune_cache_path() {
    const char *e = getenv("HMM_TUNE_CACHE");
    return (e && *e) ? e : nullptr;
}

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = tune_cache_path();
    if (!path) return;
    FILE *f = fopen(path, "r");
    if (!f) return;
    char key[512];
    int v;
    while (fscanf(f, "%511s %d%*[^\n]", key, &v) == 2) g_tune[key] = v;
    fclose(f);
}

int ilog2_ceil(int64_t x) {
    int k = 0;
    while (((int64_t)1 << k) < x && k < 62) ++k;
    return k;
}

std::string device_arch() {
    static std::mutex mu;
    static std::map<int, std::string> names;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    std::lock_guard<std::mutex> lk(mu);
    auto it = names.find(dev);
    if (it != names.end()) return it->second;
    hipDeviceProp_t prop;
    std::string n = "unknown";
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        n = prop.gcnArchName;
        for (char &ch : n)
            if (ch == ' ') ch = '_';
    }
    names[dev] = n;
    return n;
}

std::string tune_key(const Checked &c, hmm_precision prec, int route) {
    char buf[400];
    const int64_t mean = c.B > 0 ? (c.total + c.B - 1) / c.B : 0;
    snprintf(buf, sizeof buf, "%s|fam%d|N%d|D%d|prec%d|route%d|B%d|Tmean%d|Tmax%d",
             device_arch().c_str(), c.fam, c.N, c.D, (int)prec, route, ilog2_ceil(c.B),
             ilog2_ceil(mean), ilog2_ceil(c.Tmax));
    return buf;
}

// the variant a call takes: forced, else tuned for its key, else 0
int resolve_variant(const Checked &c, hmm_precision prec, int route) {
    const int nv = route_variants(route, is_f64(prec));
    const int fv = force_variant();
    if (fv >= 0) return fv < nv ? fv : nv - 1;
    if (nv == 1) return 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    auto it = g_tune.find(tune_key(c, prec, route));
    if (it == g_tune.end() || it->second < 0 || it->second >= nv) return 0;
    return it->second;
}

void tune_store(const Checked &c, hmm_precision prec, int route, int v, const float *ms, int nv) {
    const std::string key = tune_key(c, prec, route);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    g_tune[key] = v;
    const char *path = tune_cache_path();
    if (!path) return;
    FILE *f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d", key.c_str(), v);
    for (int k = 0; k < nv; ++k) fprintf(f, " %.4f", ms[k]);
    fprintf(f, "\n");
    fclose(f);
}

int chunk_len_of(int variant, bool f64) {
    static const int L[3] = {16, 32, 64};
    int v = variant < 0 ? 0 : (variant > 2 ? 2 : variant);
    if (f64 && v > 1) v = 1;
    return L[v];
}

int default_chunk_len(bool f64) {
    int v = g_chunk_len.load();
    if (v == 0) return 16;
    if (f64 && v > 32) return 32;
    return v;
}

// variant < 0: the resolved variant of the call (forced, tuned or 0)
hmm_status make_plan(hmm_op op, const Checked &c, hmm_precision prec, Plan *p, int variant = -1) {
    if (prec < HMM_PREC_F64 || prec > HMM_PREC_PLAIN_F64)
        return fail(HMM_ERR_ARG, "unknown precision %d", (int)prec);
    p->f64 = is_f64(prec);
    p->plain = is_plain(prec);
    const size_t r = p->f64 ? 8 : 4;
    const int N = c.N;
    p->S = 1 + 2 * (int64_t)N + (int64_t)N * N + (int64_t)N * family_k(c.fam, c.D);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += a256(bytes);
        return o;
    };
    p->staged = take(staged_bytes(N, c.D, c.fam, p->f64));
    if (op == HMM_OP_EMISSION) {
        p->total = off;
        return HMM_OK;
    }
    if (op == HMM_OP_VITERBI) {
        if (p->plain || prec == HMM_PREC_BF16_SCALED || prec == HMM_PREC_F16_SCALED)
            return fail(HMM_ERR_UNSUPPORTED, "Viterbi runs in HMM_PREC_F64 or HMM_PREC_F32");
        if (N > 64) return fail(HMM_ERR_UNSUPPORTED, "Viterbi: this build covers N <= 64 (N = %d)", N);
        int64_t C = 0, SC = 0;
        const int vs = vit_seg_chunks();
        for (int64_t b = 0; b < c.B; ++b) {
            const int64_t nc = (c.h_off[b + 1] - c.h_off[b] + 63) / 64;
            C += nc;
            SC += (nc + vs - 1) / vs;
        }
        if (C > INT32_MAX / 64) return fail(HMM_ERR_UNSUPPORTED, "too many chunks");
        p->C = (int)C;
        p->SC = (int)SC;
        p->SS = vs;
        p->sdesc = take((size_t)SC * sizeof(SuperDesc));
        p->lt = take((size_t)C * 64 * (p->f64 ? 8 : 4));   // shifted scores at chunk ends
        p->lsc = take((size_t)C * 8);
        p->segJ = take((size_t)SC * 8);
        p->seginc = take((size_t)SC * 8);
        p->segbad = take((size_t)SC * 4);
        p->segver = take((size_t)SC * 4);
        p->seglim = take((size_t)SC * 4);
        p->vpsi = take((size_t)c.total * N);
        p->vJ = take((size_t)C * N);
        p->vqlast = take((size_t)c.B);
        p->vqend = take((size_t)C);
        p->cbase = take((size_t)(c.B + 1) * 4);
        p->sbase = take((size_t)(c.B + 1) * 4);
        p->cdesc = take((size_t)C * sizeof(ChunkDesc));
        p->total = off;
        return HMM_OK;
    }
    if (op != HMM_OP_FORWARD_BACKWARD && op != HMM_OP_ESTEP && op != HMM_OP_POSTERIOR_DECODE)
        return fail(HMM_ERR_ARG, "unknown op %d", (int)op);
    p->ll = take((size_t)c.B * 8);
    p->st = take((size_t)c.B * 4);
    if (op == HMM_OP_POSTERIOR_DECODE) p->gam = take((size_t)c.total * N * r);
    if (p->plain) {
        p->logB = take((size_t)c.total * N * r);
        p->alpha = take((size_t)c.total * N * r);
        p->beta = take((size_t)c.total * N * r);
        p->ps = take(((size_t)c.B * p->S + (size_t)c.B) * 8);
        p->red = take((size_t)reduce_scratch_len(c.B, p->S) * 8);
    } else {
        const bool scalar = c.fam <= HMM_POISSON || c.fam == HMM_TABLE;
        p->mfma = prec == HMM_PREC_BF16_SCALED ? 1 : (prec == HMM_PREC_F16_SCALED ? 2 : 0);
        // FP64 with 32 < N <= 64 takes the one-workgroup-per-sequence path: the
        // wave path's statistics kernel would hold both A's column and row and
        // the 64 xi accumulators in FP64 per lane, more than the register file
        // (measured 1.6-1.8x slower on 256 sequences of 500-3000 steps)
        const bool f64big = p->f64 && N > 32;
        const bool mvw = !scalar && N <= 64 && !p->mfma && !f64big &&
                         (c.fam == HMM_DIAG_GAUSSIAN || c.fam == HMM_FULL_GAUSSIAN);
        if (!mvw && (!scalar || N > 64 || p->mfma || f64big)) {
            // one workgroup per sequence, emission table, xi by a matrix-core contraction
            if (N > 256)
                return fail(HMM_ERR_UNSUPPORTED,
                            "batched path: this build covers N <= 256 (N = %d); use a PLAIN "
                            "precision", N);
            p->block = true;
            p->route = ROUTE_BLOCK;
            p->variant = variant >= 0 ? variant : resolve_variant(c, prec, ROUTE_BLOCK);
            const size_t T = (size_t)c.total;
            p->etab = take(T * N * r);
            p->mt = take(T * 8);
            p->balpha = take(T * N * r);
            p->aexp = take(T * 4);
            if (op == HMM_OP_ESTEP || op == HMM_OP_FORWARD_BACKWARD) p->bgam = take(T * N * r);
            {
                // variant 1 halves the nominal slice count, variant 2 doubles it
                const int nom = xi_slices(p->f64, N, c.total);
                const int64_t K = c.total - 1;
                int nsl = p->variant == 1 ? (nom + 1) / 2 : (p->variant == 2 ? 2 * nom : nom);
                const int64_t by_rows = K > 0 ? (K + 15) / 16 : 1;   // at least 16 rows a slice
                if (nsl > by_rows) nsl = (int)by_rows;
                if (nsl < 1) nsl = 1;
                p->xi_nsl = nsl;
                const int64_t nc = xi_nc(N);
                p->xi = take((size_t)nsl * nc * nc * r);
            }
            p->xisum = take((size_t)N * N * 8);
            p->g1 = take((size_t)N * 8);
            const int64_t S2 = 1 + N + (int64_t)N * family_k(c.fam, c.D);
            const int ntile = blk_gstats_tiles(c.total, c.fam);
            p->compact = take((size_t)S2 * 8);
            p->partial = take((size_t)ntile * S2 * 8);
            p->red = take((size_t)reduce_scratch_len(ntile, S2) * 8);
            p->total = off;
            return HMM_OK;
        }
        if (N > 8 || mvw) {
            // per-sequence sweeps + one wave per chunk of WAVE_L steps
            p->wave = true;
            p->route = ROUTE_WAVE;
            p->L = WAVE_L;
            p->variant = variant >= 0 ? variant : resolve_variant(c, prec, ROUTE_WAVE);
            p->SS = wave_seg_chunks(p->variant);
            int64_t C = 0, SC = 0;
            for (int64_t b = 0; b < c.B; ++b) {
                const int64_t nc = (c.h_off[b + 1] - c.h_off[b] + WAVE_L - 1) / WAVE_L;
                C += nc;
                SC += (nc + p->SS - 1) / p->SS;
            }
            if (C > INT32_MAX / 64) return fail(HMM_ERR_UNSUPPORTED, "too many chunks");
            p->C = (int)C;
            p->SC = (int)SC;
            p->nblk = wave_stats_blocks((int)C, N);
            const int np = wave_np(N);
            p->cbase = take((size_t)(c.B + 1) * 4);
            p->sbase = take((size_t)(c.B + 1) * 4);
            p->cdesc = take((size_t)C * sizeof(ChunkDesc));
            p->sdesc = take((size_t)SC * sizeof(SuperDesc));
            p->lsc = take((size_t)C * 8);
            p->segJ = take((size_t)SC * 8);
            p->seginc = take((size_t)SC * 8);
            p->segbad = take((size_t)SC * 4);
            p->segver = take((size_t)SC * 8);
            p->seglim = take((size_t)SC * 8);
            p->F = take((size_t)C * np * r);
            p->Gb = take((size_t)C * np * r);
            p->partial = take((size_t)p->nblk * p->S * 8);
            p->red = take((size_t)reduce_scratch_len(p->nblk, p->S) * 8);
            if (mvw) {
                p->mvw = true;
                p->lt = take((size_t)c.total * N * r);
                if (op == HMM_OP_ESTEP) {
                    const int64_t S2 = 1 + N + (int64_t)N * family_k(c.fam, c.D);
                    const int ntile = blk_gstats_tiles(c.total, c.fam);
                    p->bgam = take((size_t)c.total * N * r);
                    p->fpart = take((size_t)ntile * S2 * 8);
                    p->compact = take((size_t)S2 * 8);
                    p->red2 = take((size_t)reduce_scratch_len(ntile, S2) * 8);
                }
            }
            p->total = off;
            return HMM_OK;
        }
        p->chunked = true;
        p->route = ROUTE_CHUNK;
        p->G = N <= 4 ? 4 : 8;
        p->variant = variant >= 0 ? variant : resolve_variant(c, prec, ROUTE_CHUNK);
        // hmm_set_chunk_len, when set, overrides the variant's length
        p->L = g_chunk_len.load() != 0 ? default_chunk_len(p->f64) : chunk_len_of(p->variant, p->f64);
        int64_t C = 0, SC = 0;
        for (int64_t b = 0; b < c.B; ++b) {
            int64_t T = c.h_off[b + 1] - c.h_off[b];
            int64_t nc = (T + p->L - 1) / p->L;
            C += nc;
            SC += (nc + p->SS - 1) / p->SS;
        }
        p->SC = (int)SC;
        if (C > INT32_MAX / 64) return fail(HMM_ERR_UNSUPPORTED, "too many chunks");
        p->C = (int)C;
        // statistics blocks take whole superchunks of SS chunks, one lane group per chunk
        const int spb = (BLOCK / 64) * (64 / p->G) / p->SS;
        int64_t nb = (SC + spb - 1) / spb;
        p->nblk = (int)(nb < 1 ? 1 : (nb > 2048 ? 2048 : nb));
        p->cbase = take((size_t)(c.B + 1) * 4);
        p->rec = take((size_t)C * p->G * chunk_rec_bytes(p->f64, p->G));   // one record per lane
        p->F = take((size_t)(C + 1) * p->G * r);    // + one sink slot
        p->Gb = take((size_t)(C + 1) * p->G * r);
        p->partial = take((size_t)p->nblk * p->S * 8);
        p->red = take((size_t)reduce_scratch_len(p->nblk, p->S) * 8);
        const size_t rb = chunk_rec_bytes(p->f64, p->G);
        p->sbase = take((size_t)(c.B + 1) * 4);
        p->sdesc = take((size_t)SC * sizeof(SuperDesc));
        p->srec = take((size_t)SC * p->G * rb);
        p->Fs = take((size_t)(SC + 1) * p->G * r);
        p->Gs = take((size_t)(SC + 1) * p->G * r);
    }
    p->total = off;
    return HMM_OK;
}

hmm_status check_ws(const Plan &p, void *ws, size_t ws_bytes) {
    if (ws_bytes < p.total)
        return fail(HMM_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required",
                    ws_bytes, p.total);
    if (p.total > 0 && !ws) return fail(HMM_ERR_WORKSPACE, "workspace pointer is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(HMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    return HMM_OK;
}

hmm_status device_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(HMM_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
    return ok();
}

RawModel raw(const hmm_model *m) {
    return RawModel{m->n_states, m->dim, m->family, m->log_pi, m->log_A, m->theta};
}

template <typename R>
hmm_status run_posterior_path(const hmm_model *m, const hmm_batch *b, const Checked &c,
                              const Plan &p, char *ws, double *loglik, int32_t *status,
                              void *gamma_out, double *stats, hipStream_t s) {
    StagedModel<R> sm;
    // the N <= 8 path counts its chunks in the staging launch
    const PlanArgs plan{b->offsets, c.B, p.L, p.SS, (int *)(ws + p.cbase), (int *)(ws + p.sbase)};
    launch_stage<R>(raw(m), ws + p.staged, &sm, s, (p.chunked && c.B > 0) ? &plan : nullptr);
    double *ll = loglik ? loglik : (double *)(ws + p.ll);
    int32_t *st = status ? status : (int32_t *)(ws + p.st);
    ObsDesc od{b->obs, b->obs_f64, c.B, b->offsets};
    if (c.B == 0) {
        if (stats) launch_reduce_stats(nullptr, 0, p.S, ll, st, 0, stats, nullptr, s);
        return device_check("estep (empty batch)");
    }
    hmm_status r;
    if (p.plain) {
        PlainBuffers pb{ws + p.logB, ws + p.alpha, ws + p.beta, (double *)(ws + p.ps),
                        (double *)(ws + p.red)};
        r = run_plain<R>(sm, od, pb, ll, st, gamma_out, stats, p.S, s);
    } else if (p.block) {
        BlockBuffers bb;
        bb.total = c.total;
        bb.mfma = p.mfma;
        bb.etab = ws + p.etab;
        bb.mt = (double *)(ws + p.mt);
        bb.alpha = ws + p.balpha;
        bb.aexp = (int32_t *)(ws + p.aexp);
        bb.gamma = p.bgam ? (void *)(ws + p.bgam) : nullptr;
        bb.xi = ws + p.xi;
        bb.xi_nsl = p.xi_nsl;
        bb.xisum = (double *)(ws + p.xisum);
        bb.g1 = (double *)(ws + p.g1);
        bb.partial = (double *)(ws + p.partial);
        bb.compact = (double *)(ws + p.compact);
        bb.red = (double *)(ws + p.red);
        r = run_block<R>(sm, od, bb, ll, st, gamma_out, stats, p.S, s);
    } else if (p.wave) {
        WaveBuffers wb;
        wb.C = p.C;
        wb.nblk = p.nblk;
        wb.cbase = (int *)(ws + p.cbase);
        wb.cdesc = (ChunkDesc *)(ws + p.cdesc);
        wb.F = ws + p.F;
        wb.Gb = ws + p.Gb;
        wb.partial = (double *)(ws + p.partial);
        wb.red = (double *)(ws + p.red);
        int *sbase = (int *)(ws + p.sbase);
        SuperDesc *sdesc = (SuperDesc *)(ws + p.sdesc);
        wb.SC = p.SC;
        wb.vmax = WAVE_VMAX;
        wb.sbase = sbase;
        wb.sdesc = sdesc;
        wb.lsc = (double *)(ws + p.lsc);
        wb.segJ = (double *)(ws + p.segJ);
        wb.seginc = (double *)(ws + p.seginc);
        wb.segbad = (int32_t *)(ws + p.segbad);
        wb.segver = (int32_t *)(ws + p.segver);
        wb.seglim = (int32_t *)(ws + p.seglim);
        launch_plan_chunks(b->offsets, c.B, p.L, p.SS, wb.cbase, sbase, s);
        launch_chunk_desc(b->offsets, c.B, p.L, p.SS, wb.cbase, sbase, p.C, p.SC, wb.cdesc, sdesc,
                          s);
        if (p.mvw) {
            MvBuffers mb;
            mb.total = c.total;
            mb.lt = ws + p.lt;
            mb.gamma = p.bgam ? (void *)(ws + p.bgam) : nullptr;
            mb.partial = (double *)(ws + p.fpart);
            mb.compact = (double *)(ws + p.compact);
            mb.red = (double *)(ws + p.red2);
            r = run_wave_mv<R>(sm, od, wb, mb, ll, st, gamma_out, stats, s);
        } else {
            r = run_wave<R>(sm, od, wb, ll, st, gamma_out, stats, p.S, s);
        }
    } else {
        ChunkBuffers cb;
        cb.L = p.L;
        cb.C = p.C;
        cb.G = p.G;
        cb.nblk_stats = p.nblk;
        cb.cbase = (int *)(ws + p.cbase);
        cb.rec = ws + p.rec;
        cb.F = ws + p.F;
        cb.Gb = ws + p.Gb;
        cb.partial = (double *)(ws + p.partial);
        cb.red = (double *)(ws + p.red);
        cb.S = p.SS;
        cb.SC = p.SC;
        cb.sbase = (int *)(ws + p.sbase);
        cb.srec = ws + p.srec;
        cb.Fs = ws + p.Fs;
        cb.Gs = ws + p.Gs;
        cb.sdesc = (SuperDesc *)(ws + p.sdesc);
        launch_chunk_desc(b->offsets, c.B, p.L, p.SS, cb.cbase, cb.sbase, 0, p.SC, nullptr,
                          cb.sdesc, s);
        r = run_chunked<R>(sm, od, cb, ll, st, gamma_out, stats, p.S, s);
    }
    if (r != HMM_OK) return fail(r, "unsupported configuration");
    return device_check("E-step kernels");
}

// ---------------------------------------------------------------- profiling
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
thread_local bool g_prof_on = false;
thread_local std::vector<ProfRec> g_prof;
thread_local std::vector<hipEvent_t> g_event_pool;
thread_local size_t g_pool_used = 0;

hipEvent_t pool_event() {
    if (g_pool_used == g_event_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_event_pool.push_back(e);
    }
    return g_event_pool[g_pool_used++];
}

}  // namespace

namespace hmmk {
void prof_begin(const char *name, hipStream_t s) {
    if (!g_prof_on) return;
    ProfRec r{name, pool_event(), pool_event()};
    if (r.a) hipEventRecord(r.a, s);
    g_prof.push_back(r);
}
void prof_end(hipStream_t s) {
    if (!g_prof_on || g_prof.empty()) return;
    if (g_prof.back().b) hipEventRecord(g_prof.back().b, s);
}
}  // namespace hmmk

namespace hmmk {
void launch_argmax_rows(const void *gamma, bool f64, int64_t rows, int N, int32_t *path,
                        hipStream_t s);
}

static size_t theta_len(const hmm_model *m) {
    const size_t N = (size_t)m->n_states, D = (size_t)m->dim;
    switch (m->family) {
    case HMM_GAUSSIAN:
    case HMM_GAMMA: return 2 * N;
    case HMM_STUDENT_T: return 3 * N;
    case HMM_POISSON: return N;
    case HMM_DIAG_GAUSSIAN: return 2 * N * D;
    case HMM_FULL_GAUSSIAN: return N * D + N * D * D;
    default: return 0;
    }
}

namespace hmmk {
hmm_status fail_status(hmm_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

hmm_status model_theta_len(const hmm_model *m, size_t *len) {
    hmm_status st = check_model(m);
    if (st != HMM_OK) return st;
    *len = theta_len(m);
    return HMM_OK;
}
}  // namespace hmmk


// ---------------------------------------------------------------- allocation-free E-step
// The workspace of hmm_estep_stats_noalloc is this file-scope device array.
// Its name is a host-side stand-in in host code: the device address of each
// GPU's copy comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[HMM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hmm_status scratch_for_current_device(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(HMM_ERR_DEVICE, "no current HIP device (or device index %d out of range)", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HMM_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                        hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HMM_OK;
}
}  // namespace

extern "C" {

const char *hmm_version(void) { return "hmmgpu 0.1.0 (gfx950)"; }

const char *hmm_last_error(void) { return g_err.c_str(); }

size_t hmm_stats_len(const hmm_model *model) {
    if (check_model(model) != HMM_OK) return 0;
    int k = family_k(model->family, model->dim);
    int64_t N = model->n_states;
    return (size_t)(1 + 2 * N + N * N + N * k);
}

hmm_status hmm_workspace_size(hmm_op op, const hmm_model *model, const hmm_batch *batch,
                              hmm_precision prec, size_t *bytes) {
    if (!bytes) return fail(HMM_ERR_ARG, "bytes is NULL");
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    // large enough for every variant of the route, so a tuned or forced
    // variant always fits the caller's workspace
    Plan p;
    st = make_plan(op, c, prec, &p, 0);
    if (st != HMM_OK) return st;
    size_t need = p.total;
    const int nv = route_variants(p.route, p.f64);
    for (int v = 1; v < nv; ++v) {
        Plan q;
        if ((st = make_plan(op, c, prec, &q, v)) != HMM_OK) return st;
        if (q.total > need) need = q.total;
    }
    *bytes = need;
    return ok();
}

hmm_status hmm_emission_logpdf(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                               void *log_b, void *ws, size_t ws_bytes, void *stream) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_EMISSION, c, prec, &p)) != HMM_OK) return st;
    if ((st = check_ws(p, ws, ws_bytes)) != HMM_OK) return st;
    if (c.total > 0 && !log_b) return fail(HMM_ERR_ARG, "log_b is NULL");
    hipStream_t s = (hipStream_t)stream;
    ObsDesc od{batch->obs, batch->obs_f64, c.B, batch->offsets};
    if (p.f64) {
        StagedModel<double> sm;
        launch_stage<double>(raw(model), (char *)ws + p.staged, &sm, s);
        run_emission<double>(sm, od, c.total, (double *)log_b, s);
    } else {
        StagedModel<float> sm;
        launch_stage<float>(raw(model), (char *)ws + p.staged, &sm, s);
        run_emission<float>(sm, od, c.total, (float *)log_b, s);
    }
    return device_check("emission kernel");
}

hmm_status hmm_forward_backward(const hmm_model *model, const hmm_batch *batch,
                                hmm_precision prec, double *loglik, void *gamma,
                                int32_t *seq_status, void *ws, size_t ws_bytes, void *stream) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_FORWARD_BACKWARD, c, prec, &p)) != HMM_OK) return st;
    if ((st = check_ws(p, ws, ws_bytes)) != HMM_OK) return st;
    if (c.B > 0 && !loglik) return fail(HMM_ERR_ARG, "loglik is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (p.f64)
        return run_posterior_path<double>(model, batch, c, p, (char *)ws, loglik, seq_status,
                                          gamma, nullptr, s);
    return run_posterior_path<float>(model, batch, c, p, (char *)ws, loglik, seq_status, gamma,
                                     nullptr, s);
}

hmm_status hmm_estep_stats(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                           double *stats, double *loglik, int32_t *seq_status, void *ws,
                           size_t ws_bytes, void *stream) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_ESTEP, c, prec, &p)) != HMM_OK) return st;
    if ((st = check_ws(p, ws, ws_bytes)) != HMM_OK) return st;
    if (!stats) return fail(HMM_ERR_ARG, "stats is NULL");
    hipStream_t s = (hipStream_t)stream;
    if (p.f64)
        return run_posterior_path<double>(model, batch, c, p, (char *)ws, loglik, seq_status,
                                          nullptr, stats, s);
    return run_posterior_path<float>(model, batch, c, p, (char *)ws, loglik, seq_status, nullptr,
                                     stats, s);
}

hmm_status hmm_estep_stats_noalloc(const hmm_model *model, const hmm_batch *batch,
                                   hmm_precision prec, double *stats, double *loglik,
                                   int32_t *seq_status, void *stream) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_ESTEP, c, prec, &p)) != HMM_OK) return st;
    if (p.total > (size_t)HMM_NOALLOC_SCRATCH_BYTES)
        return fail(HMM_ERR_WORKSPACE,
                    "this batch needs %zu bytes of workspace; the allocation-free E-step has a "
                    "static area of %zu bytes (use hmm_estep_stats with a caller workspace)",
                    p.total, (size_t)HMM_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    if ((st = scratch_for_current_device(&ws)) != HMM_OK) return st;
    return hmm_estep_stats(model, batch, prec, stats, loglik, seq_status, ws,
                           (size_t)HMM_NOALLOC_SCRATCH_BYTES, stream);
}

hmm_status hmm_posterior_decode(const hmm_model *model, const hmm_batch *batch,
                                hmm_precision prec, int32_t *path, double *loglik, void *ws,
                                size_t ws_bytes, void *stream) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_POSTERIOR_DECODE, c, prec, &p)) != HMM_OK) return st;
    if ((st = check_ws(p, ws, ws_bytes)) != HMM_OK) return st;
    if (c.total > 0 && !path) return fail(HMM_ERR_ARG, "path is NULL");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    void *gam = w + p.gam;
    int32_t *status = (int32_t *)(w + p.st);
    if (p.f64) st = run_posterior_path<double>(model, batch, c, p, w, loglik, status, gam, nullptr, s);
    else st = run_posterior_path<float>(model, batch, c, p, w, loglik, status, gam, nullptr, s);
    if (st != HMM_OK) return st;
    if (c.total > 0) {
        launch_argmax_rows(gam, p.f64, c.total, c.N, path, s);
        launch_mask_paths(batch->offsets, status, c.B, path, s);
    }
    return device_check("posterior decode");
}

hmm_status hmm_viterbi(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                       int32_t *path, double *path_logp, int32_t *n_ties, void *ws,
                       size_t ws_bytes, void *stream) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_VITERBI, c, prec, &p)) != HMM_OK) return st;
    if ((st = check_ws(p, ws, ws_bytes)) != HMM_OK) return st;
    if (c.total > 0 && !path) return fail(HMM_ERR_ARG, "path is NULL");
    if (c.B > 0 && !path_logp) return fail(HMM_ERR_ARG, "path_logp is NULL");
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    ObsDesc od{batch->obs, batch->obs_f64, c.B, batch->offsets};
    if (c.B == 0) return ok();
    int *cbase = (int *)(w + p.cbase);
    ChunkDesc *cdesc = (ChunkDesc *)(w + p.cdesc);
    int *sbase = (int *)(w + p.sbase);
    SuperDesc *sdesc = (SuperDesc *)(w + p.sdesc);
    launch_plan_chunks(batch->offsets, c.B, 64, p.SS, cbase, sbase, s);
    launch_chunk_desc(batch->offsets, c.B, 64, p.SS, cbase, sbase, p.C, p.SC, cdesc, sdesc, s);
    VitBuffers vb;
    vb.SC = p.SC;
    vb.sbase = sbase;
    vb.sdesc = sdesc;
    vb.vd = w + p.lt;
    vb.voff = (double *)(w + p.lsc);
    vb.J = (double *)(w + p.segJ);
    vb.inc = (double *)(w + p.seginc);
    vb.flag = (int32_t *)(w + p.segbad);
    vb.ver = (int32_t *)(w + p.segver);
    vb.lim = (int32_t *)(w + p.seglim);
    uint8_t *psi = (uint8_t *)(w + p.vpsi), *J = (uint8_t *)(w + p.vJ);
    uint8_t *ql = (uint8_t *)(w + p.vqlast), *qe = (uint8_t *)(w + p.vqend);
    if (p.f64) {
        StagedModel<double> sm;
        launch_stage<double>(raw(model), w + p.staged, &sm, s);
        run_viterbi<double>(sm, od, cbase, cdesc, p.C, vb, psi, J, ql, qe, path, path_logp,
                            n_ties, s);
    } else {
        StagedModel<float> sm;
        launch_stage<float>(raw(model), w + p.staged, &sm, s);
        run_viterbi<float>(sm, od, cbase, cdesc, p.C, vb, psi, J, ql, qe, path, path_logp,
                           n_ties, s);
    }
    return device_check("Viterbi kernels");
}

void hmm_mstep_default_opts(hmm_mstep_opts *o) {
    if (!o) return;
    o->eps_collapse = 1e-8;
    o->ridge = 1e-6;
    o->gamma_rtol = 1e-12;
    o->nu_tol = 1e-6;
    o->nu_min = 0.5;
    o->nu_max = 1e4;
    o->max_iter = 100;
    o->t_nu_printed = 0;
}

static hmm_status mstep_family(int family, const char *name, const hmm_model *model,
                               const double *stats, const hmm_mstep_opts *opts, double *theta_out,
                               int32_t *collapsed, int32_t *iters, void *stream) {
    hmm_status st = check_model(model);
    if (st != HMM_OK) return st;
    if (model->family != family)
        return fail(HMM_ERR_ARG, "%s called for a model of family %d", name, model->family);
    if (!stats || !theta_out) return fail(HMM_ERR_ARG, "%s: stats / theta_out is NULL", name);
    hmm_mstep_opts o;
    if (opts) o = *opts;
    else hmm_mstep_default_opts(&o);
    if (!(o.max_iter >= 1) || !(o.nu_min > 0) || !(o.nu_max >= o.nu_min))
        return fail(HMM_ERR_ARG, "%s: invalid options", name);
    hipStream_t s = (hipStream_t)stream;
    const size_t n = theta_len(model);
    if (theta_out != model->theta) {
        // states that keep their parameters (collapse guard) keep the input values
        hipError_t e = hipMemcpyAsync(theta_out, model->theta, n * sizeof(double),
                                      hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail(HMM_ERR_DEVICE, "%s: copy: %s", name, hipGetErrorString(e));
    }
    launch_mstep_emission(family, model->n_states, model->dim, model->theta, stats, o, theta_out,
                          collapsed, iters, s);
    return device_check(name);
}

hmm_status hmm_mstep_gaussian(const hmm_model *model, const double *stats,
                              const hmm_mstep_opts *opts, double *theta_out, int32_t *collapsed,
                              int32_t *iters, void *stream) {
    return mstep_family(HMM_GAUSSIAN, "hmm_mstep_gaussian", model, stats, opts, theta_out,
                        collapsed, iters, stream);
}
hmm_status hmm_mstep_gamma(const hmm_model *model, const double *stats, const hmm_mstep_opts *opts,
                           double *theta_out, int32_t *collapsed, int32_t *iters, void *stream) {
    return mstep_family(HMM_GAMMA, "hmm_mstep_gamma", model, stats, opts, theta_out, collapsed,
                        iters, stream);
}
hmm_status hmm_mstep_student_t(const hmm_model *model, const double *stats,
                               const hmm_mstep_opts *opts, double *theta_out, int32_t *collapsed,
                               int32_t *iters, void *stream) {
    return mstep_family(HMM_STUDENT_T, "hmm_mstep_student_t", model, stats, opts, theta_out,
                        collapsed, iters, stream);
}
hmm_status hmm_mstep_poisson(const hmm_model *model, const double *stats,
                             const hmm_mstep_opts *opts, double *theta_out, int32_t *collapsed,
                             int32_t *iters, void *stream) {
    return mstep_family(HMM_POISSON, "hmm_mstep_poisson", model, stats, opts, theta_out,
                        collapsed, iters, stream);
}
hmm_status hmm_mstep_diag_gaussian(const hmm_model *model, const double *stats,
                                   const hmm_mstep_opts *opts, double *theta_out,
                                   int32_t *collapsed, int32_t *iters, void *stream) {
    return mstep_family(HMM_DIAG_GAUSSIAN, "hmm_mstep_diag_gaussian", model, stats, opts,
                        theta_out, collapsed, iters, stream);
}
hmm_status hmm_mstep_full_gaussian(const hmm_model *model, const double *stats,
                                   const hmm_mstep_opts *opts, double *theta_out,
                                   int32_t *collapsed, int32_t *iters, void *stream) {
    if (model && model->dim > 64) return fail(HMM_ERR_UNSUPPORTED, "full covariance needs D <= 64");
    return mstep_family(HMM_FULL_GAUSSIAN, "hmm_mstep_full_gaussian", model, stats, opts,
                        theta_out, collapsed, iters, stream);
}

hmm_status hmm_mstep_transitions(const hmm_model *model, const double *stats,
                                 const hmm_mstep_opts *opts, double *log_pi_out,
                                 double *log_A_out, void *stream) {
    hmm_status st = check_model(model);
    if (st != HMM_OK) return st;
    if (!stats || !log_pi_out || !log_A_out)
        return fail(HMM_ERR_ARG, "hmm_mstep_transitions: NULL pointer");
    hmm_mstep_opts o;
    if (opts) o = *opts;
    else hmm_mstep_default_opts(&o);
    launch_mstep_trans(model->n_states, stats, model->log_A, o.eps_collapse, log_pi_out, log_A_out,
                       (hipStream_t)stream);
    return device_check("hmm_mstep_transitions");
}

hmm_status hmm_profile_enable(int32_t on) {
    g_prof_on = on != 0;
    g_prof.clear();
    g_pool_used = 0;
    return ok();
}

int32_t hmm_profile_count(void) { return (int32_t)g_prof.size(); }

hmm_status hmm_profile_get(int32_t i, const char **name, float *ms) {
    if (i < 0 || i >= (int32_t)g_prof.size() || !name || !ms)
        return fail(HMM_ERR_ARG, "profile record %d does not exist", i);
    *name = g_prof[i].name;
    hipError_t e = hipEventSynchronize(g_prof[i].b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, g_prof[i].a, g_prof[i].b);
    if (e != hipSuccess) return fail(HMM_ERR_DEVICE, "profile event: %s", hipGetErrorString(e));
    return ok();
}

hmm_status hmm_profile_reset(void) {
    g_prof.clear();
    g_pool_used = 0;
    return ok();
}

hmm_status hmm_set_variant(int32_t variant) {
    if (variant < -1) return fail(HMM_ERR_ARG, "variant must be -1 (tuned) or >= 0");
    force_variant();   // read the environment first so it cannot overwrite this
    g_force_variant.store(variant);
    return ok();
}

hmm_status hmm_get_variant(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                           int32_t *variant, int32_t *n_variants) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    Plan p;
    if ((st = make_plan(HMM_OP_ESTEP, c, prec, &p)) != HMM_OK) return st;
    if (variant) *variant = p.variant;
    if (n_variants) *n_variants = route_variants(p.route, p.f64);
    return ok();
}

hmm_status hmm_autotune(const hmm_model *model, const hmm_batch *batch, hmm_precision prec,
                        double *stats, double *loglik, int32_t *seq_status, void *ws,
                        size_t ws_bytes, void *stream, int32_t *variant, float *ms) {
    Checked c;
    hmm_status st = check_batch(batch, model, &c);
    if (st != HMM_OK) return st;
    if (!stats) return fail(HMM_ERR_ARG, "stats is NULL");
    Plan p0;
    if ((st = make_plan(HMM_OP_ESTEP, c, prec, &p0, 0)) != HMM_OK) return st;
    const int nv = route_variants(p0.route, p0.f64);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return fail(HMM_ERR_DEVICE, "hmm_autotune: cannot create events");
    }
    float t[4] = {0, 0, 0, 0};
    hmm_status r = HMM_OK;
    for (int v = 0; v < nv && r == HMM_OK; ++v) {
        Plan p;
        if ((r = make_plan(HMM_OP_ESTEP, c, prec, &p, v)) != HMM_OK) break;
        if ((r = check_ws(p, ws, ws_bytes)) != HMM_OK) break;
        float rep[3];
        for (int k = 0; k < 4 && r == HMM_OK; ++k) {   // one warm-up, three timed
            hipEventRecord(e0, s);
            r = p.f64 ? run_posterior_path<double>(model, batch, c, p, (char *)ws, loglik,
                                                   seq_status, nullptr, stats, s)
                      : run_posterior_path<float>(model, batch, c, p, (char *)ws, loglik,
                                                  seq_status, nullptr, stats, s);
            hipEventRecord(e1, s);
            if (r == HMM_OK && hipEventSynchronize(e1) != hipSuccess)
                r = fail(HMM_ERR_DEVICE, "hmm_autotune: E-step failed on the device");
            if (r == HMM_OK && k > 0) hipEventElapsedTime(&rep[k - 1], e0, e1);
        }
        if (r != HMM_OK) break;
        // median of the three
        float a = rep[0], b = rep[1], d = rep[2];
        t[v] = a > b ? (b > d ? b : (a > d ? d : a)) : (a > d ? a : (b > d ? d : b));
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (r != HMM_OK) return r;
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (t[v] < t[best]) best = v;
    tune_store(c, prec, p0.route, best, t, nv);
    if (variant) *variant = best;
    if (ms)
        for (int v = 0; v < nv; ++v) ms[v] = t[v];
    return ok();
}

hmm_status hmm_set_chunk_len(int32_t steps) {
    if (steps != 0 && steps != 16 && steps != 32 && steps != 64)
        return fail(HMM_ERR_ARG, "chunk length must be 0, 16, 32 or 64");
    g_chunk_len.store(steps);
    return ok();
}

}  // extern "C"
