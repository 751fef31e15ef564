// k_chunk.hip -- batched forward-backward E-step for small state counts
// (N <= 8), exact and time-parallel.
//
// The forward recursion of section 3.2, alpha_t(j) = lse_i[alpha_{t-1}(i) +
// log a_ij] + log b_j(y_t), is carried in linear form on a normalised vector
// with an exact log offset:  alpha_t = (alpha_{t-1} A) o e_t, where
// e_t(j) = exp(log b_j(y_t) - m_t) and m_t = max_j log b_j(y_t); every step
// is rescaled by a power of two (exact) and the exponents and the m_t are
// summed on the side.  Writing M_t = A diag(e_t), a sequence is cut into
// chunks of L steps and each chunk's transfer matrix P_c = prod_{t in c} M_t
// is formed independently (phase 1), together with the product of each
// superchunk of 16 consecutive chunks.  Then, per sequence, the boundary
// vectors alpha_{end(c)} = alpha_{end(c-1)} P_c and beta_{end(c-1)} = P_c
// beta_{end(c)} follow from a short serial scan over superchunks, and within
// each superchunk from a serial scan over its chunks (phase 2).
// Finally every chunk re-runs its own L forward steps from its boundary and
// the backward recursion beta_{t-1} = M_t beta_t down to its start, forming
// gamma_t and xi_t (definitions of section 3.1) and accumulating the
// gamma-weighted statistics of section 4 (phase 3).  The result equals the
// sequential recursion up to rounding; phase 1 costs N^3 per step instead of
// N^2 but has no serial dependency between chunks.
//
// Lanes: a chunk occupies G lanes in every phase (phase 1: lane = row of its
// transfer matrix; phases 2 and 3: lane = state).  G = 4 (N <= 4) or 8 (N <= 8); the lane exchanges
// inside a group of G lanes are DPP quad permutations and the half-row mirror.
#include <climits>

#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

struct ChunkGeom {
    int64_t nseq;
    const int64_t *offsets;
    const int *cbase;
    const SuperDesc *sdesc;   // chunk i of superchunk k: index sdesc[k].lo + i
    int SC;
    int L;
    int C;
    ObsRef obs;
};

constexpr int NEG_EXP = INT_MIN / 4;

// one observation (scalar families) or one log b_j entry (table family)
template <int FAM, typename R>
__device__ __forceinline__ R load_step(const ObsRef &o, int64_t row, int j, int N, bool live) {
    if constexpr (FAM == HMM_TABLE) {
        return live ? load_obs<R>(o, row * N + j) : neg_inf<R>();
    } else {
        return load_obs<R>(o, row);
    }
}

template <int FAM, typename R>
__device__ __forceinline__ Emit<R> emit_step(R v, const StateConsts<R> &k, bool live) {
    if constexpr (FAM == HMM_TABLE) {
        Emit<R> e;
        e.ell = live ? v : neg_inf<R>();
        e.common = 0.0;
        e.bad = live && (isnan(v) || (v > (R)0 && isinf(v)));
        return e;
    } else {
        return emit_scalar<FAM, R>(v, k, live);
    }
}

// Transfer-matrix records of a chunk (or of a superchunk of 16 chunks), one
// per lane of a G-lane group, stored once and read by both boundary scans:
// with P = diag(2^r) P~ (each nonzero row of P~ with its largest entry in
// [1/2, 1)), lane p's record holds column p of P~ in grp_dot order,
// coef[k] = P~[src(p, k)][p], the exponent r[p] of row p and the summed log
// shift m_t of the steps covered (NaN after a non-finite observation).  The
// forward scan forms f P with grp_dot, the backward scan P g with grp_tdot
// from the same coefficients.
template <typename R, int G>
struct __align__(16) ColRec {
    R coef[G];
    int r;
    int pad;
    double clog;
};

size_t chunk_rec_bytes(bool f64, int G) {
    return f64 ? (G == 8 ? sizeof(ColRec<double, 8>) : sizeof(ColRec<double, 4>))
               : (G == 8 ? sizeof(ColRec<float, 8>) : sizeof(ColRec<float, 4>));
}

// lane li writes its record from the natural-order matrix rows in LDS
template <typename R, int G, int RS>
__device__ __forceinline__ void store_colrec(ColRec<R, G> *dst, const R (*rows)[RS], int li,
                                             int r, double clog) {
    ColRec<R, G> f;
#pragma unroll
    for (int k = 0; k < G; ++k) f.coef[k] = rows[grp_src(li, k)][li];
    f.r = r;
    f.pad = 0;
    f.clog = clog;
    *dst = f;
}

// ---------------------------------------------------------------- phase 1
// One lane per row of a chunk's transfer matrix (G lanes per chunk): the
// lane keeps its row in registers and multiplies it by A diag(e_t) with A
// uniform across the block, so the product needs no lane exchange at all.
// The chunk's emissions e_t(j) are first tabulated in LDS, lane i taking the
// steps i, i + G, ... (all states of a step in one lane, so the per-step
// maximum is a local reduction).  A block holds whole superchunks (SPC = 16
// consecutive chunks of one sequence, slot i of a superchunk = its chunk i):
// after writing the chunk records it multiplies the superchunk's chunk
// matrices in a pairwise tree through LDS (slot i takes slot i + h at stride
// h = 1, 2, 4, 8) and writes the superchunk record, so the boundary scan over
// superchunks needs no separate pass over the chunk records.
constexpr int SPC = 16;

// row <- row A diag(e) for one step (e: the step's G emission factors)
template <typename R, int G>
__device__ __forceinline__ void product_step(const R (&a)[G][G], const R *e, R (&rowv)[G]) {
    R nv[G];
#pragma unroll
    for (int j = 0; j < G; ++j) {
        R acc = rowv[0] * a[0][j];
#pragma unroll
        for (int k = 1; k < G; ++k) acc = fma(rowv[k], a[k][j], acc);
        nv[j] = acc * e[j];
    }
#pragma unroll
    for (int j = 0; j < G; ++j) rowv[j] = nv[j];
}

// divide the row by 2^ex (ex = exponent of its largest entry), add ex to r
template <typename R, int G>
__device__ __forceinline__ void rescale_row(R (&rowv)[G], int &r) {
    R mxv = rowv[0];
#pragma unroll
    for (int j = 1; j < G; ++j) mxv = fmax(mxv, rowv[j]);
    const int ex = fexp(mxv);
#pragma unroll
    for (int j = 0; j < G; ++j) rowv[j] = fldexp(rowv[j], -ex);
    r += ex;
}

// nsteps product steps over the emission table es ([step][G]), rescaled after
// every NRM-th step and after the last
template <typename R, int G, int NRM>
__device__ __forceinline__ void product_steps(const R (&a)[G][G], const R *es, int nsteps,
                                              R (&rowv)[G], int &r) {
    int s = 0;
    for (; s + NRM <= nsteps; s += NRM) {
#pragma unroll
        for (int u = 0; u < NRM; ++u) product_step<R, G>(a, es + (s + u) * G, rowv);
        rescale_row<R, G>(rowv, r);
    }
    if (s < nsteps) {
        for (; s < nsteps; ++s) product_step<R, G>(a, es + s * G, rowv);
        rescale_row<R, G>(rowv, r);
    }
}


template <typename R, int G, int L, int FAM>
__global__ __launch_bounds__(BLOCK) void k_chunk_product(ChunkGeom g, const SuperDesc *__restrict__ sdesc,
                                                         int SC, StagedModel<R> m,
                                                         const R *__restrict__ A8,
                                                         ColRec<R, G> *__restrict__ rec,
                                                         ColRec<R, G> *__restrict__ srec) {
    constexpr int CPB = BLOCK / G;   // chunks per block
    constexpr int SPB = CPB / SPC;   // superchunks per block
    static_assert(SPB * SPC == CPB, "a block holds whole superchunks");
    // A slot's emission table (L x G) is dead once its product loop ends, so
    // its product rows (G rows padded to G + 4 entries, 16-byte aligned for
    // vector reads in the tree) take the same space: every lane of a wave
    // leaves the loop before any of them stores its row.
    constexpr int RS = G + 4;
    static_assert(G * RS <= L * G, "product rows fit in the emission table");
    __shared__ __align__(16) R eps[CPB][L * G];
    R (*esh)[L][G] = reinterpret_cast<R (*)[L][G]>(&eps[0][0]);
    auto psh = [&](int q) { return reinterpret_cast<R (*)[RS]>(&eps[q][0]); };
    __shared__ double msh[CPB][G];
    __shared__ __align__(16) int rsh[CPB][G];
    __shared__ double csh[CPB];
    __shared__ int nscs[SPB];

    const int li = threadIdx.x % G;
    const int slot = threadIdx.x / G;
    const int si = slot % SPC;                        // chunk index inside its superchunk
    const int sc = blockIdx.x * SPB + slot / SPC;     // superchunk
    int nsc = 0, c = 0, t0 = 0, len = 0;
    int64_t off = 0;
    if (sc < SC) {
        const SuperDesc sd = sdesc[sc];
        nsc = sd.n;
        c = sd.lo + si;
        off = sd.off;
        t0 = sd.t0 + si * L;
        len = min(L, sd.T - t0);
    }
    const bool valid = si < nsc;
    const int N = m.N;
    int ts = 0, nsteps = 0;
    if (valid) {
        ts = max(t0, 1);
        nsteps = max(t0 + len - ts, 0);
    }
    using ET = typename EmitTraits<FAM, R>::T;
    const ET *ep = consts_ptr<FAM, R>(m);

    // emissions: e_t(j) = exp(log b_j(y_t) - max_j log b_j(y_t))
    // per-state constants held across the step loop (Poisson's FP64 ones are
    // re-read instead: held, they would raise the register count)
    StateConsts<ET> kc[G];
    if constexpr (FAM != HMM_POISSON) {
#pragma unroll
        for (int j = 0; j < G; ++j) kc[j] = load_consts_row(ep, j < N ? j : 0);   // dead states masked by emit_step
    }
    double msum = 0.0;
    bool bad = false;
    // scalar families: one observation per step, shared by all states; a
    // lane's observations are all loaded up front (clamped rows, so the loads
    // are unconditional and in flight together)
    constexpr int NI = L / G;   // steps a lane tabulates, at most
    R ypre[FAM != HMM_TABLE ? NI : 1];
    if constexpr (FAM != HMM_TABLE) {
        const int64_t rlast = off + ts + max(nsteps - 1, 0);
#pragma unroll
        for (int k = 0; k < NI; ++k) ypre[k] = load_obs<R>(g.obs, min(off + ts + li + k * G, rlast));
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) {
        const int tt = li + k * G;
        if (tt >= nsteps) break;
        const int64_t row = off + ts + tt;
        ET ell[G];
        ET mx = neg_inf<ET>();
        double common = 0.0;
        const R y = (FAM != HMM_TABLE) ? ypre[FAM != HMM_TABLE ? k : 0] : (R)0;
#pragma unroll
        for (int j = 0; j < G; ++j) {
            const bool live = j < N;
            R v = (FAM != HMM_TABLE) ? y : load_step<FAM, R>(g.obs, row, j, N, live);
            StateConsts<ET> kj;
            if constexpr (FAM == HMM_POISSON) kj = load_consts(ep, j, live);
            else kj = kc[j];
            Emit<ET> em = emit_step<FAM, ET>((ET)v, kj, live);
            ell[j] = em.ell;
            mx = fmax(mx, em.ell);
            bad |= em.bad;
            common = em.common;
        }
#pragma unroll
        for (int j = 0; j < G; ++j)
            esh[slot][tt][j] = (ell[j] == neg_inf<ET>()) ? (R)0 : fexp_e((R)(ell[j] - mx));
        msum += (double)mx + common;
    }
    msh[slot][li] = bad ? __builtin_nan("") : msum;
    R a[G][G];
#pragma unroll
    for (int k = 0; k < G; ++k)
#pragma unroll
        for (int j = 0; j < G; ++j) a[k][j] = A8[k * 8 + j];
    const int nrm = *m.nrm;
    __syncthreads();

    R rowv[G];
#pragma unroll
    for (int j = 0; j < G; ++j) rowv[j] = (j == li && li < N) ? (R)1 : (R)0;
    int r = 0;
    // nrm (1, 2 or 4) is uniform: each variant runs nrm unrolled steps between
    // rescales, and the row leaves rescaled whatever its step count
    const R *es = &esh[slot][0][0];
    if (nrm == 4) product_steps<R, G, 4>(a, es, nsteps, rowv, r);
    else if (nrm == 2) product_steps<R, G, 2>(a, es, nsteps, rowv, r);
    else product_steps<R, G, 1>(a, es, nsteps, rowv, r);
    double cl = 0.0;
#pragma unroll
    for (int q = 0; q < G; ++q) cl += msh[slot][q];
#pragma unroll
    for (int j = 0; j < G; ++j) psh(slot)[li][j] = rowv[j];
    rsh[slot][li] = r;
    if (li == 0) csh[slot] = cl;
    __syncthreads();
    if (valid) store_colrec<R, G, RS>(rec + (size_t)c * G + li, psh(slot), li, r, cl);

    // pairwise tree over each superchunk's chunks, slot i taking slot i + h at
    // h = 1, 2, 4, 8.  A level's products are spread over the block's first
    // lanes, one lane per row of a product (128 / h lanes), rather than kept on
    // the lanes of the left slot, so that a level issues its work on as few
    // waves as it needs; rows and exponents stay in LDS.  A level reads only
    // slots with i % 2h == h and writes only slots with i % 2h == 0, so one
    // barrier per level orders it; the first also orders the chunk records'
    // reads of the rows before the first level's writes.
    if (li == 0 && si == 0) nscs[slot / SPC] = nsc;
#pragma unroll
    for (int h = 1; h < SPC; h *= 2) {
        __syncthreads();
        const int ppb = SPC / (2 * h);   // products per superchunk at this level
        const int task = threadIdx.x;
        if (task < SPB * ppb * G) {
            const int tl = task % G, pidx = task / G;
            const int sp = pidx / ppb, pi = pidx % ppb;
            const int lft = sp * SPC + pi * 2 * h, o = lft + h;
            if (pi * 2 * h + h < nscs[sp]) {
                // row tl of (2^r P~)(2^r' P~') with the row exponents combined
                // exactly; every operand is read unconditionally, so the tests
                // below are selects
                R rw[G];
                int ro[G];
#pragma unroll
                for (int k = 0; k < G; ++k) {
                    rw[k] = psh(lft)[tl][k];
                    ro[k] = rsh[o][k];
                }
                int Rm = NEG_EXP;
#pragma unroll
                for (int k = 0; k < G; ++k)
                    Rm = max(Rm, (rw[k] > (R)0) ? fexp(rw[k]) + ro[k] : NEG_EXP);
                if (Rm != NEG_EXP) {
                    R nv[G];
#pragma unroll
                    for (int j = 0; j < G; ++j) nv[j] = (R)0;
#pragma unroll
                    for (int k = 0; k < G; ++k) {
                        const R wk = (rw[k] > (R)0) ? fldexp(rw[k], ro[k] - Rm) : (R)0;
#pragma unroll
                        for (int j = 0; j < G; ++j) nv[j] = fma(wk, psh(o)[k][j], nv[j]);
                    }
                    R mx = nv[0];
#pragma unroll
                    for (int j = 1; j < G; ++j) mx = fmax(mx, nv[j]);
                    const int ex = fexp(mx);
#pragma unroll
                    for (int j = 0; j < G; ++j) psh(lft)[tl][j] = fldexp(nv[j], -ex);
                    rsh[lft][tl] += Rm + ex;
                }
                if (tl == 0) csh[lft] += csh[o];
            }
        }
    }
    __syncthreads();
    if (si == 0 && nsc > 0)
        store_colrec<R, G, RS>(srec + (size_t)sc * G + li, psh(slot), li, rsh[slot][li], csh[slot]);
}

// ---------------------------------------------------------------- phase 2
// Serial scans over records, G lanes per segment.  EXPAND = false: a segment
// is a sequence and the records are its superchunks (boundary vectors at
// superchunk ends, log-likelihood, status).  EXPAND = true: a segment is a
// superchunk and the records are its chunks, started from the superchunk
// boundaries found by the first pass.  The records of the next PF steps are
// kept in flight (software prefetch).
struct ScanGeom {
    int64_t nseq;
    const int64_t *offsets;
    const int *cbase;    // [B+1] chunks per sequence (prefix)
    const int *sbase;    // [B+1] superchunks per sequence (prefix)
    int S;               // chunks per superchunk
    int SC;              // number of superchunks
    int C;               // number of chunks
    const SuperDesc *sdesc;
    ObsRef obs;
};

// alpha_0 = pi o e_0 of sequence b, rescaled; returns its log offset and flags
template <typename R, int G, int FAM>
__device__ __forceinline__ R alpha0(const StagedModel<R> &m, const ObsRef &obs, int64_t off,
                                    bool valid, int p, double *logS, int *E, bool *bad) {
    const int N = m.N;
    const bool live = p < N;
    using ET = typename EmitTraits<FAM, R>::T;
    const StateConsts<ET> k = load_consts(consts_ptr<FAM, R>(m), p, live);
    R v0 = valid ? load_step<FAM, R>(obs, off, p, N, live) : (R)1;
    Emit<ET> em = emit_step<FAM, ET>((ET)v0, k, live);
    ET mx = grp_max<G, ET>(em.ell);
    R e = (em.ell == neg_inf<ET>()) ? (R)0 : fexp_e((R)(em.ell - mx));
    R f = (live ? m.pi[p] : (R)0) * e;
    *logS = (double)mx + em.common;
    *bad = grp_max_i<G>(em.bad ? 1 : 0) > 0;
    const int ex0 = fexp(grp_max_pos<G>(f));
    *E = ex0;
    return fldexp(f, -ex0);
}

template <typename R, int G, int FAM, int PF, bool EXPAND>
__global__ __launch_bounds__(BLOCK) void k_chunk_scan(ScanGeom g, StagedModel<R> m,
                                                      const ColRec<R, G> *__restrict__ rec,
                                                      const R *__restrict__ Fs,
                                                      const R *__restrict__ Gs,
                                                      R *__restrict__ Fo, R *__restrict__ Go,
                                                      double *__restrict__ loglik,
                                                      int32_t *__restrict__ status) {
    constexpr int SPW = 64 / G;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / G, p = lane % G;
    // odd waves run the backward scan over the segments of the even wave
    // before them, so both directions read a record at about the same time on
    // the same compute unit (one fetch from memory serves both)
    const bool fwd = (wave & 1) == 0;
    const int64_t seg = ((int64_t)blockIdx.x * (BLOCK / 128) + (wave >> 1)) * SPW + sub;
    const bool valid = seg < (EXPAND ? (int64_t)g.SC : g.nseq);
    const bool live = p < m.N;
    int lo = 0, n = 0;
    int64_t b = 0;
    bool head = true;   // EXPAND: the segment is its sequence's first superchunk
    // outputs of a lane group past the last segment go to the sink slot after
    // the last record, so every store is unconditional
    const int sink = EXPAND ? g.C : g.SC;
    if (valid) {
        if (EXPAND) {
            const SuperDesc d = g.sdesc[seg];
            b = d.b;
            lo = d.lo;
            n = d.n;
            head = d.head != 0;
        } else {
            b = seg;
            lo = g.sbase[b];
            n = g.sbase[b + 1] - lo;
        }
    }
    const int nmax = wave_max_i(n);

    if (fwd) {
        // forward: f <- f P_c over the segment's records
        double logS = 0.0;
        int E0 = 0;
        bool bad = false;
        const int64_t off = valid ? g.offsets[b] : 0;
        R f;
        if (!EXPAND || head) {
            f = alpha0<R, G, FAM>(m, g.obs, off, valid, p, &logS, &E0, &bad);
        } else {
            f = (R)0;
        }
        if (EXPAND && !head && valid) f = Fs[(size_t)(seg - 1) * G + p];
        int64_t E = E0;
        // loads run PF records ahead with indices clamped into the segment
        // (always in bounds, so they need no branch and their waits stay exact)
        const int lastf = lo + max(n - 1, 0);
        const int64_t fsl = valid ? -1 : (int64_t)sink;   // store slot override
        ColRec<R, G> ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) ring[q] = rec[(size_t)min(lo + q, lastf) * G + p];
        for (int s0 = 0; s0 < nmax; s0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int s = s0 + q;
                const bool act = s < n;
                const ColRec<R, G> cur = ring[q];
                ring[q] = rec[(size_t)min(lo + s + PF, lastf) * G + p];
                const int rr = act ? cur.r : 0;
                const int ce = (f > (R)0) ? fexp(f) + rr : NEG_EXP;
                const int Rm = grp_max_i<G>(ce);
                R w = (f > (R)0 && act) ? fldexp(f, rr - Rm) : (R)0;
                R coef[G];
#pragma unroll
                for (int kk = 0; kk < G; ++kk) coef[kk] = cur.coef[kk];
                R v = grp_dot<G, R>(w, coef);
                int ev = fexp(grp_max_pos<G>(v));
                v = fldexp(v, -ev);
                if (act) {
                    f = v;
                    E += (int64_t)Rm + ev;
                    logS += cur.clog;
                }
                const int64_t slot_f = fsl >= 0 ? fsl : (int64_t)min(lo + s, lastf);
                Fo[(size_t)slot_f * G + p] = f;
            }
        }
        if (!EXPAND) {
            R tot = grp_sum<G, R>(f);
            if (valid && p == 0) {
                double ll;
                int st;
                if (*m.perr) {
                    ll = __builtin_nan("");
                    st = 4;
                } else if (bad || isnan(logS)) {
                    ll = __builtin_nan("");
                    st = 2;
                } else if (!(tot > (R)0) || isinf(logS)) {
                    ll = -__builtin_inf();
                    st = 1;
                } else {
                    ll = logS + (double)E * 0.69314718055994530942 + log((double)tot);
                    st = 0;
                }
                loglik[b] = ll;
                status[b] = st;
            }
        }
    } else {
        // backward: g <- P_c g, from the segment's last record down to its second
        R gv = live ? (R)1 : (R)0;
        if (EXPAND && valid) gv = Gs[(size_t)seg * G + p];
        const int64_t gsl = valid ? -1 : (int64_t)sink;
        Go[(size_t)(gsl >= 0 ? gsl : (int64_t)(lo + n - 1)) * G + p] = gv;
        const int nb = n - 1;
        const int top = lo + max(n - 1, 0);
        ColRec<R, G> ring[PF];
#pragma unroll
        for (int q = 0; q < PF; ++q) ring[q] = rec[(size_t)max(top - q, lo) * G + p];
        for (int s0 = 0; s0 + 1 < nmax; s0 += PF) {
#pragma unroll
            for (int q = 0; q < PF; ++q) {
                const int s = s0 + q;
                const bool act = s < nb;
                const ColRec<R, G> cur = ring[q];
                ring[q] = rec[(size_t)max(top - (s + PF), lo) * G + p];
                R coef[G];
#pragma unroll
                for (int kk = 0; kk < G; ++kk) coef[kk] = act ? cur.coef[kk] : (R)0;
                const int rr = act ? cur.r : 0;
                R v = grp_tdot<G, R>(gv, coef);
                const int ce = (v > (R)0) ? fexp(v) + rr : NEG_EXP;
                const int Rm = grp_max_i<G>(ce);
                v = (v > (R)0) ? fldexp(v, rr - Rm) : (R)0;
                if (act) gv = v;
                const int64_t slot_g = gsl >= 0 ? gsl : (int64_t)max(top - 1 - s, lo);
                Go[(size_t)slot_g * G + p] = gv;
            }
        }
    }
}

// ---------------------------------------------------------------- phase 3
// One chunk per G-lane group (lane = state), 64/G chunks per wave.  Per round:
//  1. the chunk's emission factors e_t(j) are tabulated in LDS, lane p taking
//     the steps p, p + G, ... (all states of a step in one lane, so the
//     per-step maximum is local), together with y_t and log y_t;
//  2. each lane copies its own state's column e_t(p) into registers;
//  3. forward from the boundary alpha_{end(c-1)} (or pi o e_0), keeping the
//     alpha history in the same LDS table;
//  4. backward from the boundary beta_{end(c)}, forming gamma and xi and the
//     family statistics.
// The chunk occupies slots tt0 .. L-1 of the L-step frame (tt0 = L - length),
// so a short final chunk is aligned to the end of the frame.
template <typename R, int G, int L, int FAM>
struct StatsLds {
    static constexpr int GPB = (BLOCK / 64) * (64 / G);
    static constexpr int K = fam_k<FAM>();
    static constexpr int NV = G + 2 + K;
    static constexpr size_t tab = sizeof(R) * GPB * L * G;
    static constexpr size_t ysz = sizeof(R) * GPB * L * 2;
    static constexpr size_t red = sizeof(double) * GPB * G * NV;
    // G = 8: each group exchanges its vector through LDS (one store, two
    // broadcast reads) instead of seven DPP moves on the vector ALU
    static constexpr bool XL = G == 8;
    static constexpr size_t xsz = XL ? sizeof(R) * GPB * G : 0;
    static constexpr size_t loop = 2 * tab + ysz + xsz;
    static constexpr size_t bytes = loop > red ? loop : red;
};

// all G entries of the group's vector in state order (lane p stores x into
// the group's slot xs)
template <typename R, int G>
__device__ __forceinline__ void lds_vec(R x, R *xs, int p, R (&out)[G]) {
    xs[p] = x;
    wave_lds_order();
#pragma unroll
    for (int j = 0; j < G; ++j) out[j] = xs[j];
    wave_lds_order();
}

template <typename R, int G, int L, int FAM, bool WG>
__global__ __launch_bounds__(BLOCK) void k_chunk_stats(ChunkGeom g, StagedModel<R> m,
                                                       const R *__restrict__ Fi,
                                                       const R *__restrict__ Gi,
                                                       const int32_t *__restrict__ status,
                                                       double *__restrict__ partial,
                                                       R *__restrict__ gamma_out, int64_t S) {
    using LD = StatsLds<R, G, L, FAM>;
    constexpr int K = LD::K;
    constexpr int KK = K > 0 ? K : 1;
    constexpr int GPW = 64 / G, GPB = LD::GPB;
    constexpr int NV = LD::NV;
    __shared__ __align__(16) unsigned char lds_raw[LD::bytes];
    R (*tab)[L][G] = reinterpret_cast<R (*)[L][G]>(lds_raw);             // e_t(j)
    R (*atab)[L][G] = reinterpret_cast<R (*)[L][G]>(lds_raw + LD::tab);  // alpha history
    R (*ysh)[L][2] = reinterpret_cast<R (*)[L][2]>(lds_raw + 2 * LD::tab);
    constexpr bool XL = LD::XL;
    R (*xsh)[G] = reinterpret_cast<R (*)[G]>(lds_raw + 2 * LD::tab + LD::ysz);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int sub = lane / G, p = lane % G, grp = wave * GPW + sub;
    const int N = m.N;
    const bool live = p < N;
    using ET = typename EmitTraits<FAM, R>::T;
    const ET *ep = consts_ptr<FAM, R>(m);
    const StateConsts<ET> k = load_consts(ep, p, live);
    StateConsts<ET> kc[G];   // as in phase 1
    if constexpr (FAM != HMM_POISSON) {
#pragma unroll
        for (int j = 0; j < G; ++j) kc[j] = load_consts_row(ep, j < N ? j : 0);   // dead states masked by emit_step
    }
    R coefC[G], coefR[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        // state order for the LDS exchange, grp_dot order for DPP
        int i = XL ? q : grp_src(p, q);
        // clamped unconditional loads, masked once all are in flight
        const int ic = min(i, N - 1), pc = min(p, N - 1);
        coefC[q] = m.A[ic * N + pc];
        coefR[q] = m.A[pc * N + ic];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const int i = XL ? q : grp_src(p, q);
        const bool in = live && i < N;
        coefC[q] = in ? coefC[q] : (R)0;
        coefR[q] = in ? coefR[q] : (R)0;
    }
    const R pi_p = live ? m.pi[p] : (R)0;
    const int nrm = *m.nrm;

    double xacc[G], g1acc = 0.0, gsacc = 0.0, facc[KK];
#pragma unroll
    for (int q = 0; q < G; ++q) xacc[q] = 0.0;
#pragma unroll
    for (int q = 0; q < KK; ++q) facc[q] = 0.0;

    // a round takes whole superchunks, lane group si of a superchunk its
    // chunk si (groups past a short superchunk's end idle)
    constexpr int SPB = GPB / SPC;
    static_assert(SPB * SPC == GPB, "a block holds whole superchunks");
    const int si = grp % SPC;
    const int per_round = gridDim.x * SPB;
    const int nrounds = (g.SC + per_round - 1) / per_round;
    for (int rnd = 0; rnd < nrounds; ++rnd) {
        const int sc = (rnd * (int)gridDim.x + (int)blockIdx.x) * SPB + grp / SPC;
        bool valid = false;
        int c = 0, t0 = 0, len = 0;
        int64_t off = 0;
        bool use = false;
        if (sc < g.SC) {
            const SuperDesc d = g.sdesc[sc];
            valid = si < d.n;
            c = d.lo + si;
            off = d.off;
            t0 = d.t0 + si * L;
            len = valid ? min(L, d.T - t0) : 0;
            use = valid && status[d.b] == 0;
        }
        const int tt0 = L - len;
        const bool first = (t0 == 0);

        // 1. emission table (lane p takes frame slots p, p + G, ...)
        // a lane's observations loaded up front at clamped rows (unconditional
        // loads, in flight together)
        constexpr int NI = L / G;
        R ypre[FAM != HMM_TABLE ? NI : 1];
        if constexpr (FAM != HMM_TABLE) {
#pragma unroll
            for (int k = 0; k < NI; ++k) {
                const int tt = p + k * G;
                ypre[k] = load_obs<R>(g.obs, (valid && tt >= tt0) ? off + t0 + (tt - tt0) : off + t0);
            }
        }
        // the chunk's boundary vectors, requested after the observations (the
        // load counter drains in order) so that their latency overlaps the
        // emission table (clamped rows: unconditional loads)
        const int cc = min(c, g.C - 1);
        const R ap_in = Fi[(size_t)max(cc - 1, 0) * G + p];
        const R gi_in = Gi[(size_t)cc * G + p];
#pragma unroll
        for (int k = 0; k < NI; ++k) {
            const int tt = p + k * G;
            const bool act = valid && tt >= tt0;
            const int64_t row = off + t0 + (tt - tt0);
            ET ell[G];
            ET mx = neg_inf<ET>();
            R y1 = (R)1;
            const R y = (FAM != HMM_TABLE && act) ? ypre[FAM != HMM_TABLE ? k : 0] : (R)1;
#pragma unroll
            for (int j = 0; j < G; ++j) {
                const bool lj = j < N;
                R v = (FAM != HMM_TABLE) ? y : (act ? load_step<FAM, R>(g.obs, row, j, N, lj) : (R)1);
                if (j == 0) y1 = v;
                StateConsts<ET> kj;
                if constexpr (FAM == HMM_POISSON) kj = load_consts(ep, j, lj);
                else kj = kc[j];
                Emit<ET> em = emit_step<FAM, ET>((ET)v, kj, lj);
                ell[j] = em.ell;
                mx = fmax(mx, em.ell);
            }
#pragma unroll
            for (int j = 0; j < G; ++j)
                tab[grp][tt][j] =
                    (act && ell[j] != neg_inf<ET>()) ? fexp_e((R)(ell[j] - mx)) : (R)0;
            ysh[grp][tt][0] = y1;
            ysh[grp][tt][1] = (FAM == HMM_GAMMA && y1 > (R)0) ? flog(y1) : (R)0;
        }
        __syncthreads();

        // 3. forward from the chunk's boundary; alpha history into LDS
        const R ap = (valid && !first) ? ap_in : (R)0;
        R start;
        {
            R v = pi_p * tab[grp][tt0 < L ? tt0 : L - 1][p];   // tt0 = L: idle group
            start = fldexp(v, -fexp(grp_max_pos<G>(v)));
        }
        R acur = ap;
#pragma unroll 4
        for (int tt = 0; tt < L; ++tt) {
            const R xin = (tt == tt0) ? ap : acur;
            R d;
            if constexpr (XL) {
                R xa[G];
                lds_vec<R, G>(xin, xsh[grp], p, xa);
                d = xa[0] * coefC[0];
#pragma unroll
                for (int q = 1; q < G; ++q) d = fma(xa[q], coefC[q], d);
            } else {
                d = grp_dot<G, R>(xin, coefC);
            }
            R v = tab[grp][tt][p] * d;
            if (first && tt == tt0) v = start;
            if ((tt & (nrm - 1)) == nrm - 1 || tt == L - 1) v = fldexp(v, -fexp(grp_max_pos<G>(v)));
            acur = v;
            atab[grp][tt][p] = v;
        }

        // 4. backward
        R U[G], gs = (R)0, g1 = (R)0, fa[KK];
#pragma unroll
        for (int q = 0; q < G; ++q) U[q] = (R)0;
#pragma unroll
        for (int q = 0; q < KK; ++q) fa[q] = (R)0;
        R bcur = valid ? gi_in : (R)0;
        const bool own = use && live;
        {   // gamma at the chunk's last step
            R h = acur * bcur;
            R Z = grp_sum<G, R>(h);
            R gm = own ? h * frcp(Z) : (R)0;
            gs += gm;
            if constexpr (K > 0)
                fam_accumulate<FAM, R, KK>(gm, ysh[grp][L - 1][0], ysh[grp][L - 1][1], k, fa);
            // rows of excluded sequences are written too (zeros)
            if constexpr (WG) {
                if (valid && live) gamma_out[(off + t0 + len - 1) * N + p] = gm;
            }
        }
        // beta_{t-1}(i) = sum_j a_ij e_t(j) beta_t(j).  Lane i gathers
        // w_j = e_t(j) beta_t(j) from its group once and uses it twice: for
        // beta_{t-1}(i) and for xi_t(i, j) = alpha_{t-1}(i) a_ij w_j / Z_t, where
        // Z_t = sum_i alpha_{t-1}(i) beta_{t-1}(i) also normalises gamma_{t-1}.
#pragma unroll 2
        for (int tt = L - 1; tt >= 0; --tt) {
            const bool trans = (tt > tt0) || (tt == tt0 && !first);
            R w = tab[grp][tt][p] * bcur;
            R wg[G];   // w of the group: state order (LDS) or source order (DPP)
            if constexpr (XL) lds_vec<R, G>(w, xsh[grp], p, wg);
            else grp_gather<G, R>(w, wg);
            R bp = wg[0] * coefR[0];
#pragma unroll
            for (int q = 1; q < G; ++q) bp = fma(wg[q], coefR[q], bp);
            const R xprev = (tt == tt0 || tt == 0) ? ap : atab[grp][tt > 0 ? tt - 1 : 0][p];
            R h = xprev * bp;
            R Z = grp_sum<G, R>(h);
            R rz = frcp(Z);
            const R xr = (use && trans) ? xprev * rz : (R)0;
#pragma unroll
            for (int q = 0; q < G; ++q) U[q] = fma(xr, wg[q], U[q]);
            if (tt > 0) {
                const bool ok = own && tt > tt0;
                R gm = ok ? h * rz : (R)0;
                gs += gm;
                if constexpr (K > 0)
                    fam_accumulate<FAM, R, KK>(gm, ysh[grp][tt - 1][0], ysh[grp][tt - 1][1], k,
                                               fa);
                if constexpr (WG) {
                    if (valid && live && tt > tt0) gamma_out[(off + t0 + (tt - 1 - tt0)) * N + p] = gm;
                }
            }
            // rescaled every nrm steps like the forward: after a rescale, max
            // (e o beta) >= min a_ij / 2 (the state with e = 1 holds at least
            // min a_ij times the previous maximum), and each further step
            // keeps at least a fraction min a_ij of it and never grows
            if ((tt & (nrm - 1)) == 0) bp = fldexp(bp, -fexp(grp_max_pos<G>(bp)));
            if (trans) bcur = bp;
        }
        // gamma at the sequence's first step, once per chunk: after the loop a
        // first chunk's bcur is beta at tt0 (up to a power of two, which the
        // normalisation removes), and alpha at tt0 is in the history
        {
            const R h0 = atab[grp][tt0 < L ? tt0 : L - 1][p] * bcur;
            const R Z0 = grp_sum<G, R>(h0);
            g1 = (first && own) ? h0 * frcp(Z0) : (R)0;
        }
        if (use && live) {
#pragma unroll
            for (int q = 0; q < G; ++q) xacc[q] += (double)(U[q] * coefR[q]);
            gsacc += (double)gs;
            g1acc += (double)g1;
#pragma unroll
            for (int q = 0; q < KK; ++q) facc[q] += (double)fa[q];
        }
        __syncthreads();
    }

    // fixed-order reduction over the block's lane groups (reusing the LDS)
    double (*red)[G][NV] = reinterpret_cast<double (*)[G][NV]>(lds_raw);
#pragma unroll
    for (int q = 0; q < G; ++q) red[grp][p][q] = xacc[q];
    red[grp][p][G] = g1acc;
    red[grp][p][G + 1] = gsacc;
#pragma unroll
    for (int q = 0; q < K; ++q) red[grp][p][G + 2 + q] = facc[q];
    __syncthreads();
    for (int64_t s = 1 + threadIdx.x; s < S; s += BLOCK) {
        int pp, slot;
        if (s <= N) {
            pp = (int)(s - 1);
            slot = G;
        } else if (s < 1 + N + (int64_t)N * N) {
            int q = (int)(s - 1 - N);
            int i = q / N, j = q % N;
            pp = i;
            slot = XL ? j : grp_inv(i, j);
        } else if (s < 1 + 2 * N + (int64_t)N * N) {
            pp = (int)(s - 1 - N - (int64_t)N * N);
            slot = G + 1;
        } else {
            int q = (int)(s - 1 - 2 * N - (int64_t)N * N);
            pp = q / (K > 0 ? K : 1);
            slot = G + 2 + q % (K > 0 ? K : 1);
        }
        double acc = 0.0;
        for (int gi = 0; gi < GPB; ++gi) acc += red[gi][pp][slot];
        partial[(int64_t)blockIdx.x * S + s] = acc;
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * S] = 0.0;
}

// ---------------------------------------------------------------- host side
template <typename R, int G, int FAM, int L>
static void launch_phase3(int nblk, const ChunkGeom &geom, const StagedModel<R> &m, const R *F,
                          const R *Gb, const int32_t *status, double *partial, R *gamma_out,
                          int64_t S, hipStream_t s) {
    ProfScope ps("chunk_stats", s);
    if (gamma_out)
        hipLaunchKernelGGL((k_chunk_stats<R, G, L, FAM, true>), dim3(nblk), dim3(BLOCK), 0, s,
                           geom, m, F, Gb, status, partial, gamma_out, S);
    else
        hipLaunchKernelGGL((k_chunk_stats<R, G, L, FAM, false>), dim3(nblk), dim3(BLOCK), 0, s,
                           geom, m, F, Gb, status, partial, gamma_out, S);
}

template <typename R, int G, int FAM, int L>
static void launch_product(int SC, const SuperDesc *sdesc, const ChunkGeom &geom,
                           const StagedModel<R> &m, ColRec<R, G> *rec, ColRec<R, G> *srec,
                           hipStream_t s) {
    constexpr int SPB = BLOCK / G / SPC;
    hipLaunchKernelGGL((k_chunk_product<R, G, L, FAM>), dim3((SC + SPB - 1) / SPB), dim3(BLOCK),
                       0, s, geom, sdesc, SC, m, m.A8, rec, srec);
}

template <typename R, int G, int FAM>
static hmm_status run_chunked_g(const StagedModel<R> &m, const ObsDesc &o, const ChunkBuffers &cb,
                                double *loglik, int32_t *status, R *gamma_out, double *stats,
                                int64_t S, hipStream_t s) {
    ChunkGeom geom{o.nseq, o.offsets, cb.cbase, (const SuperDesc *)cb.sdesc, cb.SC, cb.L, cb.C,
                   ObsRef{o.obs, o.obs_f64}};
    constexpr int SPB = (BLOCK / 64) * (64 / G);
    if (cb.S != SPC) return HMM_ERR_UNSUPPORTED;
    auto *rec = (ColRec<R, G> *)cb.rec;
    auto *srec = (ColRec<R, G> *)cb.srec;
    const SuperDesc *sdesc = (const SuperDesc *)cb.sdesc;
    R *F = (R *)cb.F;
    R *Gb = (R *)cb.Gb;
    {
        ProfScope ps("chunk_product", s);
        switch (cb.L) {
        case 16: launch_product<R, G, FAM, 16>(cb.SC, sdesc, geom, m, rec, srec, s); break;
        case 32: launch_product<R, G, FAM, 32>(cb.SC, sdesc, geom, m, rec, srec, s); break;
        case 64: launch_product<R, G, FAM, 64>(cb.SC, sdesc, geom, m, rec, srec, s); break;
        default: return HMM_ERR_UNSUPPORTED;
        }
    }
    ScanGeom sg{o.nseq,  o.offsets, cb.cbase, cb.sbase, cb.S,
                cb.SC,   cb.C,      cb.sdesc, ObsRef{o.obs, o.obs_f64}};
    R *Fs = (R *)cb.Fs;
    R *Gs = (R *)cb.Gs;
    {
        ProfScope ps("chunk_scan", s);
        hipLaunchKernelGGL((k_chunk_scan<R, G, FAM, 8, false>),
                           dim3((unsigned)((o.nseq + SPB / 2 - 1) / (SPB / 2))), dim3(BLOCK), 0, s, sg, m,
                           (const ColRec<R, G> *)srec, (const R *)nullptr, (const R *)nullptr, Fs,
                           Gs, loglik, status);
    }
    {
        ProfScope ps("chunk_expand", s);
        hipLaunchKernelGGL((k_chunk_scan<R, G, FAM, 8, true>),
                           dim3((unsigned)((cb.SC + SPB / 2 - 1) / (SPB / 2))), dim3(BLOCK), 0, s, sg, m,
                           (const ColRec<R, G> *)rec, (const R *)Fs, (const R *)Gs, F, Gb, loglik,
                           status);
    }
    switch (cb.L) {
    case 16:
        launch_phase3<R, G, FAM, 16>(cb.nblk_stats, geom, m, F, Gb, status, cb.partial, gamma_out,
                                     S, s);
        break;
    case 32:
        launch_phase3<R, G, FAM, 32>(cb.nblk_stats, geom, m, F, Gb, status, cb.partial, gamma_out,
                                     S, s);
        break;
    case 64:
        if constexpr (sizeof(R) == 4) {
            launch_phase3<R, G, FAM, 64>(cb.nblk_stats, geom, m, F, Gb, status, cb.partial,
                                         gamma_out, S, s);
            break;
        } else {
            return HMM_ERR_UNSUPPORTED;
        }
    default:
        return HMM_ERR_UNSUPPORTED;
    }
    if (stats)
        launch_reduce_stats(cb.partial, cb.nblk_stats, S, loglik, status, o.nseq, stats, cb.red, s);
    return HMM_OK;
}

template <typename R, int G>
static hmm_status run_chunked_fam(const StagedModel<R> &m, const ObsDesc &o,
                                  const ChunkBuffers &cb, double *loglik, int32_t *status,
                                  R *gamma_out, double *stats, int64_t S, hipStream_t s) {
    switch (m.family) {
    case HMM_GAUSSIAN:
        return run_chunked_g<R, G, HMM_GAUSSIAN>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_GAMMA:
        return run_chunked_g<R, G, HMM_GAMMA>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_STUDENT_T:
        return run_chunked_g<R, G, HMM_STUDENT_T>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_POISSON:
        return run_chunked_g<R, G, HMM_POISSON>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    case HMM_TABLE:
        return run_chunked_g<R, G, HMM_TABLE>(m, o, cb, loglik, status, gamma_out, stats, S, s);
    default:
        return HMM_ERR_UNSUPPORTED;
    }
}

template <typename R>
hmm_status run_chunked(const StagedModel<R> &m, const ObsDesc &o, const ChunkBuffers &cb,
                       double *loglik, int32_t *status, void *gamma_out, double *stats,
                       int64_t S, hipStream_t s) {
    if (cb.G == 4)
        return run_chunked_fam<R, 4>(m, o, cb, loglik, status, (R *)gamma_out, stats, S, s);
    if (cb.G == 8)
        return run_chunked_fam<R, 8>(m, o, cb, loglik, status, (R *)gamma_out, stats, S, s);
    return HMM_ERR_UNSUPPORTED;
}

template hmm_status run_chunked<float>(const StagedModel<float> &, const ObsDesc &,
                                       const ChunkBuffers &, double *, int32_t *, void *,
                                       double *, int64_t, hipStream_t);
template hmm_status run_chunked<double>(const StagedModel<double> &, const ObsDesc &,
                                        const ChunkBuffers &, double *, int32_t *, void *,
                                        double *, int64_t, hipStream_t);

}  // namespace hmmk
