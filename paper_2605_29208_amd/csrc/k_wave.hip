// k_wave.hip -- batched forward-backward E-step for 8 < N <= 64 states.
//
// For these state counts a chunk transfer matrix costs N^3 per step, far more
// than the serial recursion itself, so chunk boundaries come from sequential
// sweeps (forward and backward of a sequence run at the same time):
//   forward  alpha_t = (alpha_{t-1} A) o e_t, keeping alpha at every chunk end
//            and the sequence log-likelihood (section 3.1 recursion);
//   backward beta_{t-1} = A (e_t o beta_t), keeping beta at every chunk end.
// Every chunk of WL steps then re-runs its forward steps from its boundary and
// its backward steps with gamma, xi and the family statistics, all chunks in
// parallel.  Vectors are kept normalised (largest entry in [1/2, 1), rescaled
// by powers of two every step) with the log offset summed in FP64.
//
// A lane group of NP = 16, 32 or 64 lanes (lane p = state p) owns one
// sequence direction (sweeps) or one chunk (statistics); a wave holds 64 / NP
// groups.  Vectors are exchanged through LDS (broadcast reads); group sums and
// maxima use DPP row operations and the permlane16 / permlane32 swaps.  The
// emission factors of a window of WL steps are tabulated in LDS with one lane
// per step, so the per-step maximum over states is a local reduction.
#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

constexpr int WL = WAVE_L;   // chunk length = tabulation window


// ---- group all-reductions (every lane of the group receives the result;
// each level combines the same two values in every lane, so all lanes hold
// identical bits) ----
template <int G, bool MAX>
__device__ __forceinline__ float grp_all(float v) {
    auto op = [](float a, float b) { return MAX ? fmaxf(a, b) : a + b; };
    v = op(v, dpp_v<DPP_QP_X1>(v));
    v = op(v, dpp_v<DPP_QP_X2>(v));
    v = op(v, dpp_v<DPP_HALF_MIRROR>(v));
    v = op(v, dpp_v<DPP_ROW_MIRROR>(v));
    if constexpr (G >= 32) {
        const uint32_t u = __builtin_bit_cast(uint32_t, v);
        auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        v = op(__builtin_bit_cast(float, (uint32_t)r[0]), __builtin_bit_cast(float, (uint32_t)r[1]));
    }
    if constexpr (G == 64) {
        const uint32_t u = __builtin_bit_cast(uint32_t, v);
        auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        v = op(__builtin_bit_cast(float, (uint32_t)r[0]), __builtin_bit_cast(float, (uint32_t)r[1]));
    }
    return v;
}

// the two 32-bit halves of a double through one permlane swap each
template <int W>
__device__ __forceinline__ void swap_pair(double v, double *a, double *b) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
    uint32_t l0, l1, h0, h1;
    if constexpr (W == 16) {
        auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    } else {
        auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = rl[0]; l1 = rl[1]; h0 = rh[0]; h1 = rh[1];
    }
    *a = __builtin_bit_cast(double, ((uint64_t)h0 << 32) | l0);
    *b = __builtin_bit_cast(double, ((uint64_t)h1 << 32) | l1);
}

template <int G, bool MAX>
__device__ __forceinline__ double grp_all(double v) {
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = op(v, dpp_v<DPP_QP_X1>(v));
    v = op(v, dpp_v<DPP_QP_X2>(v));
    v = op(v, dpp_v<DPP_HALF_MIRROR>(v));
    v = op(v, dpp_v<DPP_ROW_MIRROR>(v));
    double a, b;
    if constexpr (G >= 32) {
        swap_pair<16>(v, &a, &b);
        v = op(a, b);
    }
    if constexpr (G == 64) {
        swap_pair<32>(v, &a, &b);
        v = op(a, b);
    }
    return v;
}

// maximum of non-negative values: for floats an unsigned maximum of the bit
// patterns (monotone for x >= 0, and no canonicalisation of the operands)
template <int G>
__device__ __forceinline__ float grp_max_nn(float v) {
    uint32_t u = __builtin_bit_cast(uint32_t, v);
    u = max(u, (uint32_t)dpp_i<DPP_QP_X1>((int)u));
    u = max(u, (uint32_t)dpp_i<DPP_QP_X2>((int)u));
    u = max(u, (uint32_t)dpp_i<DPP_HALF_MIRROR>((int)u));
    u = max(u, (uint32_t)dpp_i<DPP_ROW_MIRROR>((int)u));
    if constexpr (G >= 32) {
        auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        u = max((uint32_t)r[0], (uint32_t)r[1]);
    }
    if constexpr (G == 64) {
        auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        u = max((uint32_t)r[0], (uint32_t)r[1]);
    }
    return __builtin_bit_cast(float, u);
}
template <int G>
__device__ __forceinline__ double grp_max_nn(double v) {
    return grp_all<G, true>(v);
}

// sum of a value over the groups of the wave (same state position), fixed order
template <int G>
__device__ __forceinline__ double across_groups(double v) {
    double a, b;
    if constexpr (G == 16) {
        swap_pair<16>(v, &a, &b);
        v = a + b;
    }
    if constexpr (G <= 32) {
        swap_pair<32>(v, &a, &b);
        v = a + b;
    }
    return v;
}

struct WaveGeom {
    int64_t nseq;
    const int64_t *offsets;
    const int *cbase;           // [B+1] chunks (WL steps) before each sequence
    const ChunkDesc *cdesc;     // [C]
    int C;
    ObsRef obs;                 // observations, or the log-emission table (TABLE)
};

// One step's observation data (the observation, or the step's row of the
// log-density table), loaded apart from its use so that a sweep can fetch the
// next window's data while it runs the current one.  Indices are clamped, so
// the loads are unconditional.
template <typename R, int NP, int FAM>
struct StepObs {
    R v[FAM == HMM_TABLE ? NP : 1];
};
template <typename R, int NP, int FAM>
__device__ __forceinline__ StepObs<R, NP, FAM> load_step_obs(const WaveGeom &g, int N, int64_t row) {
    StepObs<R, NP, FAM> o;
    if constexpr (FAM == HMM_TABLE) {
#pragma unroll
        for (int j = 0; j < NP; ++j) o.v[j] = load_obs<R>(g.obs, row * N + min(j, N - 1));
    } else {
        o.v[0] = load_obs<R>(g.obs, row);
    }
    return o;
}

// Emission factors of the NP states at one step, computed by one lane into its
// LDS row: row[j] = exp(log b_j(y) - m) with m = max_j log b_j(y).  Returns m
// plus the state-independent part in FP64 (-inf when no state can emit y);
// sets *bad for a non-finite observation.  The first pass leaves log b in the
// row (Poisson recomputes it instead: its values need FP64).
template <typename R, int NP, int FAM>
__device__ __forceinline__ double tab_step_obs(const StepObs<R, NP, FAM> &o, int N,
                                               const typename EmitTraits<FAM, R>::T *ep, R *erow,
                                               R *y1, R *ly1, bool *bad) {
    using ET = typename EmitTraits<FAM, R>::T;
    constexpr bool RECOMP = FAM == HMM_POISSON;
    ET mx = neg_inf<ET>();
    double common = 0.0;
    R y = (R)0;
    if constexpr (FAM != HMM_TABLE) y = o.v[0];
    // states in groups of eight: the group's constants are all requested
    // before any is used, so the group waits on one load latency, not eight
    constexpr int GQ = 8;
    static_assert(NP % GQ == 0, "whole groups of states");
    for (int j0 = 0; j0 < NP; j0 += GQ) {
        StateConsts<ET> kq[GQ];
        if constexpr (FAM != HMM_TABLE) {
#pragma unroll
            for (int u = 0; u < GQ; ++u) kq[u] = load_consts_row(ep, j0 + u < N ? j0 + u : 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
            const int j = j0 + u;
            const bool live = j < N;
            Emit<ET> em;
            if constexpr (FAM == HMM_TABLE) {
                R v = live ? o.v[j] : neg_inf<R>();
                em.ell = v;
                em.common = 0.0;
                em.bad = live && (isnan(v) || (v > (R)0 && isinf(v)));
            } else {
                em = emit_scalar<FAM, ET>((ET)y, kq[u], live);
            }
            if constexpr (!RECOMP) erow[j] = em.ell;
            mx = fmax(mx, em.ell);
            common = em.common;
            *bad |= em.bad;
        }
    }
    for (int j0 = 0; j0 < NP; j0 += GQ) {
        StateConsts<ET> kq[GQ];
        if constexpr (RECOMP) {
#pragma unroll
            for (int u = 0; u < GQ; ++u) kq[u] = load_consts_row(ep, j0 + u < N ? j0 + u : 0);
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int u = 0; u < GQ; ++u) {
            const int j = j0 + u;
            ET ell;
            if constexpr (RECOMP) ell = emit_scalar<FAM, ET>((ET)y, kq[u], j < N).ell;
            else ell = erow[j];
            erow[j] = (ell == neg_inf<ET>()) ? (R)0 : fexp_e((R)(ell - mx));
        }
    }
    *y1 = y;
    *ly1 = (FAM == HMM_GAMMA && y > (R)0) ? flog(y) : (R)0;
    return (double)mx + common;
}

// The same with the loads in place.  The table family reads its row eight
// states at a time here (rather than the whole row into registers first), so
// that kernels running many lane groups keep their register count down.
template <typename R, int NP, int FAM>
__device__ __forceinline__ double tab_step(const WaveGeom &g, int N, int64_t row,
                                           const typename EmitTraits<FAM, R>::T *ep, R *erow,
                                           R *y1, R *ly1, bool *bad) {
    if constexpr (FAM == HMM_TABLE) {
        constexpr int GQ = 8;
        R mx = neg_inf<R>();
        for (int j0 = 0; j0 < NP; j0 += GQ) {
            R v[GQ];
#pragma unroll
            for (int u = 0; u < GQ; ++u) v[u] = load_obs<R>(g.obs, row * N + min(j0 + u, N - 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < GQ; ++u) {
                const bool live = j0 + u < N;
                const R x = live ? v[u] : neg_inf<R>();
                *bad |= live && (isnan(x) || (x > (R)0 && isinf(x)));
                erow[j0 + u] = x;
                mx = fmax(mx, x);
            }
        }
#pragma unroll 8
        for (int j = 0; j < NP; ++j) {
            const R ell = erow[j];
            erow[j] = (ell == neg_inf<R>()) ? (R)0 : fexp_e((R)(ell - mx));
        }
        *y1 = (R)0;
        *ly1 = (R)0;
        return (double)mx;
    } else {
        return tab_step_obs<R, NP, FAM>(load_step_obs<R, NP, FAM>(g, N, row), N, ep, erow, y1,
                                        ly1, bad);
    }
}

// out = sum_i v_i c_i with v broadcast from LDS (four independent chains, so
// the dependent depth of the sweep step is NP / 4 + 2)
template <typename R, int NP>
__device__ __forceinline__ R lds_dot(const R *v, const R (&c)[NP]) {
    R acc[4] = {(R)0, (R)0, (R)0, (R)0};
#pragma unroll
    for (int i = 0; i < NP; i += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] = fma(v[i + u], c[i + u], acc[u]);
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// ---------------------------------------------------------------- sweeps
// sum of x over lanes l and l ^ 32, identical bits on both
__device__ __forceinline__ float add_halves(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
}
__device__ __forceinline__ double add_halves(double x) {
    double a, b;
    swap_pair<32>(x, &a, &b);
    return a + b;
}
// sum of x over lanes l, l ^ 16, l ^ 32, l ^ 48, identical bits on all four
__device__ __forceinline__ float add_quarters(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    return add_halves(__builtin_bit_cast(float, (uint32_t)r[0]) +
                      __builtin_bit_cast(float, (uint32_t)r[1]));
}
__device__ __forceinline__ double add_quarters(double x) {
    double a, b;
    swap_pair<16>(x, &a, &b);
    return add_halves(a + b);
}

// ---------------------------------------------------------------- segmented sweeps
// A sequence is cut into segments of whole windows (a fixed number of chunks;
// one segment when it is not split), and each (segment, direction) is swept
// by its own wave, so a sweep's serial chain is one segment long.  The vector
// entering a segment is not known when its sweep starts, so there are three
// launches:
//   1. every segment is swept from a vector of ones (the first segment's
//      forward from pi and the last one's backward from beta_{T-1} = 1, both
//      exact), storing its boundary vectors, and the forward its log scale at
//      each chunk end and the log of its end vector's sum;
//   2. every segment is swept again, from the vector that launch 1 stored for
//      its neighbour (the previous segment's last alpha, the next segment's
//      first beta), re-storing its boundaries until its vector agrees with
//      the stored one at a chunk boundary: entrywise within a relative 2^-16
//      (FP32) or 2^-40 (FP64) once scaled by the ratio of the sums, zero
//      entries in the same places.  From
//      there on the stored vectors are those of a sweep from that start, to
//      the same relative distance, since a nonnegative matrix never
//      increases the projective (Hilbert) distance of two vectors;
//   3. one wave per sequence and direction walks its segments in order,
//      re-running from the true entering vector every segment whose second
//      sweep found no agreement or started from a vector that was itself
//      re-run without agreement, and adds up the forward's log-likelihood
//      increments.
// A mixing chain forgets its start within a few hundred steps, so launch 2
// stops early and launch 3 only adds; a chain that does not is re-run segment
// by segment, which is the unsplit sweep's own serial cost.  The second sweep
// never runs a segment's last chunk (forward) or first chunk (backward) where
// a neighbour reads that boundary as its entering vector; where none does
// (the last segment's forward, the first one's backward) it may run the whole
// segment, whose values are then right with or without an agreement.
//
// Log-likelihood increment of a segment entered with w: log sum(M w) -
// log sum(w), M the product of its steps.  Launch 1 keeps J = log sum(M 1)
// and the log scale l1(c) of each chunk end (the stored vector times e^l1 is
// the unnormalised one).  A sweep from w that agrees at chunk c, with log
// scale l(c) and sum ratio rho, has M w = rho e^{l(c) - l1(c)} M 1, so its
// increment is log rho + l(c) - l1(c) + J - log sum(w).

template <typename R>
struct SegTol;
template <>
struct SegTol<float> {
    static constexpr float rel = 1.52587890625e-05f;   // 2^-16
};
template <>
struct SegTol<double> {
    static constexpr double rel = 9.094947017729282379e-13;   // 2^-40
};

constexpr double LN2_D = 0.69314718055994530942;

// One wave sweeping one direction of one segment: lane p = sl holds state
// j = sl % NP of the vector (SPL copies, h = sl / NP picks the rows of the
// product it takes).
template <typename R, int NP, int FAM, int SPL>
struct SegSweep {
    static constexpr int LPT = 64;
    static constexpr int RPL = NP / SPL;
    static constexpr int WW = 2 * WL;
    static_assert(NP * SPL == LPT && WW == LPT, "one task per wave, one window step per lane");
    using ET = typename EmitTraits<FAM, R>::T;

    const WaveGeom &g;
    const StagedModel<R> &m;
    const ET *ep;
    R (*esh)[NP + 1];
    R *vsh;
    R coef[RPL];
    int j, h, sl, N, nrm;
    bool live;

    __device__ __forceinline__ SegSweep(const WaveGeom &g_, const StagedModel<R> &m_,
                                        R (*esh_)[NP + 1], R *vsh_, bool fwd)
        : g(g_), m(m_), ep(consts_ptr<FAM, R>(m_)), esh(esh_), vsh(vsh_) {
        sl = threadIdx.x;
        j = sl % NP;
        h = sl / NP;
        N = m.N;
        nrm = *m.nrm;
        live = j < N;
        // the lane's column (forward) or row (backward) of A: clamped loads,
        // all in flight before the masking
#pragma unroll
        for (int r = 0; r < RPL; ++r) {
            const int i = min(h * RPL + r, N - 1), jj = min(j, N - 1);
            coef[r] = fwd ? m.A[i * N + jj] : m.A[jj * N + i];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < RPL; ++r) coef[r] = (live && h * RPL + r < N) ? coef[r] : (R)0;
    }

    // sum of the vector (one copy of each state)
    __device__ __forceinline__ R vsum(R x) const { return grp_all<LPT, false>(h == 0 ? x : (R)0); }

    // sum_i x_i coef_i with x broadcast through LDS
    __device__ __forceinline__ R product(R x) const {
        vsh[j] = x;
        wave_lds_order();
        R acc = lds_dot<R, RPL>(&vsh[h * RPL], coef);
        if constexpr (SPL == 2) acc = add_halves(acc);
        if constexpr (SPL == 4) acc = add_quarters(acc);
        return acc;
    }

    // v and s equal up to a positive factor (the tolerance above); *lrho =
    // log(sum v / sum s).  Identical result in every lane.
    __device__ __forceinline__ bool agree(R v, R s, double *lrho) const {
        const R sv = vsum(v), ss = vsum(s);
        const R a = (sv / ss) * s;
        // no absolute slack: an entry zero on one side only never agrees, so the
        // two vectors have the same support
        const bool ok = v == a || fabs(v - a) <= SegTol<R>::rel * fmax(v, a);
        const R nbad = grp_all<LPT, true>(ok ? (R)0 : (R)1);
        *lrho = log((double)sv) - log((double)ss);
        const bool r = sv > (R)0 && ss > (R)0 && nbad == (R)0 && isfinite(*lrho);
        return __builtin_amdgcn_readfirstlane((int)r) != 0;
    }

    // Forward steps [ta, tb) of the sequence at row off (T steps, first chunk
    // cb0), from the lane's entry v of the vector entering step ta (ta = 0:
    // pi, step 0 peeled).  At each chunk end c: with CMP and c >= cmin,
    // compare with F[c] and stop at the first agreement (*at = c, *lrho, *l1
    // = lsc[c]); otherwise with ST store v into F[c] (and with LS the log
    // scale into lsc[c]).  *ls = log scale at the stop or the range's end.
    // Returns whether it stopped at an agreement.
    __device__ __forceinline__ bool fwd(R &v, bool &bad, int64_t off, int T, int cb0, int ta, int tb, bool cmp,
                        bool st, bool lsst, int cmin, R *F, double *lsc, double *ls, double *lrho,
                        double *l1, int *at) const {
        const int k0 = ta / WW, k1 = (tb + WW - 1) / WW;
        double logS = 0.0;
        int64_t E = 0;
        bool stop = false;
        StepObs<R, NP, FAM> pre = load_step_obs<R, NP, FAM>(g, N, off + min(k0 * WW + sl, tb - 1));
        for (int k = k0; k < k1; ++k) {
            const int lo = k * WW, hi = min(tb, lo + WW), wn = hi - lo;
            __syncthreads();
            double msum = 0.0;
            if (sl < wn) {
                R y, ly;
                msum = tab_step_obs<R, NP, FAM>(pre, N, ep, &esh[sl][0], &y, &ly, &bad);
            }
            // log offsets of the window's first and second chunk
            double wa, wb;
            swap_pair<32>(grp_all<32, false>(msum), &wa, &wb);
            __syncthreads();
            if (k + 1 < k1) pre = load_step_obs<R, NP, FAM>(g, N, off + min(lo + WW + sl, tb - 1));
            // stored boundaries of the window's chunk ends, requested now
            R s0 = (R)0, s1 = (R)0;
            double q0 = 0.0, q1 = 0.0;
            if (cmp) {
                const int ca = cb0 + lo / WL, cb = cb0 + (hi - 1) / WL;
                s0 = F[(size_t)ca * NP + j];
                s1 = F[(size_t)cb * NP + j];
                q0 = lsc[ca];
                q1 = lsc[cb];
            }
            R e_cur = esh[0][j];
            for (int t = lo; t < hi; ++t) {
                const int q = t - lo;
                R nv;
                if (t == 0) {   // alpha_0 = pi o e_0
                    nv = live ? m.pi[j] * e_cur : (R)0;
                } else {
                    const R acc = product(v);
                    wave_lds_order();
                    nv = e_cur * acc;
                }
                e_cur = esh[q + 1 < wn ? q + 1 : q][j];
                if (t == 0 || (t & (nrm - 1)) == nrm - 1 || t == T - 1) {
                    const int ex = fexp(grp_max_nn<LPT>(nv));
                    v = fldexp(nv, -ex);
                    E += ex;
                } else {
                    v = nv;
                }
                if (t % WL == WL - 1 || t == T - 1) {
                    const int c = cb0 + t / WL;
                    const double lc = logS + wa + (q < WL ? 0.0 : wb) + (double)E * LN2_D;
                    if (cmp && c >= cmin) {
                        double lr;
                        if (agree(v, q < WL ? s0 : s1, &lr)) {
                            *ls = lc;
                            *lrho = lr;
                            *l1 = q < WL ? q0 : q1;
                            *at = c;
                            stop = true;
                            break;
                        }
                    }
                    if (st && h == 0) F[(size_t)c * NP + j] = v;
                    if (lsst && sl == 0) lsc[c] = lc;
                }
            }
            if (stop) break;
            logS += wa + wb;
        }
        if (!stop) *ls = logS + (double)E * LN2_D;
        return stop;
    }

    // Backward steps t = tb - 1 down to max(ta, WL), from the lane's entry v
    // of beta_{tb-1}.  At a chunk start t = c WL the vector is beta at the end
    // of chunk c - 1, slot cb0 + c - 1: with CMP and slot <= smax compare with
    // Gb there and stop at the first agreement (*at = slot); otherwise with ST
    // store it.
    __device__ __forceinline__ bool bwd(R &v, int64_t off, int T, int cb0, int ta, int tb, bool cmp, bool st,
                        int smax, R *Gb, int *at) const {
        const int lo_all = max(ta, WL);
        if (lo_all >= tb) return false;
        const int kA = (tb - 1) / WW, kB = lo_all / WW;
        bool stop = false, bad = false;
        StepObs<R, NP, FAM> pre =
            load_step_obs<R, NP, FAM>(g, N, off + min(max(kA * WW, lo_all) + sl, tb - 1));
        for (int k = kA; k >= kB; --k) {
            const int lo = max(k * WW, lo_all), hi = min(tb, k * WW + WW), wn = hi - lo;
            __syncthreads();
            if (sl < wn) {
                R y, ly;
                (void)tab_step_obs<R, NP, FAM>(pre, N, ep, &esh[sl][0], &y, &ly, &bad);
            }
            __syncthreads();
            if (k > kB) {
                const int nlo = max((k - 1) * WW, lo_all), nhi = min(tb, k * WW);
                pre = load_step_obs<R, NP, FAM>(g, N, off + min(nlo + sl, nhi - 1));
            }
            // stored boundaries at the window's chunk starts (lo, lo + WL)
            R s0 = (R)0, s1 = (R)0;
            if (cmp) {
                const int sa = cb0 + lo / WL - 1;
                s0 = Gb[(size_t)sa * NP + j];
                s1 = Gb[(size_t)(lo + WL < hi ? sa + 1 : sa) * NP + j];
            }
            R e_cur = esh[wn - 1][j];
            for (int t = hi - 1; t >= lo; --t) {
                const int q = t - lo;
                const R acc = product(e_cur * v);
                e_cur = esh[q > 0 ? q - 1 : q][j];
                wave_lds_order();
                const int c = t / WL;
                const int dist = min(T, c * WL + WL) - 1 - t;   // to the chunk's last step
                if ((dist & (nrm - 1)) == nrm - 1 || t == c * WL) {
                    const int ex = fexp(grp_max_nn<LPT>(acc));
                    v = fldexp(acc, -ex);
                } else {
                    v = acc;
                }
                if (t == c * WL) {
                    const int slot = cb0 + c - 1;
                    double lr;
                    if (cmp && slot <= smax && agree(v, t == lo ? s0 : s1, &lr)) {
                        *at = slot;
                        stop = true;
                        break;
                    }
                    if (st && h == 0) Gb[(size_t)slot * NP + j] = v;
                }
            }
            if (stop) break;
        }
        return stop;
    }
};

// value of lane k (uniform k)
__device__ __forceinline__ int lane_int(int x, int k) { return __builtin_amdgcn_readlane(x, k); }
__device__ __forceinline__ double lane_dbl(double x, int k) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, k);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

struct SegArgs {
    const SuperDesc *sdesc;   // [SC] segments (superchunks of seg chunks)
    const int *sbase;         // [B+1] segments before each sequence
    int vmax;                 // chunks a second sweep may run
    double *lsc;              // [C] launch-1 forward log scale at each chunk end
    double *J;                // [SC] launch-1 log sum of the forward end vector
    double *inc;              // [SC] forward increment found by the second sweep
    int32_t *bad;             // [SC] invalid emission values seen by the forward
    int32_t *ver;             // [2 SC] second sweep agreed (forward, backward)
    int32_t *lim;             // [2 SC] first chunk (forward) / last slot (backward)
                              //        still holding launch-1 vectors
};

__device__ __forceinline__ void seg_bounds(const SuperDesc &d, int *ta, int *tb, int *cb0) {
    *ta = d.t0;
    *tb = min(d.T, d.t0 + d.n * WL);
    *cb0 = d.lo - d.t0 / WL;
}

__device__ __forceinline__ void seq_result(double ll, bool anybad, bool perr, double *loglik,
                                           int32_t *status) {
    if (perr) {
        *loglik = __builtin_nan("");
        *status = 4;
    } else if (anybad || isnan(ll)) {
        *loglik = __builtin_nan("");
        *status = 2;
    } else if (!(ll > -__builtin_inf())) {
        *loglik = -__builtin_inf();
        *status = 1;
    } else {
        *loglik = ll;
        *status = 0;
    }
}

// Launch 1: task 2s is the forward of segment s, task 2s + 1 its backward.
// A sequence of one segment gets its log-likelihood and status here.
template <typename R, int NP, int FAM, int SPL>
__global__ __launch_bounds__(64) void k_wave_sweep(WaveGeom g, StagedModel<R> m, SegArgs sa,
                                                   R *__restrict__ F, R *__restrict__ Gb,
                                                   double *__restrict__ loglik,
                                                   int32_t *__restrict__ status) {
    __shared__ R esh[2 * WL][NP + 1];
    __shared__ __align__(16) R vsh[NP + 4];
    const int seg = blockIdx.x >> 1;
    const bool fwd = (blockIdx.x & 1) == 0;
    const SuperDesc d = sa.sdesc[seg];
    int ta, tb, cb0;
    seg_bounds(d, &ta, &tb, &cb0);
    const bool tail = tb == d.T;
    SegSweep<R, NP, FAM, SPL> w(g, m, esh, vsh, fwd);
    R v = w.live ? (R)1 : (R)0;
    if (fwd) {
        bool bad = false;
        double ls, lr, l1;
        int at;
        w.fwd(v, bad, d.off, d.T, cb0, ta, tb, false, true, true, 0, F, sa.lsc, &ls, &lr, &l1, &at);
        const double J = ls + log((double)w.vsum(v));
        const bool anybad = __ballot(bad) != 0;
        if (w.sl == 0) {
            sa.J[seg] = J;
            sa.bad[seg] = anybad ? 1 : 0;
            if (d.head && tail) seq_result(J, anybad, *m.perr != 0, loglik + d.b, status + d.b);
        }
    } else {
        if (tail && w.h == 0) Gb[(size_t)(d.lo + d.n - 1) * NP + w.j] = v;
        int at;
        w.bwd(v, d.off, d.T, cb0, ta, tb, false, true, 0, Gb, &at);
    }
}

// Launch 2: the second sweep of each segment (see above).
template <typename R, int NP, int FAM, int SPL>
__global__ __launch_bounds__(64) void k_wave_verify(WaveGeom g, StagedModel<R> m, SegArgs sa,
                                                    R *__restrict__ F, R *__restrict__ Gb) {
    __shared__ R esh[2 * WL][NP + 1];
    __shared__ __align__(16) R vsh[NP + 4];
    const int seg = blockIdx.x >> 1;
    const int dir = blockIdx.x & 1;
    const SuperDesc d = sa.sdesc[seg];
    int ta, tb, cb0;
    seg_bounds(d, &ta, &tb, &cb0);
    const bool tail = tb == d.T;
    // the sweep may run the whole segment where no neighbour reads the
    // boundary it ends on (the last segment's forward, the first one's
    // backward); it then holds the right values even without an agreement
    const bool whole = dir == 0 ? tail : d.head != 0;
    const int nv = whole ? d.n : min(sa.vmax, d.n - 1);
    if ((dir == 0 && d.head) || (dir == 1 && tail)) {   // entered exactly
        if (threadIdx.x == 0) {
            sa.ver[2 * seg + dir] = 1;
            sa.lim[2 * seg + dir] = dir == 0 ? d.lo : d.lo + d.n - 1;
        }
        return;
    }
    SegSweep<R, NP, FAM, SPL> w(g, m, esh, vsh, dir == 0);
    const int slot_in = dir == 0 ? d.lo - 1 : d.lo + d.n - 1;
    R v = w.live ? (dir == 0 ? F : Gb)[(size_t)slot_in * NP + w.j] : (R)0;
    const R sw = w.vsum(v);
    int ok = 0, lim;
    if (dir == 0) {
        lim = d.lo + max(nv, 0);
        if (nv > 0 && sw > (R)0) {
            bool bad = false;
            double ls, lr, l1;
            int at;
            if (w.fwd(v, bad, d.off, d.T, cb0, ta, whole ? tb : ta + nv * WL, true, true, false, 0,
                      F, sa.lsc, &ls, &lr, &l1, &at)) {
                ok = 1;
                lim = at;
                if (threadIdx.x == 0) sa.inc[seg] = lr + ls - l1 + sa.J[seg] - log((double)sw);
            } else if (whole) {
                const double inc = ls + log((double)w.vsum(v)) - log((double)sw);
                ok = 1;
                if (threadIdx.x == 0) sa.inc[seg] = inc;
            }
        }
    } else {
        lim = whole ? d.lo - 1 : d.lo + d.n - 2 - max(nv, 0);
        if (nv > 0 && sw > (R)0) {
            int at;
            if (w.bwd(v, d.off, d.T, cb0, whole ? ta : max(ta, tb - nv * WL), tb, true, true,
                      INT32_MAX, Gb, &at)) {
                ok = 1;
                lim = at;
            } else if (whole) {
                ok = 1;
            }
        }
    }
    if (threadIdx.x == 0) {
        sa.ver[2 * seg + dir] = ok;
        sa.lim[2 * seg + dir] = lim;
    }
}

// Launch 3: task 2b walks the forward segments of sequence b, task 2b + 1 the
// backward ones (sequences of one segment have nothing to do).
template <typename R, int NP, int FAM, int SPL>
__global__ __launch_bounds__(64) void k_wave_fixup(WaveGeom g, StagedModel<R> m, SegArgs sa,
                                                   R *__restrict__ F, R *__restrict__ Gb,
                                                   double *__restrict__ loglik,
                                                   int32_t *__restrict__ status) {
    __shared__ R esh[2 * WL][NP + 1];
    __shared__ __align__(16) R vsh[NP + 4];
    const int b = blockIdx.x >> 1;
    const bool fwd = (blockIdx.x & 1) == 0;
    const int s0 = sa.sbase[b], s1 = sa.sbase[b + 1];
    if (s1 - s0 <= 1) return;
    SegSweep<R, NP, FAM, SPL> w(g, m, esh, vsh, fwd);
    R v = (R)0;
    bool ok = true, have = false;   // entering vector: stored one right / held in v
    const int lane = threadIdx.x;
    if (fwd) {
        double ll = 0.0;
        bool anybad = false;
        // the flags of 64 segments at a time, one per lane, requested together
        for (int g0 = s0; g0 < s1; g0 += 64) {
            const int sq = min(g0 + lane, s1 - 1);
            const int qbad = sa.bad[sq], qver = sa.ver[2 * sq];
            const double qinc = sq == s0 ? sa.J[s0] : sa.inc[sq];
            const int cnt = min(64, s1 - g0);
            for (int k = 0; k < cnt; ++k) {
                const int s = g0 + k;
                anybad |= lane_int(qbad, k) != 0;
                if (anybad || !(ll > -__builtin_inf())) continue;
                if (s == s0 || (ok && lane_int(qver, k))) {
                    ll += lane_dbl(qinc, k);
                    continue;
                }
                const SuperDesc d = sa.sdesc[s];
                int ta, tb, cb0;
                seg_bounds(d, &ta, &tb, &cb0);
                if (!have) v = w.live ? F[(size_t)(d.lo - 1) * NP + w.j] : (R)0;
                const R sw = w.vsum(v);
                if (!(sw > (R)0)) {
                    ll = -__builtin_inf();
                    continue;
                }
                bool bad = false;
                double ls, lr, l1;
                int at;
                if (w.fwd(v, bad, d.off, d.T, cb0, ta, tb, true, true, false, sa.lim[2 * s], F,
                          sa.lsc, &ls, &lr, &l1, &at)) {
                    ll += lr + ls - l1 + sa.J[s] - log((double)sw);
                    ok = true;
                    have = false;
                } else {
                    ll += ls + log((double)w.vsum(v)) - log((double)sw);
                    ok = false;
                    have = true;
                }
            }
        }
        if (lane == 0) seq_result(ll, anybad, *m.perr != 0, loglik + b, status + b);
    } else {
        // the last segment is entered exactly; the others from the top down
        bool dead = false;
        for (int top = s1 - 2; top >= s0 && !dead; top -= 64) {
            const int qver = sa.ver[2 * max(top - lane, s0) + 1];
            const int cnt = min(64, top - s0 + 1);
            for (int k = 0; k < cnt; ++k) {
                const int s = top - k;
                if (ok && lane_int(qver, k)) continue;
                const SuperDesc d = sa.sdesc[s];
                int ta, tb, cb0;
                seg_bounds(d, &ta, &tb, &cb0);
                if (!have) v = w.live ? Gb[(size_t)(d.lo + d.n - 1) * NP + w.j] : (R)0;
                if (!(w.vsum(v) > (R)0)) {   // no path: the forward reports it
                    dead = true;
                    break;
                }
                int at;
                const bool hit =
                    w.bwd(v, d.off, d.T, cb0, ta, tb, true, true, sa.lim[2 * s + 1], Gb, &at);
                ok = hit;
                have = !hit;
            }
        }
    }
}

// ---------------------------------------------------------------- chunk statistics
// One lane group per chunk (grid-stride over chunks).  From alpha at the end of
// the previous chunk and beta at the end of this one: re-run the chunk's
// forward steps (alpha history in LDS), then its backward steps, forming at
// each step (beta_{t-1} normalised before the products; the normaliser
// cancels in gamma and is put back in xi)
//   h_i = alpha_{t-1}(i) beta_{t-1}(i),    gamma_{t-1} = h / sum h,
//   xi_ij = alpha_{t-1}(i) a_ij w_j / sum_k alpha_{t-1}(k) (A w)_k,  w_j = e_t(j) beta_t(j).
// Lane i keeps U_i(k) = sum_t alpha_{t-1}(i) w_t(k) / Z_t; its xi row is
// U_i(k) a_ik at the end of the chunk, added to FP64 accumulators (registers
// for NP <= 32, LDS for NP = 64).  GAMMA writes gamma rows; STATS accumulates
// the pooled statistics.
template <typename R, int NP, int FAM, bool GAMMA, bool STATS>
__global__ __launch_bounds__(64) void k_wave_stats(WaveGeom g, StagedModel<R> m,
                                                   const R *__restrict__ F,
                                                   const R *__restrict__ Gb,
                                                   const int32_t *__restrict__ status,
                                                   double *__restrict__ partial,
                                                   R *__restrict__ gamma_out, int64_t S) {
    constexpr int NG = 64 / NP;
    constexpr int VS = NP + 4;
    constexpr int K = STATS ? fam_k<FAM>() : 0;
    constexpr int KK = K > 0 ? K : 1;
    constexpr bool XLDS = STATS && NP > 32;
    constexpr int UN = STATS ? NP : 1;
    constexpr int XN = (STATS && !XLDS) ? NP : 1;
    __shared__ R esh[NG][WL][NP + 1];
    __shared__ R ash[NG][WL][NP + 1];
    __shared__ R ysh[NG][WL][2];
    __shared__ __align__(16) R vsh[NG][VS];
    __shared__ double xl[XLDS ? NP * 64 : 1];
    using ET = typename EmitTraits<FAM, R>::T;
    const ET *ep = consts_ptr<FAM, R>(m);
    const int lane = threadIdx.x;
    const int grp = lane / NP, j = lane % NP;
    const int N = m.N;
    const bool live = j < N;
    const StateConsts<ET> kj = load_consts(ep, j, live);
    R coefC[NP], coefR[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        coefC[i] = (live && i < N) ? m.A[i * N + j] : (R)0;
        coefR[i] = (live && i < N) ? m.A[j * N + i] : (R)0;
    }
    const R pi_j = live ? m.pi[j] : (R)0;
    const int nrm = *m.nrm;
    double xacc[XN], gsacc = 0.0, g1acc = 0.0, facc[KK];
#pragma unroll
    for (int k = 0; k < XN; ++k) xacc[k] = 0.0;
    if constexpr (XLDS) {
#pragma unroll
        for (int k = 0; k < NP; ++k) xl[k * 64 + lane] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < KK; ++k) facc[k] = 0.0;

    for (int c0 = blockIdx.x * NG; c0 < g.C; c0 += gridDim.x * NG) {
        const int c = c0 + grp;
        const bool valid = c < g.C;
        ChunkDesc d;
        if (valid) {
            d = g.cdesc[c];
        } else {
            d.off = 0;
            d.b = 0;
            d.t0 = 0;
            d.len = 0;
        }
        const bool use = valid && status[d.b] == 0;
        const bool first = d.t0 == 0;
        const int len = d.len;
        const int lmax = wave_max_i(len);
        bool badc = false;
        __syncthreads();
        for (int q = j; q < len; q += NP) {
            R y, ly;
            tab_step<R, NP, FAM>(g, N, d.off + d.t0 + q, ep, &esh[grp][q][0], &y, &ly, &badc);
            ysh[grp][q][0] = y;
            ysh[grp][q][1] = ly;
        }
        __syncthreads();
        // forward steps of the chunk
        const R ap = (!valid || first || !live) ? (R)0 : F[(size_t)(c - 1) * NP + j];
        R a = ap;
        R e_cur = (len > 0) ? esh[grp][0][j] : (R)0;
        for (int s = 0; s < lmax; ++s) {
            const bool on = s < len;
            const R e = e_cur;
            vsh[grp][j] = a;
            wave_lds_order();
            const R acc = lds_dot<R, NP>(&vsh[grp][0], coefC);
            e_cur = (s + 1 < len) ? esh[grp][s + 1][j] : (R)0;
            wave_lds_order();
            const R nv = (first && s == 0) ? (live ? pi_j * e : (R)0) : e * acc;
            const bool rs = (s & (nrm - 1)) == nrm - 1;
            const int ex = rs ? fexp(grp_max_nn<NP>(nv)) : 0;
            if (on) {
                a = rs ? fldexp(nv, -ex) : nv;
                ash[grp][s][j] = a;
            }
        }
        // backward steps with the posteriors
        R U[UN], gs = (R)0, g1 = (R)0, fa[KK];
#pragma unroll
        for (int k = 0; k < UN; ++k) U[k] = (R)0;
#pragma unroll
        for (int k = 0; k < KK; ++k) fa[k] = (R)0;
        const bool own = use && live;
        R be = (valid && live) ? Gb[(size_t)c * NP + j] : (R)0;
        {
            const R h = a * be;
            const R Z = grp_all<NP, false>(h);
            const R gmv = h * frcp(Z);
            if (own) {
                if constexpr (STATS) {
                    gs += gmv;
                    if constexpr (K > 0)
                        fam_accumulate<FAM, R, KK>(gmv, ysh[grp][len - 1][0], ysh[grp][len - 1][1], kj, fa);
                    if (first && len == 1) g1 += gmv;
                }
            }
            // gamma rows of excluded sequences are written as zeros
            if constexpr (GAMMA)
                if (valid && live) gamma_out[(d.off + d.t0 + len - 1) * N + j] = own ? gmv : (R)0;
        }
        const int s_stop = first ? 1 : 0;
        e_cur = (len - 1 >= s_stop) ? esh[grp][len > 0 ? len - 1 : 0][j] : (R)0;
        for (int s = lmax - 1; s >= 0; --s) {
            const bool on = s < len && s >= s_stop;
            const R e = on ? e_cur : (R)0;
            vsh[grp][j] = e * be;
            wave_lds_order();
            const R bp = lds_dot<R, NP>(&vsh[grp][0], coefR);
            if (on) e_cur = (s - 1 >= s_stop) ? esh[grp][s > 0 ? s - 1 : 0][j] : (R)0;
            const int ex = (s & (nrm - 1)) == 0 ? fexp(grp_max_nn<NP>(bp)) : 0;
            const R bn = fldexp(bp, -ex);
            const R xp = (s > 0) ? ash[grp][s > 0 ? s - 1 : 0][j] : ap;
            const R h = on ? xp * bn : (R)0;
            const R Z = grp_all<NP, false>(h);
            const R rz = frcp(Z);
            if constexpr (STATS) {
                // xi uses the unnormalised (A w): scale 1/Z by 2^-ex
                const R xr = (on && use) ? fldexp(xp * rz, -ex) : (R)0;
#pragma unroll
                for (int k = 0; k < UN; ++k) U[k] = fma(xr, vsh[grp][k], U[k]);
            }
            wave_lds_order();
            if (on) {
                const R gmv = h * rz;
                if (s > 0 && own) {
                    if constexpr (STATS) {
                        gs += gmv;
                        if constexpr (K > 0)
                            fam_accumulate<FAM, R, KK>(gmv, ysh[grp][s - 1][0], ysh[grp][s - 1][1], kj, fa);
                        if (first && s == 1) g1 += gmv;
                    }
                }
                if constexpr (GAMMA)
                    if (s > 0 && live) gamma_out[(d.off + d.t0 + s - 1) * N + j] = own ? gmv : (R)0;
                be = bn;
            }
        }
        if constexpr (STATS) {
            if (own) {
                if constexpr (XLDS) {
#pragma unroll
                    for (int k = 0; k < NP; ++k) xl[k * 64 + lane] += (double)(U[k] * coefR[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < XN; ++k) xacc[k] += (double)(U[k] * coefR[k]);
                }
                gsacc += (double)gs;
                g1acc += (double)g1;
#pragma unroll
                for (int k = 0; k < KK; ++k) facc[k] += (double)fa[k];
            }
        }
    }
    if constexpr (STATS) {
        // this block's partial statistics row (layout of hmm_stats_len), the
        // groups of the wave summed in a fixed order; entry 0 (the
        // log-likelihood) is summed from loglik by the reduction
        double *row = partial + (int64_t)blockIdx.x * S;
        const bool w = live && grp == 0;
        const double g1s = across_groups<NP>(g1acc);
        const double gss = across_groups<NP>(gsacc);
        if (w) {
            row[1 + j] = g1s;
            row[1 + N + (int64_t)N * N + j] = gss;
        }
        double *xrow = row + 1 + N + (int64_t)j * N;
        if constexpr (XLDS) {
            if (w)
                for (int k = 0; k < N; ++k) xrow[k] = xl[k * 64 + lane];
        } else {
#pragma unroll
            for (int k = 0; k < XN; ++k) {
                const double x = across_groups<NP>(xacc[k]);
                if (w && k < N) xrow[k] = x;
            }
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const double x = across_groups<NP>(facc[q]);
            if (w) row[1 + 2 * N + (int64_t)N * N + (int64_t)j * K + q] = x;
        }
    }
}

// ---------------------------------------------------------------- host side
template <typename R, int NP, int FAM>
static hmm_status run_wave_np(const StagedModel<R> &m, const ObsDesc &o, const WaveBuffers &wb,
                              double *loglik, int32_t *status, R *gamma_out, double *stats,
                              int64_t S, hipStream_t s) {
    // sweeps: one task per wave (two lanes per state for 32 states, four for 16)
    constexpr int SPL = 64 / NP;
    WaveGeom g{o.nseq, o.offsets, wb.cbase, wb.cdesc, wb.C, ObsRef{o.obs, o.obs_f64}};
    R *F = (R *)wb.F, *Gb = (R *)wb.Gb;
    const SegArgs sa{wb.sdesc, wb.sbase, wb.vmax, wb.lsc, wb.segJ, wb.seginc,
                     wb.segbad, wb.segver, wb.seglim};
    {
        ProfScope ps("wave_sweep", s);
        hipLaunchKernelGGL((k_wave_sweep<R, NP, FAM, SPL>), dim3((unsigned)(2 * wb.SC)), dim3(64),
                           0, s, g, m, sa, F, Gb, loglik, status);
    }
    if (wb.SC > o.nseq) {   // some sequence is split
        {
            ProfScope ps("wave_verify", s);
            hipLaunchKernelGGL((k_wave_verify<R, NP, FAM, SPL>), dim3((unsigned)(2 * wb.SC)),
                               dim3(64), 0, s, g, m, sa, F, Gb);
        }
        {
            ProfScope ps("wave_fixup", s);
            hipLaunchKernelGGL((k_wave_fixup<R, NP, FAM, SPL>), dim3((unsigned)(2 * o.nseq)),
                               dim3(64), 0, s, g, m, sa, F, Gb, loglik, status);
        }
    }
    if (!gamma_out && !stats) return HMM_OK;
    {
        ProfScope ps("wave_stats", s);
        if (gamma_out && stats)
            hipLaunchKernelGGL((k_wave_stats<R, NP, FAM, true, true>), dim3(wb.nblk), dim3(64), 0,
                               s, g, m, (const R *)F, (const R *)Gb, (const int32_t *)status,
                               wb.partial, gamma_out, S);
        else if (gamma_out)
            hipLaunchKernelGGL((k_wave_stats<R, NP, FAM, true, false>), dim3(wb.nblk), dim3(64), 0,
                               s, g, m, (const R *)F, (const R *)Gb, (const int32_t *)status,
                               wb.partial, gamma_out, S);
        else
            hipLaunchKernelGGL((k_wave_stats<R, NP, FAM, false, true>), dim3(wb.nblk), dim3(64), 0,
                               s, g, m, (const R *)F, (const R *)Gb, (const int32_t *)status,
                               wb.partial, gamma_out, S);
    }
    if (stats)
        launch_reduce_stats(wb.partial, wb.nblk, S, loglik, status, o.nseq, stats, wb.red, s);
    return HMM_OK;
}

template <typename R, int NP>
static hmm_status run_wave_fam(const StagedModel<R> &m, const ObsDesc &o, const WaveBuffers &wb,
                               double *loglik, int32_t *status, R *gamma_out, double *stats,
                               int64_t S, hipStream_t s) {
    switch (m.family) {
    case HMM_GAUSSIAN:
        return run_wave_np<R, NP, HMM_GAUSSIAN>(m, o, wb, loglik, status, gamma_out, stats, S, s);
    case HMM_GAMMA:
        return run_wave_np<R, NP, HMM_GAMMA>(m, o, wb, loglik, status, gamma_out, stats, S, s);
    case HMM_STUDENT_T:
        return run_wave_np<R, NP, HMM_STUDENT_T>(m, o, wb, loglik, status, gamma_out, stats, S, s);
    case HMM_POISSON:
        return run_wave_np<R, NP, HMM_POISSON>(m, o, wb, loglik, status, gamma_out, stats, S, s);
    case HMM_TABLE:
        return run_wave_np<R, NP, HMM_TABLE>(m, o, wb, loglik, status, gamma_out, stats, S, s);
    default:
        return HMM_ERR_UNSUPPORTED;
    }
}

int wave_np(int N) { return N <= 16 ? 16 : (N <= 32 ? 32 : 64); }

int wave_seg_chunks(int variant) {
    // whole windows (an even number of chunks); 2^28 chunks never splits
    static const int K[4] = {32, 1 << 28, 16, 64};
    return K[variant < 0 ? 0 : (variant > 3 ? 3 : variant)];
}

int wave_stats_blocks(int C, int N) {
    const int ng = 64 / wave_np(N);
    const int nb = (C + ng - 1) / ng;
    return nb < 1 ? 1 : (nb > 2048 ? 2048 : nb);
}

template <typename R>
hmm_status run_wave(const StagedModel<R> &m, const ObsDesc &o, const WaveBuffers &wb,
                    double *loglik, int32_t *status, void *gamma_out, double *stats, int64_t S,
                    hipStream_t s) {
    if (o.nseq == 0) return HMM_OK;
    if (m.N > 64) return HMM_ERR_UNSUPPORTED;
    switch (wave_np(m.N)) {
    case 16:
        return run_wave_fam<R, 16>(m, o, wb, loglik, status, (R *)gamma_out, stats, S, s);
    case 32:
        return run_wave_fam<R, 32>(m, o, wb, loglik, status, (R *)gamma_out, stats, S, s);
    default:
        // FP64 with N > 32 is planned onto the large-state path instead
        if constexpr (sizeof(R) == 8) return HMM_ERR_UNSUPPORTED;
        else return run_wave_fam<R, 64>(m, o, wb, loglik, status, (R *)gamma_out, stats, S, s);
    }
}

template hmm_status run_wave<float>(const StagedModel<float> &, const ObsDesc &,
                                    const WaveBuffers &, double *, int32_t *, void *, double *,
                                    int64_t, hipStream_t);
template hmm_status run_wave<double>(const StagedModel<double> &, const ObsDesc &,
                                     const WaveBuffers &, double *, int32_t *, void *, double *,
                                     int64_t, hipStream_t);

}  // namespace hmmk
