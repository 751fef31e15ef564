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

// Task 2b is the forward sweep of sequence b (alpha at chunk ends, logL and
// status), task 2b + 1 its backward sweep (beta at chunk ends), one task per
// wave.  SPL = 64 / NP lanes per state: for NP = 32 half h of the lanes takes
// rows h NP/2 .. of the vector-matrix product and the halves are added across
// the wave, which halves the dependent chain of the step; SPL = 4 does the
// same with four lanes per state for NP = 16.
template <typename R, int NP, int FAM, int SPL>
__global__ __launch_bounds__(64) void k_wave_sweep(WaveGeom g, StagedModel<R> m, R *__restrict__ F,
                                                   R *__restrict__ Gb, double *__restrict__ loglik,
                                                   int32_t *__restrict__ status) {
    static_assert(NP * SPL == 64, "one task per wave");
    constexpr int LPT = NP * SPL;   // lanes per task
    constexpr int NG = 64 / LPT;    // tasks per wave (one)
    constexpr int RPL = NP / SPL;   // rows of the product per lane
    constexpr int VS = NP + 4;
    // a window of the emission table holds two chunks
    __shared__ R esh[NG][2 * WL][NP + 1];
    __shared__ __align__(16) R vsh[NG][VS];
    using ET = typename EmitTraits<FAM, R>::T;
    const ET *ep = consts_ptr<FAM, R>(m);
    const int lane = threadIdx.x;
    const int grp = lane / LPT, sl = lane % LPT, j = sl % NP, h = sl / NP;
    const int64_t task = (int64_t)blockIdx.x * NG + grp;
    const bool tv = task < 2 * g.nseq;
    const int64_t b = tv ? (task >> 1) : 0;
    // one task per wave: the direction is uniform, so its branches are scalar
    const bool fwd = __builtin_amdgcn_readfirstlane((int)((task & 1) == 0)) != 0;
    const int N = m.N;
    const bool live = j < N;
    const int64_t off = g.offsets[b];
    int T = tv ? (int)(g.offsets[b + 1] - off) : 0;
    int cb = g.cbase[b];
    // uniform per wave: keep the loop control scalar
    T = __builtin_amdgcn_readfirstlane(T);
    cb = __builtin_amdgcn_readfirstlane(cb);
    const int nc = (T + WL - 1) / WL;
    // the lane's column (forward) or row (backward) of A: clamped loads, all
    // in flight before the masking
    R coef[RPL];
#pragma unroll
    for (int r = 0; r < RPL; ++r) {
        const int i = min(h * RPL + r, N - 1), jj = min(j, N - 1);
        coef[r] = fwd ? m.A[i * N + jj] : m.A[jj * N + i];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < RPL; ++r) coef[r] = (live && h * RPL + r < N) ? coef[r] : (R)0;
    bool bad = false;
    const int nrm = *m.nrm;   // steps between rescalings (both directions)
    R v = (tv && live) ? (R)1 : (R)0;   // running alpha (forward) or beta (backward)
    double logS = 0.0;
    int64_t E = 0;
    if (tv && !fwd && h == 0) Gb[(size_t)(cb + nc - 1) * NP + j] = v;

    // One task per wave: the direction, the length and the step are
    // uniform, so the loops below have scalar control.  A window is two
    // chunks (64 steps, one step per lane for the emission table), and the
    // observations of the next window are loaded into registers while the
    // current one runs, so the table of a window waits on no memory.
    // Rescaling points and stored boundaries are those of one-chunk
    // windows: forward after steps t = nrm - 1 (mod nrm), the last step and
    // t = 0, boundary at every chunk end; backward after the steps whose
    // distance to their chunk's end is nrm - 1 (mod nrm) and at the chunk's
    // first step, boundary beta at the end of the previous chunk.
    constexpr int WW = 2 * WL;
    static_assert(WW == LPT, "one window step per lane");
    const int nw = (T + WW - 1) / WW;
    // window k covers steps [lo, hi); the backward skips chunk 0
    auto wlo = [&](int k) { return fwd ? k * WW : max(k * WW, WL); };
    auto whi = [&](int k) { return min(T, k * WW + WW); };
    const int k0 = fwd ? 0 : nw - 1, kstep = fwd ? 1 : -1;
    const int kend = fwd ? nw : -1;
    StepObs<R, NP, FAM> pre;
    if (k0 != kend && wlo(k0) < whi(k0))
        pre = load_step_obs<R, NP, FAM>(g, N, off + min(wlo(k0) + sl, whi(k0) - 1));
    for (int k = k0; k != kend; k += kstep) {
        const int lo = wlo(k), hi = whi(k), wn = hi - lo;
        if (wn <= 0) continue;
        __syncthreads();
        double msum = 0.0;
        if (sl < wn) {
            R y, ly;
            msum = tab_step_obs<R, NP, FAM>(pre, N, ep, &esh[0][sl][0], &y, &ly, &bad);
        }
        const double wsum = grp_all<LPT, false>(msum);
        if (fwd) logS += wsum;
        __syncthreads();
        // the next window's observations, in flight during this window
        const int kn = k + kstep;
        if (kn != kend && wlo(kn) < whi(kn))
            pre = load_step_obs<R, NP, FAM>(g, N, off + min(wlo(kn) + sl, whi(kn) - 1));
        if (fwd) {
            R e_cur = esh[0][0][j];
            for (int t = lo; t < hi; ++t) {
                const int q = t - lo;
                R nv;
                if (t == 0) {   // alpha_0 = pi o e_0
                    nv = live ? m.pi[j] * e_cur : (R)0;
                } else {
                    vsh[0][j] = v;   // both halves store the same value
                    wave_lds_order();
                    R acc = lds_dot<R, RPL>(&vsh[0][h * RPL], coef);
                    if constexpr (SPL == 2) acc = add_halves(acc);
                    if constexpr (SPL == 4) acc = add_quarters(acc);
                    wave_lds_order();
                    nv = e_cur * acc;
                }
                e_cur = esh[0][q + 1 < wn ? q + 1 : q][j];
                if (t == 0 || (t & (nrm - 1)) == nrm - 1 || t == T - 1) {
                    const int ex = fexp(grp_max_nn<LPT>(nv));
                    v = fldexp(nv, -ex);
                    E += ex;
                } else {
                    v = nv;
                }
                if ((t % WL == WL - 1 || t == T - 1) && h == 0) F[(size_t)(cb + t / WL) * NP + j] = v;
            }
        } else {
            R e_cur = esh[0][wn - 1][j];
            for (int t = hi - 1; t >= lo; --t) {
                const int q = t - lo;
                vsh[0][j] = e_cur * v;
                wave_lds_order();
                R acc = lds_dot<R, RPL>(&vsh[0][h * RPL], coef);
                if constexpr (SPL == 2) acc = add_halves(acc);
                if constexpr (SPL == 4) acc = add_quarters(acc);
                e_cur = esh[0][q > 0 ? q - 1 : q][j];
                wave_lds_order();
                const int c = t / WL;
                const int dist = min(T, c * WL + WL) - 1 - t;   // to the chunk's last step
                if ((dist & (nrm - 1)) == nrm - 1 || t == c * WL) {
                    const int ex = fexp(grp_max_nn<LPT>(acc));
                    v = fldexp(acc, -ex);
                } else {
                    v = acc;
                }
                if (t == c * WL && h == 0) Gb[(size_t)(cb + c - 1) * NP + j] = v;
            }
        }
    }
    const R tot = grp_all<LPT, false>((fwd && h == 0) ? v : (R)0);
    const uint64_t bal = __ballot(bad);
    const uint64_t gmask = (LPT == 64) ? ~0ull : (((1ull << (LPT & 63)) - 1) << (grp * LPT));
    const bool anybad = (bal & gmask) != 0;
    if (tv && fwd && sl == 0) {
        double ll;
        int st;
        if (*m.perr) {
            ll = __builtin_nan("");
            st = 4;
        } else if (anybad || isnan(logS)) {
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
    constexpr int NG = 64 / (NP * SPL);
    WaveGeom g{o.nseq, o.offsets, wb.cbase, wb.cdesc, wb.C, ObsRef{o.obs, o.obs_f64}};
    R *F = (R *)wb.F, *Gb = (R *)wb.Gb;
    {
        ProfScope ps("wave_sweep", s);
        const unsigned nb = (unsigned)((2 * o.nseq + NG - 1) / NG);
        hipLaunchKernelGGL((k_wave_sweep<R, NP, FAM, SPL>), dim3(nb), dim3(64), 0, s, g, m, F, Gb,
                           loglik, status);
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
