// k_viterbi.hip -- Viterbi decoding (section 3.3) for N <= 64 states.
//
// Forward max-plus recursion, one wave per sequence, lane j = state j:
//   delta_1(j) = log pi_j + log b_j(y_1)
//   delta_t(j) = max_i [delta_{t-1}(i) + log a_ij] + log b_j(y_t),
//   psi_t(j)   = the lowest i attaining the maximum (strict comparison in
//                increasing i),
// with every step shifted by m_t = max_j delta_t(j) and the shifts summed in
// FP64 (an exact shift for the argmax; it keeps the values small).  The
// additions happen in the same order as in the plain definition, so with
// identical log b inputs the FP64 path reproduces it bit for bit.
// psi is stored as one byte per (step, state): the predecessor in the low
// seven bits and, in bit 7, whether the best and second-best candidates
// differ by less than the tie threshold (a near-tie, section 3.3 breaks
// such ties towards the lowest index; the backtrace counts the near-ties
// met along the returned path).
//
// Backtrace in three kernels: per chunk of K = 64 steps a jump table
// J_c[j] = state just before the chunk when the chunk ends in state j (the
// chunk's psi block is staged in LDS and chased on chip); a chain over the
// chunks of each sequence (one wave per sequence, next rows prefetched, the
// current state wave-uniform so J_c[q] is a lane read); and a parallel fill
// of each chunk's path from its end state.
#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

constexpr int VK = 64;   // steps per backtrace chunk and per emission window
// a decision whose best and second-best candidates differ by less than this
// (per-step shifted scores) is a near-tie
constexpr double VIT_TIE_EPS = 1e-12;

// log b_j(y) of the NMAX states of one step, computed by one lane into its
// LDS row (without the state-independent part, which is returned in FP64).
// FAM < 0 evaluates any family through emission_any.
template <typename R, int NMAX, int FAM>
__device__ __forceinline__ double vit_tab_step(const StagedModel<R> &m, const ObsRef &o, int64_t row,
                                               R *lrow, bool *bad) {
    const int N = m.N;
    double common = 0.0;
    if constexpr (FAM < 0) {
#pragma unroll 2
        for (int j = 0; j < NMAX; ++j) {
            if (j < N) {
                bool bd = false;
                lrow[j] = (R)emission_any<R>(m, o, row, j, &common, &bd);
                *bad |= bd;
            }
        }
    } else if constexpr (FAM == HMM_TABLE) {
        // eight states at a time: clamped loads, all in flight before use
        constexpr int GQ = NMAX < 8 ? NMAX : 8;
        static_assert(NMAX % GQ == 0, "whole groups of states");
        for (int j0 = 0; j0 < NMAX; j0 += GQ) {
            R v[GQ];
#pragma unroll
            for (int u = 0; u < GQ; ++u) v[u] = load_obs<R>(o, row * N + min(j0 + u, N - 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < GQ; ++u) {
                if (j0 + u < N) {
                    *bad |= isnan(v[u]) || (v[u] > (R)0 && isinf(v[u]));
                    lrow[j0 + u] = v[u];
                }
            }
        }
    } else {
        using ET = typename EmitTraits<FAM, R>::T;
        const ET *ep = consts_ptr<FAM, R>(m);
        const ET y = load_obs<ET>(o, row);
        constexpr int GQ = NMAX < 8 ? NMAX : 8;
        static_assert(NMAX % GQ == 0, "whole groups of states");
        for (int j0 = 0; j0 < NMAX; j0 += GQ) {
            StateConsts<ET> kq[GQ];
#pragma unroll
            for (int u = 0; u < GQ; ++u) kq[u] = load_consts_row(ep, min(j0 + u, N - 1));
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < GQ; ++u) {
                if (j0 + u < N) {
                    const Emit<ET> e = emit_scalar<FAM, ET>(y, kq[u], true);
                    lrow[j0 + u] = (R)e.ell;
                    common = e.common;
                    *bad |= e.bad;
                }
            }
        }
    }
    return common;
}

// ---------------------------------------------------------------- forward sweeps
// A sequence longer than one segment (VSEG chunks of VK steps) has its forward
// recursion cut into segments swept in parallel, in the manner of the E-step's
// wave path: launch 1 sweeps every segment from the all-zero score vector (the
// first from log pi, exact), writing psi and storing the shifted score vector
// and the shift sum at each chunk end; launch 2 sweeps each later segment
// again from the vector launch 1 stored at the end of the previous one,
// rewriting psi until its vector agrees with launch 1's at a chunk end (every
// entry within VIT_AGREE_EPS, the same -inf entries); launch 3 walks each
// sequence's segments in order, re-runs those whose second sweep found no
// agreement or started from a vector that was itself re-run without one, sums
// the shift increments and picks the final state.  The max-plus recursion is
// non-expansive in the largest entrywise difference, so from an agreement on
// the scores stay within that distance and a decision can differ only where
// its best and second-best candidates are closer than twice it: below the
// near-tie threshold in FP64, so such a decision is a counted near-tie.
// Segment increment: a sweep entered with w (largest entry 0) that agrees at
// chunk c with shift sum h(c) adds h(c) + J - h1(c), J and h1 launch 1's total
// and chunk-c shift sums.  The second sweep never runs a segment's last chunk,
// whose vector the next segment reads, except in the last segment.
constexpr int VSEG = 16;          // chunks per segment
constexpr int VIT_VMAX = 12;      // chunks a second sweep may run
template <typename R>
struct VitAgree;
template <>
struct VitAgree<double> {
    static constexpr double eps = 2.5e-13;   // a quarter of the near-tie threshold
};
template <>
struct VitAgree<float> {
    static constexpr float eps = 1.52587890625e-05f;   // 2^-16
};

template <typename R, int NMAX, int FAM>
struct VitSweep {
    const StagedModel<R> &m;
    ObsRef o;
    R (*lsh)[NMAX + 1];
    double *csh;
    R *dsh;
    R col[NMAX];
    int j, N;
    bool live;

    __device__ __forceinline__ VitSweep(const StagedModel<R> &m_, ObsRef o_, R (*lsh_)[NMAX + 1],
                                        double *csh_, R *dsh_)
        : m(m_), o(o_), lsh(lsh_), csh(csh_), dsh(dsh_) {
        j = threadIdx.x;
        N = m.N;
        live = j < N;
#pragma unroll
        for (int i = 0; i < NMAX; ++i) col[i] = (live && i < N) ? m.lA[i * N + j] : neg_inf<R>();
    }

    // Steps [ta, tb) of the sequence at row off (T steps, first chunk cb0),
    // from the lane's shifted score d (ta = 0: from log pi).  Writes psi of
    // each step it runs.  At each chunk end c: with CMP and c >= cmin,
    // compares d with vd[c] and stops at the first agreement (*at = c, *h1 =
    // voff[c]); with STV stores d and the shift sum into vd[c], voff[c].  *h
    // is the shift sum at the stop or the range's end.  Returns whether it
    // stopped at an agreement.
    __device__ __forceinline__ bool run(R &d, bool &bad, bool &dead, int64_t off, int64_t T,
                                        int cb0, int64_t ta, int64_t tb, bool cmp, bool stv,
                                        int cmin, uint8_t *psi, R *vd, double *voff, double *h,
                                        double *h1, int *at) const {
        const R ninf = neg_inf<R>();
        double offset = 0.0;
        bool stop = false;
        for (int64_t w0 = ta; w0 < tb; w0 += VK) {
            const int wn = (int)((tb - w0) < VK ? (tb - w0) : VK);
            const int c = cb0 + (int)(w0 / VK);
            __syncthreads();
            if (j < wn) csh[j] = vit_tab_step<R, NMAX, FAM>(m, o, off + w0 + j, &lsh[j][0], &bad);
            __syncthreads();
            R sv = ninf;
            double so = 0.0;
            if (cmp) {   // the stored vector of this window's chunk end, requested now
                sv = vd[(size_t)c * 64 + j];
                so = voff[c];
            }
            for (int s = 0; s < wn; ++s) {
                const int64_t t = w0 + s;
                const R lt = live ? lsh[s][j] : ninf;
                R nd;
                if (t == 0) {
                    nd = live ? (R)(m.lpi[j] + lt) : ninf;
                } else {
                    dsh[j] = d;
                    wave_lds_order();
                    // max over predecessors by a pairwise tree over contiguous
                    // blocks (log2 NMAX dependent levels); the right block wins
                    // only if strictly larger, so ties keep the lowest index.
                    // The runner-up value rides along (the second largest of the
                    // candidates, whatever their order).  Entries past N hold
                    // -inf (col and the dead lanes' d).
                    R vv[NMAX], v2[NMAX];
                    int aa[NMAX];
#pragma unroll
                    for (int i = 0; i < NMAX; ++i) {
                        vv[i] = dsh[i] + col[i];
                        v2[i] = ninf;
                        aa[i] = i;
                    }
#pragma unroll
                    for (int st = 1; st < NMAX; st *= 2) {
#pragma unroll
                        for (int k = 0; k + st < NMAX; k += 2 * st) {
                            const bool right = vv[k + st] > vv[k];
                            v2[k] = right ? fmax(vv[k], v2[k + st]) : fmax(v2[k], vv[k + st]);
                            vv[k] = right ? vv[k + st] : vv[k];
                            aa[k] = right ? aa[k + st] : aa[k];
                        }
                    }
                    const R best = vv[0];
                    const int arg = aa[0];
                    const bool tie = best - v2[0] < (R)VIT_TIE_EPS;   // -inf - -inf is NaN: not a tie
                    wave_lds_order();
                    nd = live ? (R)(best + lt) : ninf;
                    if (live) psi[(off + t) * N + j] = (uint8_t)(arg | (tie ? 128 : 0));
                }
                const R mt = wave_max_r(nd);
                if (mt == ninf) dead = true;
                offset += (double)mt + csh[s];
                d = (mt == ninf) ? ninf : nd - mt;
                if (s == wn - 1 && ((t + 1) % VK == 0 || t + 1 == T)) {   // chunk end
                    if (cmp && c >= cmin) {
                        const bool ok = d == sv || fabs(d - sv) <= VitAgree<R>::eps;
                        if (__ballot(!ok) == 0 && !dead) {
                            *h = offset;
                            *h1 = so;
                            *at = c;
                            stop = true;
                        }
                    }
                    if (stv) {
                        vd[(size_t)c * 64 + j] = d;
                        if (j == 0) voff[c] = offset;
                    }
                }
            }
            if (stop) break;
        }
        if (!stop) *h = offset;
        return stop;
    }

    // final state of the shifted score vector d: lowest argmax, and whether
    // its best and second-best entries form a near-tie (lane 0 holds both)
    __device__ __forceinline__ int final_state(R d, bool *near) const {
        const R ninf = neg_inf<R>();
        R best = ninf, second = ninf;
        int q = 0;
        __syncthreads();
        dsh[j] = d;
        __syncthreads();
        if (j == 0) {
            for (int i = 0; i < N; ++i) {
                if (dsh[i] > best) {
                    second = best;
                    best = dsh[i];
                    q = i;
                } else if (dsh[i] > second) {
                    second = dsh[i];
                }
            }
        }
        *near = best - second < (R)VIT_TIE_EPS;
        return q;
    }
};

struct VitSegArgs {
    const SuperDesc *sdesc;   // [SC] segments
    const int *sbase;         // [B+1]
    void *vd;                 // [C x 64] R  shifted score vector at each chunk end (launch 1)
    double *voff;             // [C]  launch-1 shift sum at each chunk end
    double *J;                // [SC] launch-1 shift sum over the segment
    double *inc;              // [SC] increment found by the second sweep
    int32_t *flag;            // [SC] bit 0 invalid observation, bit 1 no path
    int32_t *ver;             // [SC] second sweep agreed
    int32_t *lim;             // [SC] first chunk whose psi launch 1 wrote and nothing rewrote
};

__device__ __forceinline__ void vit_result(int64_t b, bool bad, bool dead, double score, int q,
                                           bool near, double *logp, uint8_t *qlast,
                                           int32_t *n_ties) {
    if (bad) {   // a non-finite observation anywhere makes the sequence undecodable
        logp[b] = __builtin_nan("");
        qlast[b] = 255;
        if (n_ties) n_ties[b] = 0;
    } else if (dead) {
        logp[b] = -__builtin_inf();
        qlast[b] = 255;
        if (n_ties) n_ties[b] = 0;
    } else {
        logp[b] = score;
        qlast[b] = (uint8_t)q;
        if (n_ties) n_ties[b] = near ? 1 : 0;
    }
}

// Launch 1: one wave per segment.  A sequence of one segment is finished here.
template <typename R, int NMAX, int FAM>
__global__ __launch_bounds__(64) void k_vit_forward(StagedModel<R> m, ObsRef o, VitSegArgs sa,
                                                    uint8_t *__restrict__ psi,
                                                    double *__restrict__ logp,
                                                    uint8_t *__restrict__ qlast,
                                                    int32_t *__restrict__ n_ties) {
    __shared__ R lsh[VK][NMAX + 1];
    __shared__ double csh[VK];
    __shared__ __align__(16) R dsh[64];
    const int seg = blockIdx.x;
    const SuperDesc sd = sa.sdesc[seg];
    const int64_t ta = sd.t0, tb = min((int64_t)sd.T, (int64_t)sd.t0 + (int64_t)sd.n * VK);
    const int cb0 = sd.lo - sd.t0 / VK;
    const bool tail = tb == sd.T;
    VitSweep<R, NMAX, FAM> w(m, o, lsh, csh, dsh);
    R d = w.live ? (R)0 : neg_inf<R>();
    bool bad = false, dead = false;
    double h, h1;
    int at;
    w.run(d, bad, dead, sd.off, sd.T, cb0, ta, tb, false, true, 0, psi, (R *)sa.vd, sa.voff, &h,
          &h1, &at);
    const bool badw = __any(bad);
    if (sd.head && tail) {
        bool near;
        const int q = w.final_state(d, &near);
        if (w.j == 0) vit_result(sd.b, badw, dead, h, q, near, logp, qlast, n_ties);
    } else if (w.j == 0) {
        sa.J[seg] = dead ? -__builtin_inf() : h;
        sa.flag[seg] = (badw ? 1 : 0) | (dead ? 2 : 0);
    }
}

// Launch 2: the second sweep of every segment after the first.
template <typename R, int NMAX, int FAM>
__global__ __launch_bounds__(64) void k_vit_verify(StagedModel<R> m, ObsRef o, VitSegArgs sa,
                                                   uint8_t *__restrict__ psi) {
    __shared__ R lsh[VK][NMAX + 1];
    __shared__ double csh[VK];
    __shared__ __align__(16) R dsh[64];
    const int seg = blockIdx.x;
    const SuperDesc sd = sa.sdesc[seg];
    const int64_t ta = sd.t0, tb = min((int64_t)sd.T, (int64_t)sd.t0 + (int64_t)sd.n * VK);
    const int cb0 = sd.lo - sd.t0 / VK;
    const bool tail = tb == sd.T;
    if (sd.head) {
        if (threadIdx.x == 0) {
            sa.ver[seg] = 1;
            sa.lim[seg] = sd.lo;
        }
        return;
    }
    const int nv = tail ? sd.n : min(VIT_VMAX, sd.n - 1);
    VitSweep<R, NMAX, FAM> w(m, o, lsh, csh, dsh);
    R *vd = (R *)sa.vd;
    R d = vd[(size_t)(sd.lo - 1) * 64 + w.j];
    const bool enter = __ballot(d != neg_inf<R>()) != 0;   // the previous segment has a path
    int ok = 0, lim = sd.lo + max(nv, 0);
    if (enter && nv > 0) {
        bool bad = false, dead = false;
        double h, h1;
        int at;
        if (w.run(d, bad, dead, sd.off, sd.T, cb0, ta, tail ? tb : ta + (int64_t)nv * VK, true,
                  false, 0, psi, vd, sa.voff, &h, &h1, &at)) {
            ok = 1;
            lim = at;
            if (threadIdx.x == 0) sa.inc[seg] = h + sa.J[seg] - h1;
        } else if (tail) {
            // the whole last segment from the right entering vector: its psi,
            // increment and final vector (read by nothing else) are right
            ok = 1;
            vd[(size_t)(sd.lo + sd.n - 1) * 64 + w.j] = d;
            if (threadIdx.x == 0) sa.inc[seg] = dead ? -__builtin_inf() : h;
        }
    }
    if (threadIdx.x == 0) {
        sa.ver[seg] = ok;
        sa.lim[seg] = lim;
    }
}

// Launch 3: one wave per sequence of several segments.
template <typename R, int NMAX, int FAM>
__global__ __launch_bounds__(64) void k_vit_fixup(StagedModel<R> m, ObsRef o, VitSegArgs sa,
                                                  uint8_t *__restrict__ psi,
                                                  double *__restrict__ logp,
                                                  uint8_t *__restrict__ qlast,
                                                  int32_t *__restrict__ n_ties) {
    __shared__ R lsh[VK][NMAX + 1];
    __shared__ double csh[VK];
    __shared__ __align__(16) R dsh[64];
    const int b = blockIdx.x;
    const int s0 = sa.sbase[b], s1 = sa.sbase[b + 1];
    if (s1 - s0 <= 1) return;
    VitSweep<R, NMAX, FAM> w(m, o, lsh, csh, dsh);
    R *vd = (R *)sa.vd;
    const int lane = threadIdx.x;
    double score = 0.0;
    bool anybad = false, dead = false, ok = true, have = false;
    R d = neg_inf<R>();
    int last = 0;   // chunk holding the final vector when not in d
    for (int g0 = s0; g0 < s1; g0 += 64) {
        // the flags of 64 segments at a time, one per lane, requested together
        const int sq = min(g0 + lane, s1 - 1);
        const int qfl = sa.flag[sq], qver = sa.ver[sq];
        const double qinc = sq == s0 ? sa.J[s0] : sa.inc[sq];
        const int cnt = min(64, s1 - g0);
        for (int k = 0; k < cnt; ++k) {
            const int s = g0 + k;
            const int fl = __builtin_amdgcn_readlane(qfl, k);
            anybad |= (fl & 1) != 0;
            if (anybad || dead) continue;
            const SuperDesc sd = sa.sdesc[s];
            last = sd.lo + sd.n - 1;
            if (s == s0 || (ok && __builtin_amdgcn_readlane(qver, k))) {
                const uint64_t u = __builtin_bit_cast(uint64_t, qinc);
                const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, k);
                const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), k);
                score += __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
                if (!(score > -__builtin_inf())) dead = true;
                have = false;
                continue;
            }
            const int64_t ta = sd.t0, tb = min((int64_t)sd.T, (int64_t)sd.t0 + (int64_t)sd.n * VK);
            const int cb0 = sd.lo - sd.t0 / VK;
            if (!have) d = vd[(size_t)(sd.lo - 1) * 64 + w.j];
            if (__ballot(d != neg_inf<R>()) == 0) {
                dead = true;
                continue;
            }
            bool bad = false, dd = false;
            double h, h1;
            int at;
            if (w.run(d, bad, dd, sd.off, sd.T, cb0, ta, tb, true, false, sa.lim[s], psi, vd,
                      sa.voff, &h, &h1, &at)) {
                score += h + sa.J[s] - h1;
                ok = true;
                have = false;
            } else {
                score += h;
                ok = false;
                have = true;
                if (dd) dead = true;
            }
        }
    }
    if (!have) d = vd[(size_t)last * 64 + w.j];
    bool near;
    const int q = w.final_state(d, &near);
    if (lane == 0) vit_result(b, anybad, dead, score, q, near, logp, qlast, n_ties);
}

// J[c][j] for chunk c covering steps [t0, t1): follow psi from (t1 - 1, j)
// back through step t0 (t0 >= 1) or down to step 0 (first chunk).
__global__ __launch_bounds__(64) void k_vit_jump(const ChunkDesc *__restrict__ cdesc, int N,
                                                 const uint8_t *__restrict__ psi,
                                                 uint8_t *__restrict__ J) {
    __shared__ uint8_t blk[VK * 64];
    const int c = blockIdx.x;
    const ChunkDesc d = cdesc[c];
    const int tid = threadIdx.x;
    // stage the chunk's psi rows (len x N bytes)
    const int nbytes = d.len * N;
    const uint8_t *src = psi + (d.off + d.t0) * N;
    for (int k = tid; k < nbytes; k += 64) blk[k] = src[k];
    __syncthreads();
    if (tid < N) {
        int q = tid;
        const int stop = d.t0 == 0 ? 1 : 0;   // psi_0 does not exist
        for (int tt = d.len - 1; tt >= stop; --tt) q = blk[tt * N + q] & 127;
        J[(size_t)c * N + tid] = (uint8_t)q;
    }
}

// end state of every chunk: one wave per sequence walks its chunks backwards
__global__ __launch_bounds__(64) void k_vit_chain(const int *__restrict__ cbase, int N,
                                                  const uint8_t *__restrict__ qlast,
                                                  const uint8_t *__restrict__ J,
                                                  uint8_t *__restrict__ qend) {
    constexpr int PF = 8;
    const int64_t b = blockIdx.x;
    const int lane = threadIdx.x;
    const int c0 = cbase[b], c1 = cbase[b + 1];
    int q = qlast[b];
    if (q == 255) {
        for (int c = c0 + lane; c < c1; c += 64) qend[c] = 255;
        return;
    }
    int ring[PF];
#pragma unroll
    for (int k = 0; k < PF; ++k) {
        const int c = max(c1 - 1 - k, c0);
        ring[k] = lane < N ? J[(size_t)c * N + lane] : 0;
    }
    for (int s0 = 0; s0 < c1 - c0; s0 += PF) {
#pragma unroll
        for (int k = 0; k < PF; ++k) {
            const int s = s0 + k;
            const int c = c1 - 1 - s;
            const int row = ring[k];
            const int cn = max(c1 - 1 - (s + PF), c0);
            ring[k] = lane < N ? J[(size_t)cn * N + lane] : 0;
            if (c >= c0) {
                if (lane == 0) qend[c] = (uint8_t)q;
                q = __builtin_amdgcn_readlane(row, q);
            }
        }
    }
}

// path of every chunk from its end state (one lane chases, the wave stages
// psi); the near-ties met on the chunk's part of the path are added to the
// sequence's count (integer atomics: the total does not depend on the order)
__global__ __launch_bounds__(64) void k_vit_fill(const ChunkDesc *__restrict__ cdesc, int N,
                                                 const uint8_t *__restrict__ psi,
                                                 const uint8_t *__restrict__ qend,
                                                 int32_t *__restrict__ path,
                                                 int32_t *__restrict__ n_ties) {
    __shared__ uint8_t blk[VK * 64];
    __shared__ int32_t out[VK];
    const int c = blockIdx.x;
    const ChunkDesc d = cdesc[c];
    const int tid = threadIdx.x;
    const int nbytes = d.len * N;
    const uint8_t *src = psi + (d.off + d.t0) * N;
    for (int k = tid; k < nbytes; k += 64) blk[k] = src[k];
    __syncthreads();
    if (tid == 0) {
        int q = qend[c];
        if (q == 255) {
            for (int tt = 0; tt < d.len; ++tt) out[tt] = -1;
        } else {
            int ties = 0;
            for (int tt = d.len - 1; tt >= 0; --tt) {
                out[tt] = q;
                if (tt > 0 || d.t0 > 0) {
                    const int e = blk[tt * N + q];
                    ties += e >> 7;
                    q = e & 127;
                }
            }
            if (n_ties && ties) atomicAdd(n_ties + d.b, ties);
        }
    }
    __syncthreads();
    if (tid < d.len) path[d.off + d.t0 + tid] = out[tid];
}

template <typename R, int NMAX, int FAM>
static void launch_vit_forward_f(const StagedModel<R> &m, const ObsDesc &o, const VitSegArgs &sa,
                                 int SC, uint8_t *psi, double *logp, uint8_t *qlast,
                                 int32_t *n_ties, hipStream_t s) {
    const ObsRef obs{o.obs, o.obs_f64};
    {
        ProfScope ps("vit_forward", s);
        hipLaunchKernelGGL((k_vit_forward<R, NMAX, FAM>), dim3((unsigned)SC), dim3(64), 0, s, m,
                           obs, sa, psi, logp, qlast, n_ties);
    }
    if (SC > o.nseq) {   // some sequence is split
        {
            ProfScope ps("vit_verify", s);
            hipLaunchKernelGGL((k_vit_verify<R, NMAX, FAM>), dim3((unsigned)SC), dim3(64), 0, s,
                               m, obs, sa, psi);
        }
        {
            ProfScope ps("vit_fixup", s);
            hipLaunchKernelGGL((k_vit_fixup<R, NMAX, FAM>), dim3((unsigned)o.nseq), dim3(64), 0,
                               s, m, obs, sa, psi, logp, qlast, n_ties);
        }
    }
}

template <typename R, int NMAX>
static void launch_vit_forward_n(const StagedModel<R> &m, const ObsDesc &o, const VitSegArgs &sa,
                                 int SC, uint8_t *psi, double *logp, uint8_t *qlast, int32_t *nt,
                                 hipStream_t s) {
    switch (m.family) {
    case HMM_GAUSSIAN: return launch_vit_forward_f<R, NMAX, HMM_GAUSSIAN>(m, o, sa, SC, psi, logp, qlast, nt, s);
    case HMM_GAMMA: return launch_vit_forward_f<R, NMAX, HMM_GAMMA>(m, o, sa, SC, psi, logp, qlast, nt, s);
    case HMM_STUDENT_T: return launch_vit_forward_f<R, NMAX, HMM_STUDENT_T>(m, o, sa, SC, psi, logp, qlast, nt, s);
    case HMM_POISSON: return launch_vit_forward_f<R, NMAX, HMM_POISSON>(m, o, sa, SC, psi, logp, qlast, nt, s);
    case HMM_TABLE: return launch_vit_forward_f<R, NMAX, HMM_TABLE>(m, o, sa, SC, psi, logp, qlast, nt, s);
    default: return launch_vit_forward_f<R, NMAX, -1>(m, o, sa, SC, psi, logp, qlast, nt, s);
    }
}

int vit_seg_chunks() { return VSEG; }

template <typename R>
hmm_status run_viterbi(const StagedModel<R> &m, const ObsDesc &o, const int *cbase,
                       const ChunkDesc *cdesc, int C, const VitBuffers &vb, uint8_t *psi,
                       uint8_t *J, uint8_t *qlast, uint8_t *qend, int32_t *path, double *logp,
                       int32_t *n_ties, hipStream_t s) {
    if (o.nseq == 0) return HMM_OK;
    const VitSegArgs sa{vb.sdesc, vb.sbase, vb.vd, vb.voff, vb.J, vb.inc, vb.flag, vb.ver, vb.lim};
    if (m.N <= 8) launch_vit_forward_n<R, 8>(m, o, sa, vb.SC, psi, logp, qlast, n_ties, s);
    else if (m.N <= 16) launch_vit_forward_n<R, 16>(m, o, sa, vb.SC, psi, logp, qlast, n_ties, s);
    else if (m.N <= 32) launch_vit_forward_n<R, 32>(m, o, sa, vb.SC, psi, logp, qlast, n_ties, s);
    else launch_vit_forward_n<R, 64>(m, o, sa, vb.SC, psi, logp, qlast, n_ties, s);
    {
        ProfScope ps("vit_jump", s);
        hipLaunchKernelGGL(k_vit_jump, dim3((unsigned)C), dim3(64), 0, s, cdesc, m.N,
                           (const uint8_t *)psi, J);
    }
    {
        ProfScope ps("vit_chain", s);
        hipLaunchKernelGGL(k_vit_chain, dim3((unsigned)o.nseq), dim3(64), 0, s, cbase, m.N,
                           (const uint8_t *)qlast, (const uint8_t *)J, qend);
    }
    {
        ProfScope ps("vit_fill", s);
        hipLaunchKernelGGL(k_vit_fill, dim3((unsigned)C), dim3(64), 0, s, cdesc, m.N,
                           (const uint8_t *)psi, (const uint8_t *)qend, path, n_ties);
    }
    return HMM_OK;
}

template hmm_status run_viterbi<float>(const StagedModel<float> &, const ObsDesc &, const int *,
                                       const ChunkDesc *, int, const VitBuffers &, uint8_t *,
                                       uint8_t *, uint8_t *, uint8_t *, int32_t *, double *,
                                       int32_t *, hipStream_t);
template hmm_status run_viterbi<double>(const StagedModel<double> &, const ObsDesc &, const int *,
                                        const ChunkDesc *, int, const VitBuffers &, uint8_t *,
                                        uint8_t *, uint8_t *, uint8_t *, int32_t *, double *,
                                        int32_t *, hipStream_t);

}  // namespace hmmk
