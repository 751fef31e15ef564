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

// one wave per sequence; NMAX bounds the (unrolled) predecessor loop.  The
// emissions of a window of VK steps are tabulated first, one lane per step.
template <typename R, int NMAX, int FAM>
__global__ __launch_bounds__(64) void k_vit_forward(StagedModel<R> m, ObsRef o, int64_t nseq,
                                                    const int64_t *__restrict__ offsets,
                                                    uint8_t *__restrict__ psi,
                                                    double *__restrict__ logp,
                                                    uint8_t *__restrict__ qlast,
                                                    int32_t *__restrict__ n_ties, R tie_eps) {
    __shared__ R lsh[VK][NMAX + 1];
    __shared__ double csh[VK];
    __shared__ __align__(16) R dsh[64];
    const int64_t b = blockIdx.x;
    const int j = threadIdx.x;
    const int N = m.N;
    const bool live = j < N;
    const int64_t off = offsets[b], T = offsets[b + 1] - off;
    R col[NMAX];
#pragma unroll
    for (int i = 0; i < NMAX; ++i) col[i] = (live && i < N) ? m.lA[i * N + j] : neg_inf<R>();
    const R ninf = neg_inf<R>();
    bool bad = false, dead = false;
    double offset = 0.0;
    R d = ninf;
    for (int64_t w0 = 0; w0 < T; w0 += VK) {
        const int wn = (int)((T - w0) < VK ? (T - w0) : VK);
        __syncthreads();
        if (j < wn) csh[j] = vit_tab_step<R, NMAX, FAM>(m, o, off + w0 + j, &lsh[j][0], &bad);
        __syncthreads();
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
                const bool tie = best - v2[0] < tie_eps;   // -inf - -inf is NaN: not a tie
                wave_lds_order();
                nd = live ? (R)(best + lt) : ninf;
                if (live) psi[(off + t) * N + j] = (uint8_t)(arg | (tie ? 128 : 0));
            }
            const R mt = wave_max_r(nd);
            if (mt == ninf) dead = true;
            offset += (double)mt + csh[s];
            d = (mt == ninf) ? ninf : nd - mt;
        }
    }
    // final state: lowest argmax; a near-tie there counts once
    R best = ninf, second = ninf;
    int q = 0;
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
        logp[b] = dead ? -__builtin_inf() : offset + (double)best;
        qlast[b] = (uint8_t)(dead ? 255 : q);
        if (n_ties) n_ties[b] = (!dead && best - second < tie_eps) ? 1 : 0;
    }
    // a non-finite observation anywhere makes the whole sequence undecodable
    const int badw = __any(bad);
    if (j == 0 && badw) {
        logp[b] = __builtin_nan("");
        qlast[b] = 255;
        if (n_ties) n_ties[b] = 0;
    }
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
static void launch_vit_forward_f(const StagedModel<R> &m, const ObsDesc &o, uint8_t *psi,
                                 double *logp, uint8_t *qlast, int32_t *n_ties, hipStream_t s) {
    hipLaunchKernelGGL((k_vit_forward<R, NMAX, FAM>), dim3((unsigned)o.nseq), dim3(64), 0, s, m,
                       ObsRef{o.obs, o.obs_f64}, o.nseq, o.offsets, psi, logp, qlast, n_ties,
                       (R)VIT_TIE_EPS);
}

template <typename R, int NMAX>
static void launch_vit_forward_n(const StagedModel<R> &m, const ObsDesc &o, uint8_t *psi,
                                 double *logp, uint8_t *qlast, int32_t *nt, hipStream_t s) {
    switch (m.family) {
    case HMM_GAUSSIAN: return launch_vit_forward_f<R, NMAX, HMM_GAUSSIAN>(m, o, psi, logp, qlast, nt, s);
    case HMM_GAMMA: return launch_vit_forward_f<R, NMAX, HMM_GAMMA>(m, o, psi, logp, qlast, nt, s);
    case HMM_STUDENT_T: return launch_vit_forward_f<R, NMAX, HMM_STUDENT_T>(m, o, psi, logp, qlast, nt, s);
    case HMM_POISSON: return launch_vit_forward_f<R, NMAX, HMM_POISSON>(m, o, psi, logp, qlast, nt, s);
    case HMM_TABLE: return launch_vit_forward_f<R, NMAX, HMM_TABLE>(m, o, psi, logp, qlast, nt, s);
    default: return launch_vit_forward_f<R, NMAX, -1>(m, o, psi, logp, qlast, nt, s);
    }
}

template <typename R>
static void launch_vit_forward(const StagedModel<R> &m, const ObsDesc &o, uint8_t *psi,
                               double *logp, uint8_t *qlast, int32_t *nt, hipStream_t s) {
    if (m.N <= 8) launch_vit_forward_n<R, 8>(m, o, psi, logp, qlast, nt, s);
    else if (m.N <= 16) launch_vit_forward_n<R, 16>(m, o, psi, logp, qlast, nt, s);
    else if (m.N <= 32) launch_vit_forward_n<R, 32>(m, o, psi, logp, qlast, nt, s);
    else launch_vit_forward_n<R, 64>(m, o, psi, logp, qlast, nt, s);
}

template <typename R>
hmm_status run_viterbi(const StagedModel<R> &m, const ObsDesc &o, const int *cbase,
                       const ChunkDesc *cdesc, int C, uint8_t *psi, uint8_t *J, uint8_t *qlast,
                       uint8_t *qend, int32_t *path, double *logp, int32_t *n_ties,
                       hipStream_t s) {
    if (o.nseq == 0) return HMM_OK;
    {
        ProfScope ps("vit_forward", s);
        launch_vit_forward<R>(m, o, psi, logp, qlast, n_ties, s);
    }
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
                                       const ChunkDesc *, int, uint8_t *, uint8_t *, uint8_t *,
                                       uint8_t *, int32_t *, double *, int32_t *, hipStream_t);
template hmm_status run_viterbi<double>(const StagedModel<double> &, const ObsDesc &, const int *,
                                        const ChunkDesc *, int, uint8_t *, uint8_t *, uint8_t *,
                                        uint8_t *, int32_t *, double *, int32_t *, hipStream_t);

}  // namespace hmmk
