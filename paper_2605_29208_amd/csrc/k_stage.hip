// k_stage.hip -- parameter staging, chunk planning and the fixed-order
// reduction of partial statistics.
#include <math.h>

#include "dev_common.hpp"
#include "hmm_internal.hpp"

namespace hmmk {

static inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t mv_count(int N, int D, int family) {
    if (family == HMM_DIAG_GAUSSIAN) return (size_t)2 * N * D;
    if (family == HMM_FULL_GAUSSIAN) return (size_t)N * D + (size_t)N * D * D;
    return 0;
}

size_t staged_bytes(int N, int D, int family, bool f64) {
    size_t r = f64 ? 8 : 4;
    size_t n = (size_t)N, nn = n * n;
    return align256(n * r) * 2 + align256(nn * r) * 3 + align256(n * EP_STRIDE * r) +
           align256(n * EP_STRIDE * 8) + align256(mv_count(N, D, family) * r + r) + 256 +
           align256(64 * r) + 256;
}

// Chunk plan in one block of NT threads: cbase and sbase are the exclusive
// prefix sums of the per-sequence chunk and superchunk counts.  A tile of
// NT * PER sequences takes one round of loads (each thread its PER
// consecutive sequences), a scan inside each wave through lane shuffles and
// one barrier for the wave totals, so B sequences cost about B / (NT * PER)
// load latencies.
template <int NT, int PER>
__device__ void plan_scan(const int64_t *offsets, int64_t nseq, int L, int S, int *cbase,
                          int *sbase) {
    constexpr int NW = NT / 64, TILE = NT * PER;
    __shared__ int w_nc[NW], w_ns[NW];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    int carry_c = 0, carry_s = 0;
    for (int64_t base = 0; base < nseq; base += TILE) {
        const int64_t b0 = base + (int64_t)t * PER;
        int64_t o[PER + 1];
#pragma unroll
        for (int k = 0; k <= PER; ++k) o[k] = offsets[min(b0 + k, nseq)];
        int nc[PER], ns[PER], sc = 0, ss = 0;
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const bool in = b0 + k < nseq;
            nc[k] = in ? (int)((o[k + 1] - o[k] + L - 1) / L) : 0;
            ns[k] = (nc[k] + S - 1) / S;
            sc += nc[k];
            ss += ns[k];
        }
        int ic = sc, is = ss;   // inclusive scans over the wave
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int u = __shfl_up(ic, d), v = __shfl_up(is, d);
            if (lane >= d) {
                ic += u;
                is += v;
            }
        }
        if (lane == 63) {
            w_nc[wv] = ic;
            w_ns[wv] = is;
        }
        __syncthreads();
        int cc = carry_c + ic - sc, cs = carry_s + is - ss, tc = 0, ts = 0;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if (w < wv) {
                cc += w_nc[w];
                cs += w_ns[w];
            }
            tc += w_nc[w];
            ts += w_ns[w];
        }
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            if (b0 + k < nseq) {
                cbase[b0 + k] = cc;
                sbase[b0 + k] = cs;
            }
            cc += nc[k];
            cs += ns[k];
        }
        carry_c += tc;
        carry_s += ts;
        __syncthreads();   // the wave totals are rewritten by the next tile
    }
    if (t == 0) {
        cbase[nseq] = carry_c;
        sbase[nseq] = carry_s;
    }
}

__device__ void plan_block(const PlanArgs &a) {
    plan_scan<BLOCK, 4>(a.offsets, a.nseq, a.L, a.S, a.cbase, a.sbase);
}

// Block 0 computes the initial probabilities, the per-state emission
// constants (see dev_common.hpp for their meaning), the diagonal-Gaussian
// location and -1/(2 var) vectors, the full-Gaussian means, the parameter
// check and the rescale interval.  Blocks 1 .. nmat fill A, A^T and log A in
// R (block 0 does it when nmat = 0); for the full Gaussian, block
// 1 + nmat + j forms L_j^{-1}, one thread per column.  With a plan
// (plan.nseq > 0) the last block forms the chunk plan.
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_stage(RawModel m, int nmat, PlanArgs plan, R *pi, R *A,
                                                 R *AT, R *lpi, R *lA, R *ep, double *ep64, R *mv,
                                                 int *perr, R *A8, int *nrm) {
    const int N = m.N, D = m.D;
    const int64_t NN = (int64_t)N * N;
    const int bx = blockIdx.x;
    if (plan.nseq > 0 && bx == (int)gridDim.x - 1) {
        plan_block(plan);
        return;
    }
    if (bx > nmat) {
        // L_j^{-1} column by column: L x = e_col by forward substitution (FP64),
        // the column kept in LDS (thread col owns column col)
        __shared__ double xs[64 * 64];
        const int j = bx - 1 - nmat, col = threadIdx.x;
        if (col >= D) return;
        const double *L = m.theta + (size_t)N * D + (size_t)j * D * D;
        R *Li = mv + (size_t)N * D + (size_t)j * D * D;
        for (int r = 0; r < D; ++r) {
            double x = 0.0;
            if (r >= col) {
                double acc = (r == col) ? 1.0 : 0.0;
                for (int q = col; q < r; ++q) acc -= L[r * D + q] * xs[q * 64 + col];
                x = acc / L[r * D + r];
            }
            xs[r * 64 + col] = x;
            Li[r * D + col] = (R)x;
        }
        return;
    }
    if (bx > 0 || nmat == 0) {
        const int64_t stride = (int64_t)(nmat > 0 ? nmat : 1) * BLOCK;
        for (int64_t k = (int64_t)(bx > 0 ? bx - 1 : 0) * BLOCK + threadIdx.x; k < NN; k += stride) {
            const double l = m.log_A[k];
            const R av = (R)exp(l);
            A[k] = av;
            lA[k] = (R)l;
            AT[(k % N) * N + k / N] = av;
        }
        if (bx > 0) return;
    }
    int bad = 0;
    __shared__ double amin_sh[BLOCK];
    // min log a_ij (exp is monotone: min a_ij = exp(min log a_ij)).  Only the
    // transfer-matrix path (N <= 8) uses the rescale interval; larger models
    // get interval 1 without the scan.
    double lmin = NN <= 4096 ? 0.0 : -__builtin_inf();
    for (int64_t k = threadIdx.x; k < (NN <= 4096 ? NN : 0); k += BLOCK) lmin = fmin(lmin, m.log_A[k]);
    amin_sh[threadIdx.x] = lmin;
    for (int k = threadIdx.x; k < 64; k += BLOCK) {
        int i = k / 8, j = k % 8;
        A8[k] = (i < N && j < N) ? (R)exp(m.log_A[i * N + j]) : (R)0;
    }
    for (int j = threadIdx.x; j < N; j += BLOCK) {
        double l = m.log_pi[j];
        pi[j] = (R)exp(l);
        lpi[j] = (R)l;
    }

    const double *th = m.theta;
    const double kLog2Pi = 1.8378770664093454835606594728112;
    for (int j = threadIdx.x; j < N; j += BLOCK) {
        double c[EP_STRIDE] = {0, 0, 0, 0, 0, 0, 0, 0};
        switch (m.family) {
        case HMM_GAUSSIAN: {
            double mu = th[j], var = th[N + j];
            bad |= !(var > 0.0) || !isfinite(mu);
            c[0] = mu;
            c[1] = -0.5 / var;
            c[2] = -0.5 * log(2.0 * M_PI * var);
            break;
        }
        case HMM_GAMMA: {
            double a = th[j], b = th[N + j];
            bad |= !(a > 0.0) || !(b > 0.0);
            c[0] = a * log(b) - lgamma(a);
            c[1] = a - 1.0;
            c[2] = -b;
            break;
        }
        case HMM_STUDENT_T: {
            double mu = th[j], s = th[N + j], nu = th[2 * N + j];
            bad |= !(s > 0.0) || !(nu > 0.0) || !isfinite(mu);
            c[0] = mu;
            c[1] = 1.0 / (nu * s * s);
            c[2] = -0.5 * (nu + 1.0);
            c[3] = lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) - 0.5 * log(nu * M_PI * s * s);
            c[4] = (nu + 1.0) / nu;
            break;
        }
        case HMM_POISSON: {
            double lam = th[j];
            bad |= !(lam > 0.0);
            c[0] = log(lam);
            c[1] = -lam;
            break;
        }
        case HMM_DIAG_GAUSSIAN: {
            double s = 0.0;
            for (int d = 0; d < D; ++d) {
                double mu = th[(size_t)j * D + d], var = th[(size_t)N * D + (size_t)j * D + d];
                bad |= !(var > 0.0) || !isfinite(mu);
                s += -0.5 * log(2.0 * M_PI * var);
                mv[(size_t)j * D + d] = (R)mu;
                mv[(size_t)N * D + (size_t)j * D + d] = (R)(-0.5 / var);
            }
            c[0] = s;
            break;
        }
        case HMM_FULL_GAUSSIAN: {
            const double *L = th + (size_t)N * D + (size_t)j * D * D;
            double logdet = 0.0;
            for (int d = 0; d < D; ++d) {
                mv[(size_t)j * D + d] = (R)th[(size_t)j * D + d];
                bad |= !(L[d * D + d] > 0.0);
                logdet += log(L[d * D + d]);
            }
            c[0] = -logdet - 0.5 * D * kLog2Pi;
            break;
        }
        default:
            break;
        }
        for (int k = 0; k < EP_STRIDE; ++k) {
            ep[j * EP_STRIDE + k] = (R)c[k];
            ep64[j * EP_STRIDE + k] = c[k];
        }
    }
    int any = __syncthreads_or(bad);
    for (int o = BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o)
            amin_sh[threadIdx.x] = fmin(amin_sh[threadIdx.x], amin_sh[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *perr = any;
        const double a = exp(amin_sh[0]);
        // The largest entry of a product of forward-type steps (row vector times
        // A diag(e), max e = 1) grows by at most N <= 1024 = 2^10 and shrinks by
        // at most min a_ij per step, so rescaling every 4 steps keeps single
        // precision in range when min a_ij >= 2^-25 (2^-200 for double).
        const double lim4 = sizeof(R) == 4 ? 0x1p-25 : 0x1p-200;
        const double lim2 = sizeof(R) == 4 ? 0x1p-50 : 0x1p-400;
        *nrm = a >= lim4 ? 4 : (a >= lim2 ? 2 : 1);
    }
}

template <typename R>
void launch_stage(const RawModel &m, void *region, StagedModel<R> *out, hipStream_t s,
                  const PlanArgs *plan) {
    size_t r = sizeof(R);
    size_t n = (size_t)m.N, nn = n * n;
    char *p = (char *)region;
    R *pi = (R *)p; p += align256(n * r);
    R *lpi = (R *)p; p += align256(n * r);
    R *A = (R *)p; p += align256(nn * r);
    R *AT = (R *)p; p += align256(nn * r);
    R *lA = (R *)p; p += align256(nn * r);
    R *ep = (R *)p; p += align256(n * EP_STRIDE * r);
    double *ep64 = (double *)p; p += align256(n * EP_STRIDE * 8);
    R *mv = (R *)p; p += align256(mv_count(m.N, m.D, m.family) * r + r);
    int *perr = (int *)p; p += 256;
    R *A8 = (R *)p; p += align256(64 * r);
    int *nrm = (int *)p;
    {
        ProfScope ps("stage", s);
        // small matrices are filled by block 0 itself
        const int64_t nn2 = (int64_t)m.N * m.N;
        const int nmat = nn2 <= 4 * BLOCK ? 0 : (int)((nn2 + BLOCK - 1) / BLOCK < 512 ? (nn2 + BLOCK - 1) / BLOCK : 512);
        const int nfull = m.family == HMM_FULL_GAUSSIAN ? m.N : 0;
        const PlanArgs pa = plan ? *plan : PlanArgs{nullptr, 0, 0, 0, nullptr, nullptr};
        const int nplan = pa.nseq > 0 ? 1 : 0;
        hipLaunchKernelGGL(k_stage<R>, dim3((unsigned)(1 + nmat + nfull + nplan)), dim3(BLOCK), 0,
                           s, m, nmat, pa, pi, A, AT, lpi, lA, ep, ep64, mv, perr, A8, nrm);
    }
    out->N = m.N;
    out->D = m.D;
    out->family = m.family;
    out->pi = pi;
    out->A = A;
    out->AT = AT;
    out->lpi = lpi;
    out->lA = lA;
    out->ep = ep;
    out->ep64 = ep64;
    out->mv = mv;
    out->perr = perr;
    out->A8 = A8;
    out->nrm = nrm;
}

template void launch_stage<float>(const RawModel &, void *, StagedModel<float> *, hipStream_t,
                                  const PlanArgs *);
template void launch_stage<double>(const RawModel &, void *, StagedModel<double> *, hipStream_t,
                                   const PlanArgs *);

// cbase[b] = sum_{b' < b} ceil(T_b' / L) and sbase[b] = sum_{b' < b}
// ceil(nchunks_b' / S), one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_plan_chunks(const int64_t *offsets, int64_t nseq, int L,
                                                      int S, int *cbase, int *sbase) {
    plan_scan<1024, 4>(offsets, nseq, L, S, cbase, sbase);
}

void launch_plan_chunks(const int64_t *offsets, int64_t nseq, int L, int S, int *cbase,
                        int *sbase, hipStream_t s) {
    ProfScope ps("plan_chunks", s);
    hipLaunchKernelGGL(k_plan_chunks, dim3(1), dim3(1024), 0, s, offsets, nseq, L, S, cbase, sbase);
}

// Last sequence b < nseq with base[b] <= c0 (base non-decreasing, base[0] = 0
// <= c0), found by the whole block: each round probes BLOCK evenly spaced
// entries at once and keeps the bracket between the last probe that passes
// and the next one, so B sequences take about log_BLOCK(B) dependent loads.
__device__ __forceinline__ int block_find_seq(const int *base, int nseq, int c0) {
    int lo = 0, hi = nseq - 1;
    while (lo < hi) {   // uniform
        const int64_t span = (int64_t)(hi - lo) + 1;
        const int pk = lo + (int)(((int64_t)threadIdx.x * span) / BLOCK);
        // the probes are non-decreasing in the thread index and probe 0 (= lo)
        // passes, so the passing ones are threads 0 .. cnt - 1
        const int cnt = __syncthreads_count(base[pk] <= c0);
        const int k = cnt - 1;
        const int plo = lo + (int)(((int64_t)k * span) / BLOCK);
        const int phi = (k + 1 < BLOCK) ? lo + (int)(((int64_t)(k + 1) * span) / BLOCK) - 1 : hi;
        lo = plo;
        hi = phi;
    }
    return lo;
}

// Descriptors of the chunks (i < C) and superchunks (i < SC), thread i of the
// grid for entry i.  A block's BLOCK consecutive entries belong to at most
// BLOCK consecutive sequences (every sequence has one chunk and one superchunk
// or more), so after the block finds the first one, the window of BLOCK + 1
// prefix entries that follows is staged in LDS and each thread searches it.
__device__ __forceinline__ int window_find_seq(const int *base, int nseq, int i0, int i, int *win) {
    const int bl = block_find_seq(base, nseq, i0);
    const int nw = min(BLOCK, nseq - bl);   // sequences in the window
    for (int k = threadIdx.x; k <= nw; k += BLOCK) win[k] = base[bl + k];
    __syncthreads();
    int lo = 0, hi = nw - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (win[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return bl + lo;
}

__global__ __launch_bounds__(BLOCK) void k_chunk_desc(const int64_t *offsets, int64_t nseq, int L,
                                                      int S, const int *cbase, const int *sbase,
                                                      int C, int SC, ChunkDesc *cdesc,
                                                      SuperDesc *sdesc) {
    __shared__ int win[BLOCK + 1];
    const int i0 = blockIdx.x * BLOCK;
    const int i = i0 + threadIdx.x;
    if (i0 < C) {   // uniform
        const int b = window_find_seq(cbase, (int)nseq, i0, min(i, C - 1), win);
        if (i < C) {
            int64_t off = offsets[b];
            int T = (int)(offsets[b + 1] - off);
            ChunkDesc d;
            d.off = off;
            d.b = b;
            d.t0 = (i - cbase[b]) * L;
            d.len = min(L, T - d.t0);
            d.pad0 = 0;
            d.pad1 = 0;
            cdesc[i] = d;
        }
        __syncthreads();   // the window is reused below
    }
    if (i0 < SC) {   // uniform
        const int b = window_find_seq(sbase, (int)nseq, i0, min(i, SC - 1), win);
        if (i < SC) {
            SuperDesc d;
            d.off = offsets[b];
            d.b = b;
            d.lo = cbase[b] + (i - sbase[b]) * S;
            d.n = min(S, cbase[b + 1] - d.lo);
            d.head = (i == sbase[b]) ? 1 : 0;
            d.t0 = (d.lo - cbase[b]) * L;
            d.T = (int)(offsets[b + 1] - d.off);
            sdesc[i] = d;
        }
    }
}

void launch_chunk_desc(const int64_t *offsets, int64_t nseq, int L, int S, const int *cbase,
                       const int *sbase, int C, int SC, ChunkDesc *cdesc, SuperDesc *sdesc,
                       hipStream_t s) {
    ProfScope ps("chunk_desc", s);
    const int n = C > SC ? C : SC;
    hipLaunchKernelGGL(k_chunk_desc, dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, offsets,
                       nseq, L, S, cbase, sbase, C, SC, cdesc, sdesc);
}

// Pooled statistics from per-part rows partial[p * S + s] (p < nparts), in a
// fixed order so that repeated calls give identical bits.  A block covers 64
// consecutive entries (one per lane, so every load is a coalesced 512-byte
// row segment) and its four waves take interleaved parts: wave w sums parts
// w, w + 4, ... of its range, with RED_U independent loads in flight, and the
// four wave sums are added in wave order.  More than RED_G parts are first
// summed in groups of RED_G (pass 1), then the group rows (pass 2).  Entry 0
// is the sum of the log-likelihoods of the sequences with status 0 (a block
// tree of its own).
constexpr int RED_G = 64;
constexpr int RED_U = 16;   // loads in flight per lane (a group's rows in one round)

int64_t reduce_scratch_len(int64_t nparts, int64_t S) {
    return nparts > RED_G ? ((nparts + RED_G - 1) / RED_G) * S : 0;
}

// sum of rows[r * S + s] over r in [r0, r1), fixed order, result valid in wave 0
__device__ __forceinline__ double block_rows_sum(const double *__restrict__ rows, int r0, int r1,
                                                 int64_t S, int64_t s, bool live) {
    __shared__ double sh[BLOCK / 64][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double acc = 0.0;
    if (live) {
        for (int r = r0 + w; r < r1; r += (BLOCK / 64) * RED_U) {
            double v[RED_U];
#pragma unroll
            for (int u = 0; u < RED_U; ++u) {
                // clamped unconditional loads (r < r1), so all are in flight
                const int q = r + u * (BLOCK / 64);
                const double x = rows[(int64_t)min(q, r1 - 1) * S + s];
                v[u] = q < r1 ? x : 0.0;
            }
            __builtin_amdgcn_sched_barrier(0);   // keep every load ahead of the sums
#pragma unroll
            for (int u = 0; u < RED_U; ++u) acc += v[u];
        }
    }
    sh[w][lane] = acc;
    __syncthreads();
    double t = sh[0][lane];
#pragma unroll
    for (int q = 1; q < BLOCK / 64; ++q) t += sh[q][lane];
    return t;
}

__global__ __launch_bounds__(BLOCK) void k_reduce_parts(const double *__restrict__ partial,
                                                       int nparts, int64_t S,
                                                       double *__restrict__ red) {
    const int64_t s = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const int g = blockIdx.y;
    const int r1 = min(nparts, (g + 1) * RED_G);
    const double t = block_rows_sum(partial, g * RED_G, r1, S, s, s < S);
    if (threadIdx.x < 64 && s < S) red[(int64_t)g * S + s] = t;
}

__global__ __launch_bounds__(BLOCK) void k_reduce_final(const double *__restrict__ rows, int nrows,
                                                       int64_t S, const double *loglik,
                                                       const int32_t *status, int64_t nseq,
                                                       double *stats) {
    if (blockIdx.x == gridDim.x - 1) {
        __shared__ double sh[BLOCK];
        // a lane's sequences b = lane, lane + BLOCK, ... in order, eight
        // loads of each array in flight at a time
        constexpr int U = 8;
        double acc = 0.0;
        for (int64_t b0 = threadIdx.x; b0 < nseq; b0 += (int64_t)BLOCK * U) {
            double lv[U];
            int32_t sv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t b = min(b0 + (int64_t)u * BLOCK, nseq - 1);
                lv[u] = loglik[b];
                sv[u] = status[b];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (b0 + (int64_t)u * BLOCK < nseq && sv[u] == 0) acc += lv[u];
        }
        sh[threadIdx.x] = acc;
        __syncthreads();
        for (int o = BLOCK / 2; o > 0; o >>= 1) {
            if (threadIdx.x < (unsigned)o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) stats[0] = sh[0];
        return;
    }
    const int64_t s = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
    const double t = block_rows_sum(rows, 0, nrows, S, s, s >= 1 && s < S);
    if (threadIdx.x < 64 && s >= 1 && s < S) stats[s] = t;
}

void launch_reduce_stats(const double *partial, int nparts, int64_t S, const double *loglik,
                         const int32_t *status, int64_t nseq, double *stats, double *red,
                         hipStream_t s) {
    ProfScope ps("reduce_stats", s);
    const unsigned sb = (unsigned)((S + 63) / 64);
    const double *rows = partial;
    int nrows = nparts;
    if (nparts > RED_G) {
        const int ng = (nparts + RED_G - 1) / RED_G;
        hipLaunchKernelGGL(k_reduce_parts, dim3(sb, (unsigned)ng), dim3(BLOCK), 0, s, partial,
                           nparts, S, red);
        rows = red;
        nrows = ng;
    }
    hipLaunchKernelGGL(k_reduce_final, dim3(sb + 1), dim3(BLOCK), 0, s, rows, nrows, S, loglik,
                       status, nseq, stats);
}

}  // namespace hmmk

namespace hmmk {

// posterior decoding: path[r] = lowest argmax_j gamma[r, j]
template <typename R>
__global__ __launch_bounds__(BLOCK) void k_argmax_rows(const R *g, int64_t rows, int N,
                                                      int32_t *path) {
    const int64_t r = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= rows) return;
    const R *row = g + r * N;
    int q = 0;
    R best = row[0];
    for (int j = 1; j < N; ++j)
        if (row[j] > best) {
            best = row[j];
            q = j;
        }
    path[r] = q;
}

void launch_argmax_rows(const void *gamma, bool f64, int64_t rows, int N, int32_t *path,
                        hipStream_t s) {
    dim3 grid((unsigned)((rows + BLOCK - 1) / BLOCK));
    if (f64)
        hipLaunchKernelGGL(k_argmax_rows<double>, grid, dim3(BLOCK), 0, s, (const double *)gamma,
                           rows, N, path);
    else
        hipLaunchKernelGGL(k_argmax_rows<float>, grid, dim3(BLOCK), 0, s, (const float *)gamma,
                           rows, N, path);
}

// one block per sequence; sequences with a non-zero status get path -1
__global__ __launch_bounds__(BLOCK) void k_mask_paths(const int64_t *__restrict__ offsets,
                                                      const int32_t *__restrict__ status,
                                                      int32_t *__restrict__ path) {
    const int64_t b = blockIdx.x;
    if (status[b] == 0) return;
    const int64_t o0 = offsets[b], o1 = offsets[b + 1];
    for (int64_t r = o0 + threadIdx.x; r < o1; r += BLOCK) path[r] = -1;
}

void launch_mask_paths(const int64_t *offsets, const int32_t *status, int64_t nseq, int32_t *path,
                       hipStream_t s) {
    if (nseq <= 0) return;
    hipLaunchKernelGGL(k_mask_paths, dim3((unsigned)nseq), dim3(BLOCK), 0, s, offsets, status, path);
}

}  // namespace hmmk
