// hmm_internal.hpp -- internal declarations shared by the host runtime
// (abi.cpp) and the kernel translation units: staged-parameter layout,
// kernel argument blocks and launcher prototypes.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "hmm_gpu.h"

namespace hmmk {

constexpr int EP_STRIDE = 8;       // per-state emission-constant slots
constexpr int BLOCK = 256;         // threads per block of every kernel

// Parameters staged on the device once per call (section 3.2 notes that log A
// is prepared once per training iteration; the linear A, pi and the per-state
// emission constants are prepared the same way).  R = float or double.
template <typename R>
struct StagedModel {
    int N, D, family;
    const R *pi;        // [N]      exp(log pi)
    const R *A;         // [N*N]    exp(log A), row i = from state i
    const R *AT;        // [N*N]    its transpose, row j = into state j
    const R *lpi;       // [N]      log pi in R
    const R *lA;        // [N*N]    log A in R
    const R *ep;        // [N*EP_STRIDE] emission constants
    const double *ep64; // the same constants in FP64 (families evaluated in FP64)
    const R *mv;        // multivariate constants: diag [mu(N*D), -1/(2 var)(N*D)],
                        // full [mu(N*D), Linv(N*D*D)] (Linv lower, row-major)
    const int *perr;    // parameter-domain flag written by the staging kernel
    const R *A8;        // [8*8] exp(log A) zero-padded to 8 states (small-N kernels)
    const int *nrm;     // steps between rescalings of forward-type products (1, 2 or 4)
};

// Raw (not yet staged) model, FP64 device pointers from the ABI.
struct RawModel {
    int N, D, family;
    const double *log_pi, *log_A, *theta;
};

struct ObsDesc {
    const void *obs;
    int obs_f64;
    int64_t nseq;
    const int64_t *offsets;   // device [B+1]
};

// Optional per-kernel timing: when enabled with hmm_profile_enable, every
// launcher brackets its kernel with hipEvents recorded on the launch stream.
void prof_begin(const char *name, hipStream_t s);
void prof_end(hipStream_t s);
struct ProfScope {
    hipStream_t s;
    ProfScope(const char *name, hipStream_t st) : s(st) { prof_begin(name, st); }
    ~ProfScope() { prof_end(s); }
};

// byte sizes of the staged region for precision R
size_t staged_bytes(int N, int D, int family, bool f64);

// ----- launchers (each defined in the kernel translation unit) -----
// Chunk counts of the N <= 8 path, formed in the staging launch: cbase and
// sbase, [B+1] exclusive prefix counts of chunks (L steps) and superchunks
// (S chunks)
struct PlanArgs {
    const int64_t *offsets;
    int64_t nseq;
    int L, S;
    int *cbase, *sbase;
};
template <typename R>
void launch_stage(const RawModel &m, void *region, StagedModel<R> *out, hipStream_t s,
                  const PlanArgs *plan = nullptr);

// Per-chunk and per-superchunk descriptors, written once per call so the
// kernels find their sequence with a single load.
struct __align__(16) ChunkDesc {
    int64_t off;    // first observation row of the owning sequence
    int b;          // owning sequence
    int t0;         // first step of the chunk inside the sequence
    int len;        // steps in the chunk (<= L)
    int pad0;
    int64_t pad1;
};
struct __align__(16) SuperDesc {
    int64_t off;    // first observation row of the owning sequence
    int b;          // owning sequence
    int lo;         // first chunk of the superchunk
    int n;          // chunks in the superchunk (<= S)
    int head;       // 1 if it is the sequence's first superchunk
    int t0;         // first step of its first chunk inside the sequence
    int T;          // steps of the owning sequence
};
void launch_chunk_desc(const int64_t *offsets, int64_t nseq, int L, int S, const int *cbase,
                       const int *sbase, int C, int SC, ChunkDesc *cdesc, SuperDesc *sdesc,
                       hipStream_t s);

// cbase[b] = chunks before sequence b (L steps each); sbase[b] = superchunks
// (S chunks each) before sequence b; both [B+1]
void launch_plan_chunks(const int64_t *offsets, int64_t nseq, int L, int S, int *cbase,
                        int *sbase, hipStream_t s);

// batched small-N path (G = 4 or 8 lanes per chunk)
struct ChunkBuffers {
    int L, C, G, nblk_stats;
    int S, SC;           // chunks per superchunk, number of superchunks
    int *cbase;          // [B+1]
    int *sbase;          // [B+1]
    SuperDesc *sdesc;    // [SC] (chunk c = sdesc.lo + i covers steps t0 + i L ...)
    void *srec;          // [SC*G] superchunk transfer-matrix records (one per lane)
    void *Fs;            // [SC*G] R  alpha at each superchunk end
    void *Gs;            // [SC*G] R  beta at each superchunk end
    void *rec;           // [C*G] chunk records (one per lane): column of P_c, row exponent, log shift
    void *F;             // [C*G] R  alpha at each chunk end (normalised)
    void *Gb;            // [C*G] R  beta at each chunk end (normalised)
    double *partial;     // [nblk_stats * S]
    double *red;         // reduction scratch (reduce_scratch_len doubles)
};
// bytes of one chunk (or superchunk) transfer-matrix record
size_t chunk_rec_bytes(bool f64, int G);
template <typename R>
hmm_status run_chunked(const StagedModel<R> &m, const ObsDesc &o, const ChunkBuffers &cb,
                       double *loglik, int32_t *status, void *gamma_out, double *stats,
                       int64_t stats_len, hipStream_t s);

// batched path for 8 < N <= 64: per-sequence sweeps give alpha/beta at the
// ends of chunks of WAVE_L steps, one lane group per chunk forms the statistics
struct WaveBuffers {
    int C, nblk;
    int *cbase;          // [B+1]
    ChunkDesc *cdesc;    // [C]
    void *F;             // [C*NP] R  alpha at each chunk end (normalised)
    void *Gb;            // [C*NP] R  beta at each chunk end (normalised)
    double *partial;     // [nblk * S]
    double *red;         // reduction scratch (reduce_scratch_len doubles)
    // sweep segments (superchunks of seg_chunks chunks; SC == B: none split)
    int SC, vmax;        // segments, chunks a second sweep may run
    const int *sbase;    // [B+1] segments before each sequence
    const SuperDesc *sdesc;   // [SC]
    double *lsc;         // [C]   forward log scale at each chunk end
    double *segJ;        // [SC]  log sum of each segment's forward end vector
    double *seginc;      // [SC]  forward log-likelihood increment
    int32_t *segbad;     // [SC]  invalid emission values
    int32_t *segver;     // [2SC] second sweep agreed (forward, backward)
    int32_t *seglim;     // [2SC] first chunk / last slot still from the first sweep
};
constexpr int WAVE_L = 32;          // chunk length of the wave path
constexpr int WAVE_VMAX = 24;       // chunks a second sweep of a segment may run
int wave_seg_chunks(int variant);   // chunks per sweep segment of a wave-route variant
int wave_np(int N);                 // lanes per group = padded state count (16, 32 or 64)
int wave_stats_blocks(int C, int N);   // blocks (= partial rows) of the statistics kernel
template <typename R>
hmm_status run_wave(const StagedModel<R> &m, const ObsDesc &o, const WaveBuffers &wb,
                    double *loglik, int32_t *status, void *gamma_out, double *stats,
                    int64_t stats_len, hipStream_t s);

// batched path for large N (<= 256) and the multivariate families: one
// workgroup per sequence, emission table, stored alpha, xi by a contraction
// over stored alpha and w' on the matrix cores
constexpr int BLK_TS = 1024;    // steps per tile of the family-sum kernels
constexpr int FULL_TS = 8192;   // steps per tile of the full-covariance family sums
constexpr int BLK_GS_BLOCKS = 1024;   // blocks (partial rows) of the per-state family-sum kernel
struct BlockBuffers {
    int64_t total;       // sum of T
    int mfma = 0;        // sweeps: 0 FP32/FP64 vector ALU, 1 bf16 MFMA, 2 fp16 MFMA
    void *etab;          // [total * N] R  emission factors, then w' (in place)
    double *mt;          // [total]   per-step log shift
    void *alpha;         // [total * N] R  normalised alpha
    int32_t *aexp;       // [total]   binary exponent removed at each forward step
    void *gamma;         // [total * N] R  posteriors (when the caller gives none)
    void *xi;            // [xi_nsl * xi_nc(N)^2] R  per-slice partial sums of the xi contraction
    int xi_nsl;          // slices of the contraction
    double *xisum;       // [N * N] sum_k alpha_k^T w'_{k+1}, row-major
    double *g1;          // [N]
    double *partial;     // [tiles * (1 + N + N*K)]
    double *compact;     // [1 + N + N*K]
    double *red;         // reduction scratch
};
// nominal slice count of the xi contraction
int xi_nc(int N);   // padded state count of the contraction (128 or 256)
int xi_slices(bool f64, int N, int64_t total);
// out [N x N] FP64 = sum_k alpha[k]^T wp[k + 1] over k < K (K >= 1)
template <typename R>
void launch_xi_sum(const R *alpha, const R *wp, int N, int64_t K, R *part, int nsl, double *out,
                   hipStream_t s);
// tiled forward (fwd) or backward sweeps of the large-state path, 64 < N <= 256
template <typename R>
void launch_sw_sweep(bool fwd, const StagedModel<R> &m, const int64_t *offsets, int64_t nseq,
                     R *etab, const double *mt, R *alpha, int32_t *aexp, double *loglik,
                     int32_t *status, R *gamma, hipStream_t s);
// scaled bf16 (bf16 true) or fp16 sweeps of the large-state path, sixteen
// sequences per workgroup on the matrix cores, N <= 256
void launch_grp_sweep(bool fwd, bool bf16, const StagedModel<float> &m, const int64_t *offsets,
                      int64_t nseq, float *etab, const double *mt, float *alpha, int32_t *aexp,
                      double *loglik, int32_t *status, float *gamma, hipStream_t s);
int blk_gstats_tiles(int64_t total, int family);
template <typename R>
hmm_status run_block(const StagedModel<R> &m, const ObsDesc &o, const BlockBuffers &bb,
                     double *loglik, int32_t *status, void *gamma_out, double *stats,
                     int64_t stats_len, hipStream_t s);

// Multivariate families with N <= 64 on the wave path: the log-density table
// [total x N] feeds the table-family sweeps and statistics (which also give
// gamma), then the family sums are formed from gamma.
struct MvBuffers {
    int64_t total;       // sum of T
    void *lt;            // [total * N] R  log b_j(y_t)
    void *gamma;         // [total * N] R  posteriors (when statistics are asked for and the caller gives none)
    double *partial;     // [blk_gstats_tiles * (1 + N + N*K)]
    double *compact;     // [1 + N + N*K]
    double *red;         // reduction scratch
};
template <typename R>
hmm_status run_wave_mv(const StagedModel<R> &m, const ObsDesc &o, const WaveBuffers &wb,
                       const MvBuffers &mb, double *loglik, int32_t *status, void *gamma_out,
                       double *stats, hipStream_t s);

// number of family-statistic slots per state (runtime family)
__host__ __device__ inline int family_k_hd(int family, int D) {
    switch (family) {
    case HMM_GAUSSIAN: return 2;
    case HMM_GAMMA: return 3;
    case HMM_STUDENT_T: return 4;
    case HMM_POISSON: return 1;
    case HMM_DIAG_GAUSSIAN: return 2 * D;
    case HMM_FULL_GAUSSIAN: return D + D * (D + 1) / 2;
    default: return 0;
    }
}

// plain path (one thread per sequence, literal log-sum-exp)
struct PlainBuffers {
    void *logB, *alpha, *beta;   // [sum T * N] R
    double *ps;                  // [B * S] per-sequence statistics
    double *red;                 // reduction scratch (reduce_scratch_len doubles)
};
template <typename R>
hmm_status run_plain(const StagedModel<R> &m, const ObsDesc &o, const PlainBuffers &pb,
                     double *loglik, int32_t *status, void *gamma_out, double *stats,
                     int64_t stats_len, hipStream_t s);

// emission table
template <typename R>
hmm_status run_emission(const StagedModel<R> &m, const ObsDesc &o, int64_t total_steps,
                        R *out, hipStream_t s);

// Viterbi (N <= 64): psi [sum T * N] bytes, J [C * N], qlast [B], qend [C];
// n_ties [B] (or NULL): near-ties met along each returned path.  The forward
// recursion runs in segments of vit_seg_chunks() chunks of 64 steps (SC ==
// B: none split).
struct VitBuffers {
    int SC;                   // segments
    const int *sbase;         // [B+1] segments before each sequence
    const SuperDesc *sdesc;   // [SC]
    void *vd;                 // [C x 64] R  shifted score vector at each chunk end
    double *voff;             // [C]  shift sum at each chunk end
    double *J;                // [SC]
    double *inc;              // [SC]
    int32_t *flag, *ver, *lim;   // [SC] each
};
int vit_seg_chunks();
template <typename R>
hmm_status run_viterbi(const StagedModel<R> &m, const ObsDesc &o, const int *cbase,
                       const ChunkDesc *cdesc, int C, const VitBuffers &vb, uint8_t *psi,
                       uint8_t *J, uint8_t *qlast, uint8_t *qend, int32_t *path, double *logp,
                       int32_t *n_ties, hipStream_t s);

// path[t] = -1 on every step of the sequences whose status is not 0
void launch_mask_paths(const int64_t *offsets, const int32_t *status, int64_t nseq, int32_t *path,
                       hipStream_t s);

// M-steps (section 4), FP64 on the device
void launch_mstep_trans(int N, const double *stats, const double *log_A_in, double eps,
                        double *log_pi_out, double *log_A_out, hipStream_t s);
void launch_mstep_emission(int family, int N, int D, const double *theta_in,
                           const double *stats, const hmm_mstep_opts &o, double *theta_out,
                           int32_t *collapsed, int32_t *iters, hipStream_t s);

// error reporting (message for hmm_last_error of this thread) and model
// validation shared with the serving runtime
hmm_status fail_status(hmm_status st, const char *fmt, ...);
hmm_status model_theta_len(const hmm_model *m, size_t *len);

// fixed-order reduction of per-block partial statistics + log-likelihood sum;
// red is scratch of reduce_scratch_len(nparts, S) doubles
int64_t reduce_scratch_len(int64_t nparts, int64_t S);
void launch_reduce_stats(const double *partial, int nparts, int64_t S, const double *loglik,
                         const int32_t *status, int64_t nseq, double *stats, double *red,
                         hipStream_t s);

}  // namespace hmmk
