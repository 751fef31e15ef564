// k_grp.hip -- the scaled bf16/fp16 sweeps of the large-state path, several
// sequences per workgroup on the matrix cores.
//
// The scaled alternative to log-space (section 3.2) multiplies normalised
// vectors by A in a narrow format with FP32 accumulation and rescales by
// powers of two.  One vector per sequence fills only one row of a 16-row
// MFMA operand, so a workgroup steps several sequences together (GSZ: 4 for
// N > 128, 8 for N <= 128, 16 for N <= 64) and takes the transposed product
//     D[c][s] = sum_k Mop[c][k] x_s[k]     (v_mfma_f32_16x16x32_{bf16,f16})
// with the matrix as operand A (Mop[c][k] = a_kc forward, a_ck backward, in
// registers) and the input vectors as operand B (from LDS; the columns of
// unused slots are zero).  Operand
// layout (lane l): A row l % 16, k = 8 (l / 16) + q; B column l % 16, same k;
// result column l % 16, rows 4 (l / 16) + i.  So lane l of compute wave w owns
// sequence slot l % 16 and, in each of its TPW tiles of 16 output states, the
// four consecutive states 16 (w + 4 tw) + 4 (l / 16) + i; a sequence's
// maximum or sum needs two permlane swaps inside the wave plus one LDS
// exchange across the four compute waves.
//
// The workgroup is split by role, four compute waves (0-3) and four load
// waves (4-7), each load wave serving a quarter of the group.  The two roles
// run separate loops with the same number of barriers per step (the hardware
// barrier counts waves, not code sites), so neither role's registers are held
// while the other role's code runs.  A load wave keeps a register ring of the
// rows a step reads filled several steps ahead and stages each step's rows
// into double-buffered LDS one step ahead of use.  Rows go to HBM as whole
// 1 KiB rows per instruction (sixteen 64-byte pieces per instruction, straight
// from the matrix-core layout, cost several times more):
//   forward: the compute waves stage alpha^_t in LDS, the load waves store it;
//   backward: the compute waves only propagate b and stage it in LDS, the
//   load waves form gamma_t and w'_t from it and the rows they hold (the row
//   sums Z_t need no exchange across waves there) and stage them in LDS, and
//   the compute waves, which issue no global loads, store them.
//
// bf16 keeps FP32's exponent range: a step's output is scaled by the
// exponent of the largest entry of the step's input, folded into the
// emission factors before the product, one barrier per step.  fp16 has a
// 5-bit exponent, so each vector is normalised exactly (largest entry in
// [1/2, 1)) before it is rounded, at the cost of a second barrier per step.
//
// The sequences of a group are consecutive in the batch and step in
// lockstep for the group's longest length, in whole passes of a few steps; a
// shorter member keeps computing on clamped rows (finite values in its own
// column only) and stores nothing after its end (forward) or before its
// start (backward, which runs each sequence from its own last step).
#include "dev_common.hpp"

namespace hmmk {

typedef __bf16 gbf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 ghalf8_t __attribute__((ext_vector_type(8)));
typedef __bf16 gbf16x4_t __attribute__((ext_vector_type(4)));
typedef _Float16 ghalf4_t __attribute__((ext_vector_type(4)));
typedef float gfloatx4_t __attribute__((ext_vector_type(4)));
typedef float gfloatx8_t __attribute__((ext_vector_type(8)));

template <typename T16>
struct GMfma;
template <>
struct GMfma<__bf16> {
    using V8 = gbf16x8_t;
    using V4 = gbf16x4_t;
    static constexpr bool EXACT = false;
    static __device__ __forceinline__ gfloatx4_t mma(V8 a, V8 b, gfloatx4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct GMfma<_Float16> {
    using V8 = ghalf8_t;
    using V4 = ghalf4_t;
    static constexpr bool EXACT = true;
    static __device__ __forceinline__ gfloatx4_t mma(V8 a, V8 b, gfloatx4_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};

constexpr int GS = 16;   // sequence slots of the matrix-core operand

template <int NCT>
struct GCfg {
    static constexpr int NT = 512;         // four compute waves, then four load waves
    static constexpr int TPW = NCT / 64;   // tiles of 16 output states per compute wave
    static constexpr int KCH = NCT / 32;   // k-chunks of the 16x16x32 instruction
    static constexpr int XP = NCT + 8;     // LDS row pitch of an input vector (T16)
    static constexpr int EP = NCT + 4;     // LDS row pitch of a staged FP32 row
    static constexpr int CPR = NCT / 4;    // 16-byte chunks of a row
    // Rows (sequences) per load wave, one chunk per lane, and sequences per
    // workgroup: 4 for N > 128, so that the rows a step moves are spread over
    // a quarter as many sequences per compute unit (one compute unit's loads
    // in flight cannot cover sixteen sequences' rows per step); the unused
    // operand columns cost nothing, the product's issue time being the same.
    static constexpr int RPH = CPR >= 64 ? 1 : 64 / CPR;
    static constexpr int GSZ = 4 * RPH;
    static constexpr int HK = 1;           // chunks per load-wave lane, table and step
    static constexpr int D = 4;            // steps between a load's issue and its staging
};

__device__ __forceinline__ uint32_t ghi(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t gumax(uint32_t a, uint32_t b) { return a > b ? a : b; }
// exponent of the largest of four non-negative floats given as bit patterns
__device__ __forceinline__ int gexp4(const uint32_t *g) {
    return fexp(__builtin_bit_cast(float, gumax(gumax(g[0], g[1]), gumax(g[2], g[3]))));
}
// maximum over the four lanes of one sequence slot (l, l^16, l^32, l^48)
__device__ __forceinline__ uint32_t slot_umax(uint32_t u) {
    auto r16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    u = gumax((uint32_t)r16[0], (uint32_t)r16[1]);
    auto r32 = __builtin_amdgcn_permlane32_swap(u, u, false, false);
    return gumax((uint32_t)r32[0], (uint32_t)r32[1]);
}
__device__ __forceinline__ float slot_sum(float x) {
    const uint32_t u = __builtin_bit_cast(uint32_t, x);
    auto r16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
    x = __builtin_bit_cast(float, (uint32_t)r16[0]) + __builtin_bit_cast(float, (uint32_t)r16[1]);
    const uint32_t v = __builtin_bit_cast(uint32_t, x);
    auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return __builtin_bit_cast(float, (uint32_t)r32[0]) + __builtin_bit_cast(float, (uint32_t)r32[1]);
}
__device__ __forceinline__ double slot_sum(double x) {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    auto l16 = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
    auto h16 = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
    x = __builtin_bit_cast(double, ((uint64_t)(uint32_t)h16[0] << 32) | (uint32_t)l16[0]) +
        __builtin_bit_cast(double, ((uint64_t)(uint32_t)h16[1] << 32) | (uint32_t)l16[1]);
    const uint64_t v = __builtin_bit_cast(uint64_t, x);
    auto l32 = __builtin_amdgcn_permlane32_swap((uint32_t)v, (uint32_t)v, false, false);
    auto h32 = __builtin_amdgcn_permlane32_swap((uint32_t)(v >> 32), (uint32_t)(v >> 32), false, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)h32[0] << 32) | (uint32_t)l32[0]) +
           __builtin_bit_cast(double, ((uint64_t)(uint32_t)h32[1] << 32) | (uint32_t)l32[1]);
}

// sum over aligned groups of LPR (16, 32 or 64) lanes, in every lane of the
// group: DPP rotations inside each row of 16 lanes, then the permlane swaps
template <int LPR>
__device__ __forceinline__ float group_sum(float v) {
    static_assert(LPR == 16 || LPR == 32 || LPR == 64, "groups of 16, 32 or 64 lanes");
#define HMM_ROR(n)                                                                                   \
    v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),        \
                                                               0x120 + (n), 0xf, 0xf, false))
    HMM_ROR(8);
    HMM_ROR(4);
    HMM_ROR(2);
    HMM_ROR(1);
#undef HMM_ROR
    if constexpr (LPR >= 32) {
        const uint32_t u = __builtin_bit_cast(uint32_t, v);
        auto r = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        v = __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
    }
    if constexpr (LPR == 64) {
        const uint32_t u = __builtin_bit_cast(uint32_t, v);
        auto r = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        v = __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
    }
    return v;
}

// four consecutive FP32 entries of row `row` from column c.  Columns at or
// past N read a copy of an entry inside the row instead (no branch around the
// load, so the load waves' waits stay exact); the sweeps multiply every such
// column by a zero row of the matrix operand or a zero beta entry.
template <bool VEC>
__device__ __forceinline__ float4 gload4(const float *__restrict__ base, int64_t row, int c, int N) {
    if constexpr (VEC) {   // N % 4 == 0: wholly inside or outside the row
        return *reinterpret_cast<const float4 *>(base + row * N + min(c, N - 4));
    } else {
        const float *p = base + row * N;
        return make_float4(p[min(c, N - 1)], p[min(c + 1, N - 1)], p[min(c + 2, N - 1)],
                           p[min(c + 3, N - 1)]);
    }
}

// A load wave's store of one staged 16-byte chunk (columns at or past N are
// not written).
template <bool VEC>
__device__ __forceinline__ void hstore4(float *__restrict__ base, int64_t row, int c, int N, float4 v) {
    if constexpr (VEC) {
        if (c < N) *reinterpret_cast<float4 *>(base + row * N + c) = v;
    } else {
        const float a[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (c + i < N) base[row * N + c + i] = a[i];
    }
}

__device__ __forceinline__ float f4at(const float4 &v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
__device__ __forceinline__ float4 lds4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

// the compute wave's operand-A registers: Mop[c][k] for c = 16 (w + 4 tw) +
// l % 16, k = 32 kc + 8 (l / 16) + q, read from M[c][k] (M = A^T forward,
// A backward), zero outside N x N
template <typename T16, int NCT>
__device__ __forceinline__ void gload_aop(const float *M, int N, int w, int l,
                                          typename GMfma<T16>::V8 (&aop)[GCfg<NCT>::TPW][GCfg<NCT>::KCH]) {
    using C = GCfg<NCT>;
#pragma unroll
    for (int tw = 0; tw < C::TPW; ++tw) {
        const int c = 16 * (w + 4 * tw) + (l & 15);
#pragma unroll
        for (int kc = 0; kc < C::KCH; ++kc) {
            gfloatx8_t f;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int k = 32 * kc + 8 * (l >> 4) + q;
                const float v = M[min(c, N - 1) * N + min(k, N - 1)];
                f[q] = (c < N && k < N) ? v : 0.0f;
            }
            // converted here, as packed pairs (kept from sinking the conversion
            // to the loop, which would hold every entry as FP32 until then)
            aop[tw][kc] = __builtin_convertvector(f, typename GMfma<T16>::V8);
            asm volatile("" : "+v"(aop[tw][kc]));
        }
        // one tile's loads in flight at a time (all of them at once would
        // need a register per entry)
        __builtin_amdgcn_sched_barrier(0);
    }
}

// D = Mop x for the wave's tiles, x = the sixteen operand columns in xs
template <typename T16, int NCT>
__device__ __forceinline__ void gproduct(const T16 *xs, int l,
                                         const typename GMfma<T16>::V8 (&aop)[GCfg<NCT>::TPW][GCfg<NCT>::KCH],
                                         float (&out)[GCfg<NCT>::TPW][4]) {
    using C = GCfg<NCT>;
    using V8 = typename GMfma<T16>::V8;
    gfloatx4_t acc[C::TPW];
#pragma unroll
    for (int tw = 0; tw < C::TPW; ++tw) acc[tw] = gfloatx4_t{0.f, 0.f, 0.f, 0.f};
    const T16 *row = xs + (l & 15) * C::XP + 8 * (l >> 4);
#pragma unroll
    for (int kc = 0; kc < C::KCH; ++kc) {
        const V8 b = *reinterpret_cast<const V8 *>(row + 32 * kc);
#pragma unroll
        for (int tw = 0; tw < C::TPW; ++tw) acc[tw] = GMfma<T16>::mma(aop[tw][kc], b, acc[tw]);
    }
#pragma unroll
    for (int tw = 0; tw < C::TPW; ++tw)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[tw][i] = acc[tw][i];
}

// the lane's outputs as T16 into its sequence's LDS row
template <typename T16, int NCT>
__device__ __forceinline__ void gput(T16 *xs, int w, int l, const float (&x)[GCfg<NCT>::TPW][4]) {
    using C = GCfg<NCT>;
    using V4 = typename GMfma<T16>::V4;
    T16 *row = xs + (l & 15) * C::XP + 4 * (l >> 4);
#pragma unroll
    for (int tw = 0; tw < C::TPW; ++tw) {
        V4 v;
#pragma unroll
        for (int i = 0; i < 4; ++i) v[i] = (T16)x[tw][i];
        *reinterpret_cast<V4 *>(row + 16 * (w + 4 * tw)) = v;
    }
}

// A load wave's share of the staging: its lane l < RPH CPR moves, per table
// and step, chunk l % CPR (columns 4 (l % CPR) ..) of the row of sequence slot
// h RPH + l / CPR (h = wave - 4); lanes past RPH CPR (N in (128, 192]) idle.
template <int NCT>
struct LoadShare {
    int64_t off[GCfg<NCT>::HK];
    int T[GCfg<NCT>::HK];
    int lds[GCfg<NCT>::HK];   // offset of the chunk in a staged table
    int col[GCfg<NCT>::HK];
    bool act;
    __device__ void init(const int64_t *offsets, int64_t nseq, int64_t g0, int h, int l) {
        using C = GCfg<NCT>;
        act = l < C::RPH * C::CPR;
        const int r = act ? l / C::CPR : 0;
        col[0] = act ? 4 * (l % C::CPR) : 0;
        const int slot = h * C::RPH + r;
        lds[0] = slot * C::EP + col[0];
        const int64_t s = g0 + slot;
        const bool v = act && s < nseq;
        off[0] = v ? offsets[s] : 0;
        T[0] = v ? (int)(offsets[s + 1] - off[0]) : 0;
    }
};

// zero the staged emission rows of the operand's unused sequence slots, so
// that their columns stay finite (compute waves, before the first barrier)
template <int NCT>
__device__ __forceinline__ void zero_unused_rows(float (&es)[2][GS * GCfg<NCT>::EP], int tid) {
    using C = GCfg<NCT>;
    constexpr int n = (GS - C::GSZ) * C::EP;
    for (int i = tid; i < 2 * n; i += 256) es[i / n][C::GSZ * C::EP + i % n] = 0.f;
}

// ---------------------------------------------------------------- forward
template <typename T16, int NCT, bool VEC>
__global__ __launch_bounds__(512) void k_grp_fwd(StagedModel<float> m, const int64_t *__restrict__ offsets,
                                                 int64_t nseq, const float *__restrict__ etab,
                                                 const double *__restrict__ mt,
                                                 float *__restrict__ alpha, int32_t *__restrict__ aexp,
                                                 double *__restrict__ loglik,
                                                 int32_t *__restrict__ status) {
    using C = GCfg<NCT>;
    using G = GMfma<T16>;
    constexpr int TPW = C::TPW, HK = C::HK, D = C::D, EP = C::EP;
    __shared__ __align__(16) float es[2][GS * EP];    // e_t, staged by the load waves
    __shared__ __align__(16) float ast[2][GS * EP];   // alpha^_t, staged for the load waves' stores
    __shared__ __align__(16) T16 xs[2][GS * C::XP];
    __shared__ int axs[2][GS];
    __shared__ uint32_t gm[2][GS][4];
    __shared__ uint32_t gE[GS][4];
    __shared__ float zz[GS][4];
    __shared__ double ls[GS][4];
    const int N = m.N, tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t g0 = (int64_t)blockIdx.x * C::GSZ;
    const int sl = l & 15, ig = l >> 4;
    const int64_t sidx = g0 + sl;
    const bool sv = sl < C::GSZ && sidx < nseq;
    const int64_t off = sv ? offsets[sidx] : 0;
    const int T = sv ? (int)(offsets[sidx + 1] - off) : 0;
    const int Tg = __builtin_amdgcn_readfirstlane(wave_max_i(T));   // the group's longest
    // steps 1 .. tl run in whole passes of D (steps past Tg are masked like
    // any step past a member's end)
    const int tl = Tg > 1 ? D * ((Tg - 1 + D - 1) / D) : 0;
    auto col0 = [&](int tw) { return 16 * (w + 4 * tw) + 4 * ig; };

    if (w < 4) {
        // ------------------------------------------------ compute waves
        typename G::V8 aop[TPW][C::KCH];
        gload_aop<T16, NCT>(m.AT, N, w, l, aop);
        zero_unused_rows<NCT>(es, tid);
        float x[TPW][4];
        auto stage = [&](int b, int ex) {
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw)
                *reinterpret_cast<float4 *>(&ast[b][sl * EP + col0(tw)]) =
                    make_float4(x[tw][0], x[tw][1], x[tw][2], x[tw][3]);
            if (w == 0 && ig == 0) axs[b][sl] = ex;
        };
        __syncthreads();   // e_0, e_1 staged
        // t = 0: pi o e_0, normalised exactly
        {
            uint32_t mx = 0;
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw) {
                const float4 e = lds4(&es[0][sl * EP + col0(tw)]);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int c = col0(tw) + i;
                    x[tw][i] = (T > 0 && c < N) ? m.pi[min(c, N - 1)] * f4at(e, i) : 0.f;
                    mx = gumax(mx, ghi(x[tw][i]));
                }
            }
            mx = slot_umax(mx);
            if (ig == 0) gE[sl][w] = mx;
        }
        __syncthreads();
        const int ex0 = gexp4(gE[sl]);
        int64_t E = ex0;
        {
            uint32_t mx = 0;
            float zl = 0.f;
#pragma unroll
            for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    x[tw][i] = fldexp(x[tw][i], -ex0);
                    mx = gumax(mx, ghi(x[tw][i]));
                    zl += x[tw][i];
                }
            stage(0, ex0);
            mx = slot_umax(mx);
            zl = slot_sum(zl);
            if (ig == 0) {
                gm[0][sl][w] = mx;
                if (T == 1) zz[sl][w] = zl;
            }
            gput<T16, NCT>(xs[0], w, l, x);
        }
        __syncthreads();
        for (int t0 = 1; t0 < tl; t0 += D) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int t = t0 + u;
                const int pb = (t - 1) & 1, cb = t & 1;
                float ev[TPW][4];
                int exs = 0;
                if constexpr (!G::EXACT) {
                    // the step's scale 2^-x (x = exponent of the input's largest
                    // entry, at least -126 so that the factor stays finite) goes
                    // into the emission factors while the products run
                    exs = max(gexp4(gm[pb][sl]), -126);
                    const float sc = fldexp(1.0f, -exs);
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw) {
                        const float4 e = lds4(&es[cb][sl * EP + col0(tw)]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) ev[tw][i] = f4at(e, i) * sc;
                    }
                } else {
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw) {
                        const float4 e = lds4(&es[cb][sl * EP + col0(tw)]);
#pragma unroll
                        for (int i = 0; i < 4; ++i) ev[tw][i] = f4at(e, i);
                    }
                }
                gproduct<T16, NCT>(xs[pb], l, aop, x);
#pragma unroll
                for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                    for (int i = 0; i < 4; ++i) x[tw][i] *= ev[tw][i];
                if constexpr (G::EXACT) {
                    uint32_t mx = 0;
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                        for (int i = 0; i < 4; ++i) mx = gumax(mx, ghi(x[tw][i]));
                    mx = slot_umax(mx);
                    if (ig == 0) gE[sl][w] = mx;
                    __syncthreads();
                    exs = gexp4(gE[sl]);
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                        for (int i = 0; i < 4; ++i) x[tw][i] = fldexp(x[tw][i], -exs);
                }
                E += t < T ? exs : 0;
                stage(cb, exs);
                if constexpr (!G::EXACT) {
                    uint32_t mx = 0;
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                        for (int i = 0; i < 4; ++i) mx = gumax(mx, ghi(x[tw][i]));
                    mx = slot_umax(mx);
                    if (ig == 0) gm[cb][sl][w] = mx;
                }
                if (t == T - 1) {   // the member's last step: sum_j alpha^_{T-1}(j)
                    float zl = 0.f;
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                        for (int i = 0; i < 4; ++i) zl += x[tw][i];
                    zl = slot_sum(zl);
                    if (ig == 0) zz[sl][w] = zl;
                }
                gput<T16, NCT>(xs[cb], w, l, x);
                __syncthreads();
            }
        }
        // log P(y) = sum of the per-step log shifts + E log 2 + log sum_j alpha^_{T-1}(j)
        double lsum = 0.0;
        for (int t = 4 * w + ig; t < T; t += 16) lsum += mt[off + t];
        lsum = slot_sum(lsum);
        if (ig == 0) ls[sl][w] = lsum;
        __syncthreads();
        if (w == 0 && ig == 0 && sv) {
            const double logS = (ls[sl][0] + ls[sl][1]) + (ls[sl][2] + ls[sl][3]);
            const float z = (zz[sl][0] + zz[sl][1]) + (zz[sl][2] + zz[sl][3]);
            double ll;
            int st;
            if (*m.perr) {
                ll = __builtin_nan("");
                st = 4;
            } else if (isnan(logS)) {
                ll = __builtin_nan("");
                st = 2;
            } else if (!(z > 0.0f) || isinf(logS)) {
                ll = -__builtin_inf();
                st = 1;
            } else {
                ll = logS + (double)E * 0.69314718055994530942 + log((double)z);
                st = 0;
            }
            loglik[sidx] = ll;
            status[sidx] = st;
        }
    } else {
        // ------------------------------------------------ load waves
        const int h = w - 4;
        LoadShare<NCT> sh;
        sh.init(offsets, nseq, g0, h, l);
        // lane l < RPH also stores the exponents of sequence slot h RPH + l
        const int64_t sx = g0 + h * C::RPH + (l % C::RPH);
        const int64_t offx = sx < nseq ? offsets[sx] : 0;
        const int Tx = sx < nseq ? (int)(offsets[sx + 1] - offx) : 0;
        auto row = [&](int k, int s) { return sh.off[k] + (sh.T[k] > 0 ? min(s, sh.T[k] - 1) : 0); };
        // alpha^_s and its exponent from the staging buffer to HBM (whole rows)
        auto store_step = [&](int s) {
#pragma unroll
            for (int k = 0; k < HK; ++k)
                if (s < sh.T[k])
                    hstore4<VEC>(alpha, sh.off[k] + s, sh.col[k], N, lds4(&ast[s & 1][sh.lds[k]]));
            if (l < C::RPH && s < Tx) aexp[offx + s] = axs[s & 1][h * C::RPH + l];
        };
        float4 ring[D][HK];
#pragma unroll
        for (int k = 0; k < HK; ++k) {
            const float4 e0 = gload4<VEC>(etab, row(k, 0), sh.col[k], N);
            const float4 e1 = gload4<VEC>(etab, row(k, 1), sh.col[k], N);
            if (sh.act) {
                *reinterpret_cast<float4 *>(&es[0][sh.lds[k]]) = e0;
                *reinterpret_cast<float4 *>(&es[1][sh.lds[k]]) = e1;
            }
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int k = 0; k < HK; ++k) ring[j][k] = gload4<VEC>(etab, row(k, 2 + j), sh.col[k], N);
            __builtin_amdgcn_sched_barrier(0);
        }
        // nothing in flight on entry to the loop, so that the compiler's
        // count of loads outstanding at the top of a pass is the steady one
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();   // e_0, e_1 staged
        __syncthreads();   // step 0, first half
        __syncthreads();   // step 0
        for (int t0 = 1; t0 < tl; t0 += D) {
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int t = t0 + u;
                // e_{t+1} (ring slot u) goes to the buffer step t + 1 reads;
                // the slot is refilled with e_{t+1+D}; then step t - 1 is stored
#pragma unroll
                for (int k = 0; k < HK; ++k)
                    if (sh.act) *reinterpret_cast<float4 *>(&es[(t + 1) & 1][sh.lds[k]]) = ring[u][k];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int k = 0; k < HK; ++k) ring[u][k] = gload4<VEC>(etab, row(k, t + 1 + D), sh.col[k], N);
                __builtin_amdgcn_sched_barrier(0);
                store_step(t - 1);
                if constexpr (G::EXACT) __syncthreads();
                __syncthreads();
            }
        }
        store_step(tl);    // staged before the last barrier
        __syncthreads();   // the log-likelihood exchange
    }
}

// ---------------------------------------------------------------- backward
// Step tau of the sweep is step t = T - 1 - tau of a member.  The compute
// waves only propagate: w_t = e_t o b_t (normalised exactly for fp16) is the
// product input, b_{t-1} = A w_t (times 2^-x with x the exponent of the
// input's largest entry, bf16), and each b_t is staged in LDS.  The load
// waves form the outputs from the staged b_t and the rows they loaded:
// Z_t = sum_j alpha^_t(j) b_t(j) (one row per wave or lane group, so no
// exchange across waves), gamma_t = alpha^_t o b_t / Z_t and
// w'_t = e_t o b_t 2^{-x_t} / Z_t (written over e_t; zero on each sequence's
// first step), one step behind the compute waves.
template <int NCT>
struct BwdCfg {
    static constexpr int R = 5;            // register ring: steps tau - 1 .. tau + R - 2
    static constexpr int LPR = NCT / 4;    // lanes of a load wave that share a row
};

template <typename T16, int NCT, bool VEC>
__global__ __launch_bounds__(512) void k_grp_bwd(StagedModel<float> m, const int64_t *__restrict__ offsets,
                                                 int64_t nseq, float *__restrict__ etab,
                                                 const float *__restrict__ alpha,
                                                 const int32_t *__restrict__ aexp,
                                                 const int32_t *__restrict__ status,
                                                 float *__restrict__ gamma) {
    using C = GCfg<NCT>;
    using G = GMfma<T16>;
    constexpr int TPW = C::TPW, HK = C::HK, EP = C::EP, R = BwdCfg<NCT>::R, LPR = BwdCfg<NCT>::LPR;
    static_assert(64 % LPR == 0, "a row's chunks lie in one aligned lane group");
    __shared__ __align__(16) float es[2][GS * EP];    // e_t, staged by the load waves
    __shared__ __align__(16) float bst[2][GS * EP];   // b_t, staged by the compute waves
    __shared__ __align__(16) float gst[2][GS * EP];   // gamma_t, staged by the load waves
    __shared__ __align__(16) float wst[2][GS * EP];   // w'_t
    __shared__ __align__(16) T16 xs[2][GS * C::XP];
    __shared__ uint32_t gm[2][GS][4];
    const int N = m.N, tid = threadIdx.x, l = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t g0 = (int64_t)blockIdx.x * C::GSZ;
    int Tl = 0;
    {
        const int64_t s = g0 + (l & 15);
        if ((l & 15) < C::GSZ && s < nseq) Tl = (int)(offsets[s + 1] - offsets[s]);
    }
    const int Tg = __builtin_amdgcn_readfirstlane(wave_max_i(Tl));
    const int taul = R * ((Tg + R - 1) / R) - 1;   // last step of the whole passes

    if (w < 4) {
        // ------------------------------------------------ compute waves
        const int sl = l & 15, ig = l >> 4;
        auto col0 = [&](int tw) { return 16 * (w + 4 * tw) + 4 * ig; };
        typename G::V8 aop[TPW][C::KCH];
        gload_aop<T16, NCT>(m.A, N, w, l, aop);
        zero_unused_rows<NCT>(es, tid);
        // gamma and w' of sweep step s for the wave's four sequences, from LDS
        // to HBM in whole rows
        LoadShare<NCT> cp;
        cp.init(offsets, nseq, g0, w, l);
        // (the LDS reads are issued first and the stores after the step's
        // products, so that the reads' latency is hidden)
        float4 cpg[HK], cpw[HK];
        auto copy_read = [&](int s) {
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                cpg[k] = lds4(&gst[s & 1][cp.lds[k]]);
                cpw[k] = lds4(&wst[s & 1][cp.lds[k]]);
            }
        };
        auto copy_write = [&](int s) {
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                const int t = cp.T[k] - 1 - s;
                if (t >= 0) {
                    hstore4<VEC>(gamma, cp.off[k] + t, cp.col[k], N, cpg[k]);
                    hstore4<VEC>(etab, cp.off[k] + t, cp.col[k], N, cpw[k]);
                }
            }
        };
        float bt[TPW][4];
#pragma unroll
        for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
            for (int i = 0; i < 4; ++i) bt[tw][i] = (Tl > 0 && col0(tw) + i < N) ? 1.0f : 0.0f;
        __syncthreads();   // e of step 0 staged
        for (int u0 = 0; u0 <= taul; u0 += R) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int tau = u0 + u, cb = tau & 1;
                if (tau >= 2) copy_read(tau - 2);   // staged two barriers ago
                float wv[TPW][4];
                uint32_t mx = 0;
#pragma unroll
                for (int tw = 0; tw < TPW; ++tw) {
                    const float4 e = lds4(&es[cb][sl * EP + col0(tw)]);
                    *reinterpret_cast<float4 *>(&bst[cb][sl * EP + col0(tw)]) =
                        make_float4(bt[tw][0], bt[tw][1], bt[tw][2], bt[tw][3]);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        wv[tw][i] = f4at(e, i) * bt[tw][i];
                        mx = gumax(mx, ghi(wv[tw][i]));
                    }
                }
                mx = slot_umax(mx);
                if (ig == 0) gm[cb][sl][w] = mx;
                if constexpr (G::EXACT) {
                    // fp16: the input is normalised exactly before it is rounded
                    __syncthreads();
                    const int exw = gexp4(gm[cb][sl]);
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                        for (int i = 0; i < 4; ++i) wv[tw][i] = fldexp(wv[tw][i], -exw);
                }
                gput<T16, NCT>(xs[cb], w, l, wv);
                __syncthreads();
                gproduct<T16, NCT>(xs[cb], l, aop, bt);
                if (tau >= 2) copy_write(tau - 2);
                if constexpr (!G::EXACT) {
                    // bf16: scaled by the exponent of the input's largest entry
                    // (the fp16 input was normalised, so its product already is)
                    const float sc = fldexp(1.0f, -max(gexp4(gm[cb][sl]), -126));
#pragma unroll
                    for (int tw = 0; tw < TPW; ++tw)
#pragma unroll
                        for (int i = 0; i < 4; ++i) bt[tw][i] *= sc;
                }
            }
        }
        copy_read(taul - 1);
        copy_write(taul - 1);
        __syncthreads();   // the last step's outputs staged
        copy_read(taul);
        copy_write(taul);
    } else {
        // ------------------------------------------------ load waves
        const int h = w - 4;
        LoadShare<NCT> sh;
        sh.init(offsets, nseq, g0, h, l);
        bool use[HK];
#pragma unroll
        for (int k = 0; k < HK; ++k) {
            const int64_t s = g0 + (sh.lds[k] / EP);
            use[k] = sh.T[k] > 0 && status[s] == 0;
        }
        auto row = [&](int k, int s) { return sh.off[k] + (sh.T[k] > 0 ? max(sh.T[k] - 1 - s, 0) : 0); };
        float4 ra[R][HK], re[R][HK];
        int rx[R][HK];
        auto fill = [&](int slot, int s) {
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                ra[slot][k] = gload4<VEC>(alpha, row(k, s), sh.col[k], N);
                re[slot][k] = gload4<VEC>(etab, row(k, s), sh.col[k], N);
                rx[slot][k] = aexp[row(k, s)];
            }
        };
        // gamma and w' of sweep step s from ring slot `slot` and the staged b
        auto outputs = [&](int slot, int s) {
            float p[HK];
            float4 b[HK];
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                b[k] = lds4(&bst[s & 1][sh.lds[k]]);
                p[k] = 0.f;
#pragma unroll
                for (int i = 0; i < 4; ++i) p[k] += f4at(ra[slot][k], i) * f4at(b[k], i);
            }
            // Z per row: a sum over the row's lane group
#pragma unroll
            for (int k = 0; k < HK; ++k) p[k] = group_sum<LPR>(p[k]);
#pragma unroll
            for (int k = 0; k < HK; ++k) {
                const float rz = __builtin_amdgcn_rcpf(p[k]);
                const int t = sh.T[k] - 1 - s;
                const float gz = use[k] ? rz : 0.f;
                const float wz = (use[k] && t > 0) ? fldexp(rz, -rx[slot][k]) : 0.f;
                if (sh.act) {
                    float4 g, wp;
                    g.x = f4at(ra[slot][k], 0) * f4at(b[k], 0) * gz;
                    g.y = f4at(ra[slot][k], 1) * f4at(b[k], 1) * gz;
                    g.z = f4at(ra[slot][k], 2) * f4at(b[k], 2) * gz;
                    g.w = f4at(ra[slot][k], 3) * f4at(b[k], 3) * gz;
                    wp.x = f4at(re[slot][k], 0) * f4at(b[k], 0) * wz;
                    wp.y = f4at(re[slot][k], 1) * f4at(b[k], 1) * wz;
                    wp.z = f4at(re[slot][k], 2) * f4at(b[k], 2) * wz;
                    wp.w = f4at(re[slot][k], 3) * f4at(b[k], 3) * wz;
                    *reinterpret_cast<float4 *>(&gst[s & 1][sh.lds[k]]) = g;
                    *reinterpret_cast<float4 *>(&wst[s & 1][sh.lds[k]]) = wp;
                }
            }
        };
#pragma unroll
        for (int s = 0; s < R - 1; ++s) {
            __builtin_amdgcn_sched_barrier(0);
            fill(s, s);
            __builtin_amdgcn_sched_barrier(0);
        }
        // nothing in flight on entry to the loop, so that the compiler's count
        // of loads outstanding at the top of a pass is the steady one
        __builtin_amdgcn_s_waitcnt(0);
#pragma unroll
        for (int k = 0; k < HK; ++k)
            if (sh.act) *reinterpret_cast<float4 *>(&es[0][sh.lds[k]]) = re[0][k];
        __syncthreads();   // e of step 0 staged
        for (int u0 = 0; u0 <= taul; u0 += R) {
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const int tau = u0 + u;
                // e of step tau + 1 goes to the buffer that step reads; the
                // outputs of step tau - 1 are formed and stored; that slot is
                // refilled with step tau - 1 + R
                const int sn = (u + 1) % R, sp = (u + R - 1) % R;
#pragma unroll
                for (int k = 0; k < HK; ++k)
                    if (sh.act) *reinterpret_cast<float4 *>(&es[(tau + 1) & 1][sh.lds[k]]) = re[sn][k];
                if (tau >= 1) outputs(sp, tau - 1);
                __builtin_amdgcn_sched_barrier(0);
                fill(sp, tau - 1 + R);
                __builtin_amdgcn_sched_barrier(0);
                if constexpr (G::EXACT) __syncthreads();
                __syncthreads();
            }
        }
        outputs(R - 1, taul);   // taul = R n - 1; b staged before the last barrier
        __syncthreads();        // the last step's outputs staged
    }
}

template <typename T16, int NCT>
static void launch_grp_t(bool fwd, const StagedModel<float> &m, const int64_t *offsets,
                         int64_t nseq, float *etab, const double *mt, float *alpha,
                         int32_t *aexp, double *loglik, int32_t *status, float *gamma,
                         hipStream_t s) {
    const dim3 grid((unsigned)((nseq + GCfg<NCT>::GSZ - 1) / GCfg<NCT>::GSZ));
    const dim3 block(GCfg<NCT>::NT);
    const bool vec = m.N % 4 == 0;
    if (fwd) {
        if (vec)
            hipLaunchKernelGGL((k_grp_fwd<T16, NCT, true>), grid, block, 0, s, m, offsets, nseq,
                               (const float *)etab, mt, alpha, aexp, loglik, status);
        else
            hipLaunchKernelGGL((k_grp_fwd<T16, NCT, false>), grid, block, 0, s, m, offsets, nseq,
                               (const float *)etab, mt, alpha, aexp, loglik, status);
        return;
    }
    if constexpr (64 % BwdCfg<NCT>::LPR == 0) {
        if (vec)
            hipLaunchKernelGGL((k_grp_bwd<T16, NCT, true>), grid, block, 0, s, m, offsets, nseq,
                               etab, (const float *)alpha, (const int32_t *)aexp,
                               (const int32_t *)status, gamma);
        else
            hipLaunchKernelGGL((k_grp_bwd<T16, NCT, false>), grid, block, 0, s, m, offsets, nseq,
                               etab, (const float *)alpha, (const int32_t *)aexp,
                               (const int32_t *)status, gamma);
    }
}

template <typename T16>
static void launch_grp_nc(bool fwd, const StagedModel<float> &m, const int64_t *offsets,
                          int64_t nseq, float *etab, const double *mt, float *alpha,
                          int32_t *aexp, double *loglik, int32_t *status, float *gamma,
                          hipStream_t s) {
    const int nc = ((m.N + 63) / 64) * 64;
    switch (nc) {
    case 64:
        return launch_grp_t<T16, 64>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
    case 128:
        return launch_grp_t<T16, 128>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
    case 192:   // the backward kernel needs a row's chunks in one lane group: 256
        if (fwd)
            return launch_grp_t<T16, 192>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
        return launch_grp_t<T16, 256>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
    default:
        return launch_grp_t<T16, 256>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
    }
}

void launch_grp_sweep(bool fwd, bool bf16, const StagedModel<float> &m, const int64_t *offsets,
                      int64_t nseq, float *etab, const double *mt, float *alpha, int32_t *aexp,
                      double *loglik, int32_t *status, float *gamma, hipStream_t s) {
    if (bf16)
        launch_grp_nc<__bf16>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
    else
        launch_grp_nc<_Float16>(fwd, m, offsets, nseq, etab, mt, alpha, aexp, loglik, status, gamma, s);
}

}  // namespace hmmk
