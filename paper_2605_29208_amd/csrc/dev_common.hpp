// dev_common.hpp -- device helpers shared by the HIP kernels of the library:
// DPP lane-group primitives, per-state emission constants, scalar emission
// log-densities and the per-state sufficient-statistic terms.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hmm_internal.hpp"

namespace hmmk {

// ---------------------------------------------------------------------------
// DPP control words (CDNA data-parallel-primitive encoding)
// ---------------------------------------------------------------------------
enum : int {
    DPP_QP_X1 = 0xB1,          // quad_perm [1,0,3,2]: lane ^ 1 inside each quad
    DPP_QP_X2 = 0x4E,          // quad_perm [2,3,0,1]: lane ^ 2
    DPP_QP_X3 = 0x1B,          // quad_perm [3,2,1,0]: lane ^ 3
    DPP_HALF_MIRROR = 0x141,   // row_half_mirror: lane p <-> 7 - p inside each 8 lanes
    DPP_ROW_MIRROR = 0x140     // row_mirror: lane p <-> 15 - p inside each row of 16
};

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ float dpp_v(float v) {
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_v(double v) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)dpp_i<CTRL>((int)(uint32_t)u);
    uint32_t hi = (uint32_t)dpp_i<CTRL>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Lane-group of G consecutive lanes (G = 4 or 8); position p = lane % G.
// Source k of position p: k < 4 -> p ^ k; k >= 4 -> 7 - (p ^ (k - 4)).
// For G = 8 the eight sources of every position are the eight lanes of its
// group; for G = 4 the first four are the four lanes of its quad.
__host__ __device__ constexpr int grp_src(int p, int k) {
    return k < 4 ? (p ^ k) : (7 - (p ^ (k - 4)));
}
// inverse: the k with grp_src(p, k) == i
__host__ __device__ constexpr int grp_inv(int p, int i) {
    return ((i ^ p) < 4) ? (i ^ p) : (4 + ((7 - i) ^ p));
}

// x_k = value of x held by source k of this lane
template <int G, typename R>
__device__ __forceinline__ void grp_gather(R x, R (&out)[G]) {
    out[0] = x;
    out[1] = dpp_v<DPP_QP_X1>(x);
    out[2] = dpp_v<DPP_QP_X2>(x);
    out[3] = dpp_v<DPP_QP_X3>(x);
    if constexpr (G == 8) {
        R m = dpp_v<DPP_HALF_MIRROR>(x);
        out[4] = m;
        out[5] = dpp_v<DPP_QP_X1>(m);
        out[6] = dpp_v<DPP_QP_X2>(m);
        out[7] = dpp_v<DPP_QP_X3>(m);
    }
}

// wave-wide all-reductions through DPP row operations and the permlane
// swaps (every lane receives the result, identical in all lanes)
template <typename V, typename Op>
__device__ __forceinline__ V wave_all(V v, Op op) {
    v = op(v, dpp_v<DPP_QP_X1>(v));
    v = op(v, dpp_v<DPP_QP_X2>(v));
    v = op(v, dpp_v<DPP_HALF_MIRROR>(v));
    v = op(v, dpp_v<DPP_ROW_MIRROR>(v));
    if constexpr (sizeof(V) == 4) {
        const uint32_t u = __builtin_bit_cast(uint32_t, v);
        auto r16 = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        v = op(__builtin_bit_cast(V, (uint32_t)r16[0]), __builtin_bit_cast(V, (uint32_t)r16[1]));
        const uint32_t w = __builtin_bit_cast(uint32_t, v);
        auto r32 = __builtin_amdgcn_permlane32_swap(w, w, false, false);
        v = op(__builtin_bit_cast(V, (uint32_t)r32[0]), __builtin_bit_cast(V, (uint32_t)r32[1]));
    } else {
        uint64_t u = __builtin_bit_cast(uint64_t, v);
        auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)u, (uint32_t)u, false, false);
        auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
        v = op(__builtin_bit_cast(V, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]),
               __builtin_bit_cast(V, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]));
        u = __builtin_bit_cast(uint64_t, v);
        auto lo2 = __builtin_amdgcn_permlane32_swap((uint32_t)u, (uint32_t)u, false, false);
        auto hi2 = __builtin_amdgcn_permlane32_swap((uint32_t)(u >> 32), (uint32_t)(u >> 32), false, false);
        v = op(__builtin_bit_cast(V, ((uint64_t)(uint32_t)hi2[0] << 32) | (uint32_t)lo2[0]),
               __builtin_bit_cast(V, ((uint64_t)(uint32_t)hi2[1] << 32) | (uint32_t)lo2[1]));
    }
    return v;
}
template <typename R>
__device__ __forceinline__ R wave_sum_r(R v) {
    return wave_all(v, [](R a, R b) { return a + b; });
}
template <typename R>
__device__ __forceinline__ R wave_max_r(R v) {
    return wave_all(v, [](R a, R b) { return fmax(a, b); });
}

// Orders this wave's LDS accesses around a lane exchange.  LDS instructions
// of one wave are performed in program order, so a wavefront-scope fence
// (which only stops the compiler from moving accesses across it) is enough
// between the lanes' store of a vector and their broadcast reads of it, and
// between those reads and the next store: no wait for completion.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
}

// sum_k x[src_k] * c[k]
template <int G, typename R>
__device__ __forceinline__ R grp_dot(R x, const R (&c)[G]) {
    R s = x * c[0];
    s = fma(dpp_v<DPP_QP_X1>(x), c[1], s);
    s = fma(dpp_v<DPP_QP_X2>(x), c[2], s);
    s = fma(dpp_v<DPP_QP_X3>(x), c[3], s);
    if constexpr (G == 8) {
        R m = dpp_v<DPP_HALF_MIRROR>(x);
        s = fma(m, c[4], s);
        s = fma(dpp_v<DPP_QP_X1>(m), c[5], s);
        s = fma(dpp_v<DPP_QP_X2>(m), c[6], s);
        s = fma(dpp_v<DPP_QP_X3>(m), c[7], s);
    }
    return s;
}

// Transposed counterpart of grp_dot: lane i receives sum_k u_k(src(i, k)),
// where u_k = x * c[k] on every lane.  Each source map src(., k) is an
// involution, so if lane q holds c[k] = M[src(q, k)][q] (its column of M in
// grp_dot order) this is sum_j M[i][j] x_j, the matrix-vector product from
// the same coefficients.  The quad permutations commute with the mirror, so
// the upper four terms share one mirror move.
template <int G, typename R>
__device__ __forceinline__ R grp_tdot(R x, const R (&c)[G]) {
    R s = x * c[0];
    s += dpp_v<DPP_QP_X1>(x * c[1]);
    s += dpp_v<DPP_QP_X2>(x * c[2]);
    s += dpp_v<DPP_QP_X3>(x * c[3]);
    if constexpr (G == 8) {
        R h = x * c[4];
        h += dpp_v<DPP_QP_X1>(x * c[5]);
        h += dpp_v<DPP_QP_X2>(x * c[6]);
        h += dpp_v<DPP_QP_X3>(x * c[7]);
        s += dpp_v<DPP_HALF_MIRROR>(h);
    }
    return s;
}

// U[k] += x[src_k] * w
template <int G, typename R>
__device__ __forceinline__ void grp_outer_acc(R x, R w, R (&U)[G]) {
    U[0] = fma(x, w, U[0]);
    U[1] = fma(dpp_v<DPP_QP_X1>(x), w, U[1]);
    U[2] = fma(dpp_v<DPP_QP_X2>(x), w, U[2]);
    U[3] = fma(dpp_v<DPP_QP_X3>(x), w, U[3]);
    if constexpr (G == 8) {
        R m = dpp_v<DPP_HALF_MIRROR>(x);
        U[4] = fma(m, w, U[4]);
        U[5] = fma(dpp_v<DPP_QP_X1>(m), w, U[5]);
        U[6] = fma(dpp_v<DPP_QP_X2>(m), w, U[6]);
        U[7] = fma(dpp_v<DPP_QP_X3>(m), w, U[7]);
    }
}

template <int G, typename R>
__device__ __forceinline__ R grp_max(R v) {
    v = fmax(v, dpp_v<DPP_QP_X1>(v));
    v = fmax(v, dpp_v<DPP_QP_X2>(v));
    if constexpr (G == 8) v = fmax(v, dpp_v<DPP_HALF_MIRROR>(v));
    return v;
}
template <int G, typename R>
__device__ __forceinline__ R grp_sum(R v) {
    v = v + dpp_v<DPP_QP_X1>(v);
    v = v + dpp_v<DPP_QP_X2>(v);
    if constexpr (G == 8) v = v + dpp_v<DPP_HALF_MIRROR>(v);
    return v;
}
// maximum of non-negative values: for IEEE floats >= 0 the bit patterns order
// like the values, so an unsigned integer maximum needs no NaN canonicalisation
template <int G>
__device__ __forceinline__ float grp_max_pos(float v) {
    unsigned u = __builtin_bit_cast(unsigned, v);
    u = max(u, (unsigned)dpp_i<DPP_QP_X1>((int)u));
    u = max(u, (unsigned)dpp_i<DPP_QP_X2>((int)u));
    if constexpr (G == 8) u = max(u, (unsigned)dpp_i<DPP_HALF_MIRROR>((int)u));
    return __builtin_bit_cast(float, u);
}
template <int G>
__device__ __forceinline__ double grp_max_pos(double v) {
    return grp_max<G, double>(v);
}

template <int G>
__device__ __forceinline__ int grp_max_i(int v) {
    v = max(v, dpp_i<DPP_QP_X1>(v));
    v = max(v, dpp_i<DPP_QP_X2>(v));
    if constexpr (G == 8) v = max(v, dpp_i<DPP_HALF_MIRROR>(v));
    return v;
}

// wave-wide integer maximum (used once per kernel for uniform trip counts)
__device__ __forceinline__ int wave_max_i(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// binary exponent helpers: x = m * 2^e with |m| in [1/2, 1); exponent of 0 is 0
__device__ __forceinline__ int fexp(float x) { return __builtin_amdgcn_frexp_expf(x); }
__device__ __forceinline__ int fexp(double x) { return __builtin_amdgcn_frexp_exp(x); }
__device__ __forceinline__ float fldexp(float x, int e) { return __builtin_amdgcn_ldexpf(x, e); }
__device__ __forceinline__ double fldexp(double x, int e) { return __builtin_amdgcn_ldexp(x, e); }

__device__ __forceinline__ float fexp_e(float x) { return __expf(x); }
__device__ __forceinline__ double fexp_e(double x) { return exp(x); }
__device__ __forceinline__ float flog(float x) { return __logf(x); }
__device__ __forceinline__ double flog(double x) { return log(x); }
// log(1 + x) for x >= 0 in single precision by Goldberg's correction of the
// rounded argument (D. Goldberg, "What every computer scientist should know
// about floating-point arithmetic", 1991, theorem 4): with u = fl(1 + x),
// log1p(x) = log(u) x / (u - 1), exact in the rounding of u; u = 1 gives x.
// A few ulps from the hardware logarithm, against about a hundred
// instructions for the library routine.
__device__ __forceinline__ float flog1p(float x) {
    const float u = 1.0f + x;
    const float d = u - 1.0f;
    return (d == 0.0f || isinf(x)) ? x : __logf(u) * (x * __builtin_amdgcn_rcpf(d));
}
__device__ __forceinline__ double flog1p(double x) { return log1p(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
// v_rcp_f64 and one Newton step (r + r (1 - x r)): within an ulp or two for
// the positive, normal-range sums it is used on, in a third of the
// instructions of an IEEE division
__device__ __forceinline__ double frcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return fma(r, fma(-x, r, 1.0), r);
}

template <typename R> __device__ __forceinline__ R neg_inf() { return -__builtin_inf(); }

// ---------------------------------------------------------------------------
// observations
// ---------------------------------------------------------------------------
struct ObsRef {
    const void *p;
    int f64;
};
template <typename R>
__device__ __forceinline__ R load_obs(const ObsRef &o, int64_t idx) {
    if (o.f64) return (R)((const double *)o.p)[idx];
    return (R)((const float *)o.p)[idx];
}

// ---------------------------------------------------------------------------
// scalar emission families (compile-time family)
//
// Per-state constants ep[8] (filled by the staging kernel from theta):
//   GAUSSIAN   ep0 = mu, ep1 = -1/(2 var), ep2 = -log(2 pi var)/2
//              log b = ep2 + ep1 (y - mu)^2
//   GAMMA      ep0 = a log(rate) - lgamma(a), ep1 = a - 1, ep2 = -rate
//              log b = ep0 + ep1 log y + ep2 y          (y > 0, else -inf)
//   STUDENT_T  ep0 = mu, ep1 = 1/(nu s^2), ep2 = -(nu+1)/2,
//              ep3 = lgamma((nu+1)/2) - lgamma(nu/2) - log(nu pi s^2)/2, ep4 = (nu+1)/nu
//              log b = ep3 + ep2 log1p(ep1 (y - mu)^2);  u = ep4 / (1 + ep1 (y-mu)^2)
//   POISSON    ep0 = log(lambda), ep1 = -lambda
//              log b = y ep0 + ep1 - lgamma(y + 1)      (y a non-negative integer)
//              The state-independent -lgamma(y+1) is returned separately in
//              FP64 ("common") so the single-precision values stay small.
//   TABLE      log b is read from the observation table [sum T, N].
// ---------------------------------------------------------------------------
template <typename R>
struct StateConsts {
    R c0, c1, c2, c3, c4;
};

// State j's constants with no condition on the load (j must be a valid
// state), for callers that mask dead states afterwards (emit_scalar does):
// the loads of many states can then be in flight together.
template <typename R>
__device__ __forceinline__ StateConsts<R> load_consts_row(const R *ep, int j) {
    const R *q = ep + j * EP_STRIDE;
    StateConsts<R> s;
    s.c0 = q[0];
    s.c1 = q[1];
    s.c2 = q[2];
    s.c3 = q[3];
    s.c4 = q[4];
    return s;
}

template <typename R>
__device__ __forceinline__ StateConsts<R> load_consts(const R *ep, int j, bool live) {
    StateConsts<R> s;
    if (live) {
        s.c0 = ep[j * EP_STRIDE + 0];
        s.c1 = ep[j * EP_STRIDE + 1];
        s.c2 = ep[j * EP_STRIDE + 2];
        s.c3 = ep[j * EP_STRIDE + 3];
        s.c4 = ep[j * EP_STRIDE + 4];
    } else {
        s.c0 = s.c1 = s.c2 = s.c3 = s.c4 = (R)0;
    }
    return s;
}

// per-step observation: y (scalar families) and whether it is finite
template <typename R>
struct Emit {
    R ell;          // log b_j(y_t) without the state-independent part
    double common;  // state-independent part (Poisson: -lgamma(y+1)); 0 otherwise
    bool bad;       // non-finite observation
};

template <int FAM, typename R>
__device__ __forceinline__ Emit<R> emit_scalar(R y, const StateConsts<R> &k, bool live) {
    Emit<R> e;
    e.common = 0.0;
    e.bad = !isfinite(y);
    if constexpr (FAM == HMM_GAUSSIAN) {
        R d = y - k.c0;
        e.ell = fma(k.c1, d * d, k.c2);
    } else if constexpr (FAM == HMM_GAMMA) {
        e.ell = (y > (R)0) ? fma(k.c2, y, fma(k.c1, flog(y), k.c0)) : neg_inf<R>();
    } else if constexpr (FAM == HMM_STUDENT_T) {
        R d = y - k.c0;
        e.ell = fma(k.c2, flog1p(k.c1 * d * d), k.c3);
    } else if constexpr (FAM == HMM_POISSON) {
        bool ok = (y >= (R)0) && (floor(y) == y);
        e.ell = ok ? fma(y, k.c0, k.c1) : neg_inf<R>();
        e.common = ok ? -lgamma((double)y + 1.0) : 0.0;
    } else {
        e.ell = y;   // table: the value itself is log b
    }
    if (!live) e.ell = neg_inf<R>();
    return e;
}

// Arithmetic type of the emission evaluation.  Poisson log-densities are of
// the size of y log(lambda) (hundreds for counts near 100), so in the
// single-precision path they are evaluated, shifted by their per-step maximum
// and summed into the log offset in FP64; only the shifted difference is
// rounded to the recursion's type.
template <int FAM, typename R>
struct EmitTraits {
    using T = R;
};
template <typename R>
struct EmitTraits<HMM_POISSON, R> {
    using T = double;
};

template <int FAM, typename R>
__device__ __forceinline__ const typename EmitTraits<FAM, R>::T *consts_ptr(
    const StagedModel<R> &m) {
    if constexpr (FAM == HMM_POISSON) return m.ep64;
    else return m.ep;
}

// number of family-statistic slots per state
template <int FAM>
__host__ __device__ constexpr int fam_k() {
    return FAM == HMM_GAUSSIAN ? 2 : FAM == HMM_GAMMA ? 3 : FAM == HMM_STUDENT_T ? 4
         : FAM == HMM_POISSON ? 1 : 0;
}

// acc[k] += g * term_k(y) for one state (compile-time family)
// ly = log y (used by the Gamma family only)
template <int FAM, typename R, int K, typename KT>
__device__ __forceinline__ void fam_accumulate(R g, R y, R ly, const StateConsts<KT> &k,
                                               R (&acc)[K]) {
    if constexpr (FAM == HMM_GAUSSIAN) {
        R d = y - (R)k.c0;
        R gd = g * d;
        acc[0] += gd;
        acc[1] = fma(gd, d, acc[1]);
    } else if constexpr (FAM == HMM_GAMMA) {
        R gy = g * y;
        acc[0] += gy;
        acc[1] = fma(g, ly, acc[1]);
        acc[2] = fma(gy, y, acc[2]);
    } else if constexpr (FAM == HMM_STUDENT_T) {
        R d = y - (R)k.c0;
        R q = (R)k.c1 * d * d;
        R u = (R)k.c4 * frcp((R)1 + q);
        R gu = g * u;
        acc[0] += gu;
        acc[1] = fma(gu, d, acc[1]);
        acc[2] = fma(gu * d, d, acc[2]);
        acc[3] = fma(g, flog(u) - u, acc[3]);
    } else if constexpr (FAM == HMM_POISSON) {
        acc[0] = fma(g, y, acc[0]);
    }
}

// log b_j(y_t) without the state-independent part, for any family (runtime),
// returned in FP64.  Poisson is evaluated from the FP64 constants (its values
// are of the size of y log lambda); the other families in R.
template <typename R>
__device__ __forceinline__ double emission_any(const StagedModel<R> &m, const ObsRef &o, int64_t row, int j,
                               double *common, bool *bad) {
    const int N = m.N, D = m.D;
    switch (m.family) {
    case HMM_GAUSSIAN:
    case HMM_GAMMA:
    case HMM_STUDENT_T: {
        R y = load_obs<R>(o, row);
        StateConsts<R> k = load_consts(m.ep, j, true);
        Emit<R> e;
        if (m.family == HMM_GAUSSIAN) e = emit_scalar<HMM_GAUSSIAN, R>(y, k, true);
        else if (m.family == HMM_GAMMA) e = emit_scalar<HMM_GAMMA, R>(y, k, true);
        else e = emit_scalar<HMM_STUDENT_T, R>(y, k, true);
        *common = e.common;
        *bad = e.bad;
        return (double)e.ell;
    }
    case HMM_POISSON: {
        double y = load_obs<double>(o, row);
        StateConsts<double> k = load_consts(m.ep64, j, true);
        Emit<double> e = emit_scalar<HMM_POISSON, double>(y, k, true);
        *common = e.common;
        *bad = e.bad;
        return e.ell;
    }
    case HMM_DIAG_GAUSSIAN: {
        R s = m.ep[j * EP_STRIDE];
        bool b = false;
        for (int d = 0; d < D; ++d) {
            R y = load_obs<R>(o, row * D + d);
            b |= !isfinite(y);
            R dv = y - m.mv[(size_t)j * D + d];
            s = fma(m.mv[(size_t)N * D + (size_t)j * D + d], dv * dv, s);
        }
        *common = 0.0;
        *bad = b;
        return (double)s;
    }
    case HMM_FULL_GAUSSIAN: {
        const R *mu = m.mv + (size_t)j * D;
        const R *Li = m.mv + (size_t)N * D + (size_t)j * D * D;
        R q = (R)0;
        bool b = false;
        for (int r = 0; r < D; ++r) {
            R z = (R)0;
            for (int c = 0; c <= r; ++c) {
                R y = load_obs<R>(o, row * D + c);
                z = fma(Li[r * D + c], y - mu[c], z);
            }
            q = fma(z, z, q);
        }
        for (int c = 0; c < D; ++c) b |= !isfinite(load_obs<R>(o, row * D + c));
        *common = 0.0;
        *bad = b;
        return (double)(m.ep[j * EP_STRIDE] - (R)0.5 * q);
    }
    default: {   // table
        R v = load_obs<R>(o, row * N + j);
        *common = 0.0;
        *bad = isnan(v) || (v > (R)0 && isinf(v));
        return (double)v;
    }
    }
}

// locate the sequence b owning chunk c: largest b with cbase[b] <= c
__device__ __forceinline__ int find_seq(const int *cbase, int nseq, int c) {
    int lo = 0, hi = nseq - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (cbase[mid] <= c) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace hmmk
