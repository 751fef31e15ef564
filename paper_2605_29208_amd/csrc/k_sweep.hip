// k_sweep.hip -- forward and backward sweeps of the large-state path
// (64 < N <= 256, FP32 and FP64): one workgroup of 512 threads per sequence.
//
// The recursions of section 3.2 (reading R13: normalised vectors with exact
// power-of-two offsets) need one vector-matrix product per step,
//   forward   x_t = e_t o (x_{t-1} A),      backward  b_{t-1} = A (e_t o b_t),
// i.e. N^2 FMA per step and sequence.  Each thread owns a register tile of
// the matrix (M = A forward, M = A^T backward) of r = NC/16 rows by s = NC/32
// columns (NC = padded state count, 128 or 256), so that an input entry read
// from LDS feeds s FMA and a partial sum written back covers r rows.
//
// Thread t = 64 w + l: row block q = 4 (w % 4) + l / 16, column block
// cb = 16 (w / 4) + l % 16.  A step is
//   1. the tile product over the wave's copy of the input vector (LDS,
//      wave-private, read with 16-byte broadcasts);
//   2. a reduce-scatter over the wave's four row blocks through the gfx950
//      permlane32/permlane16 swaps (one swap and one add per pair), leaving
//      s/4 column sums per lane;
//   3. these partial sums go to LDS (double-buffered by step parity);
//   4. one workgroup barrier;
//   5. every wave adds the four group partials of the NC/4 states that its
//      own row blocks consume next, scales them and writes its private copy
//      of the next input vector.  The two waves of a row group both do this,
//      so the next step needs no second barrier.
// Rescaling uses the largest entry of the step's input vector (known to
// every wave after the barrier), so the output stays in [min a_ij / 2, N]
// times a power of two, the range an exactly normalised input would give.
// When the staging kernel finds min a_ij too small for that (rescale
// interval 1), the output's own maximum is taken instead, at the cost of a
// second barrier per step.
//
// Double precision with NC = 256 keeps 12 of the tile's 16 rows in
// registers and the other 4 in LDS (128 KB): the matrix alone is 512 KB, the
// size of the register file.
#include "dev_common.hpp"

namespace hmmk {

template <typename R, int NC>
struct SwCfg {
    static constexpr int NT = 512;
    static constexpr int NW = NT / 64;
    static constexpr int r = NC / 16;              // tile rows
    static constexpr int s = NC / 32;              // tile columns
    static constexpr int RR = (sizeof(R) == 8 && NC == 256) ? 12 : r;   // rows in registers
    static constexpr int RL = r - RR;              // rows in LDS
    static constexpr int WR = NC / 4;              // states a wave produces (= 8 s)
    static constexpr int SV = s / 4;               // column sums per lane after the reduce
    static constexpr int PG = NC;                  // psum entries per row group
    // psum position of output column (cb, c): s cb + (c ^ H(cb)).  The XOR
    // swizzle puts the writers of one LDS pass (16 column blocks, one or two
    // residues c) and the readers (consecutive columns) on distinct banks,
    // for 4- and 8-byte entries alike (checked exhaustively on the host).
    __host__ __device__ static constexpr int H(int cbk) {
        return sizeof(R) == 4
                   ? (s == 8 ? (((cbk >> 2) & 1) | ((cbk >> 2) & 2) << 1) : 2 * ((cbk >> 3) & 1))
                   : (s == 8 ? (cbk >> 1) & 7 : (cbk >> 2) & 3);
    }
    __host__ __device__ static constexpr int pos(int col) {
        return s * (col / s) + ((col % s) ^ H(col / s));
    }
    static constexpr int XV = 16 / (int)sizeof(R); // entries per 16-byte LDS read
    // steps of inputs prefetched into registers (fewer where the tile fills them)
    static constexpr int PF = (sizeof(R) == 8 && NC == 256) ? 2 : 4;
    static constexpr int PFB = (sizeof(R) == 8 && NC == 256) ? 1 : 4;   // backward (three rings)
    static_assert(RR % XV == 0 && RL % XV == 0, "tile rows must fill 16-byte reads");
};

template <typename R, int NC>
struct SwShared {
    using C = SwCfg<R, NC>;
    R psum[2][4][C::PG];
    R xw[C::NW][C::WR];
    R hw[C::NW][C::WR];   // backward: a_t o b_t of the wave's states, kept over the barrier
    uint32_t gmax[2][4];   // high words of group maxima (see hiword)
    uint32_t gE[4];
    R zsum[2][4];
    double red[C::NW];
};

template <typename R>
struct Vec16;
template <>
struct Vec16<float> {
    typedef float4 T;
    __device__ static float get(const float4 &v, int k) {
        return k == 0 ? v.x : (k == 1 ? v.y : (k == 2 ? v.z : v.w));
    }
};
template <>
struct Vec16<double> {
    typedef double2 T;
    __device__ static double get(const double2 &v, int k) { return k == 0 ? v.x : v.y; }
};

// Sum of x over lanes l and l ^ 32 in lanes with bit 5 clear, sum of y in
// the others (one permlane32 swap).
__device__ __forceinline__ float pair_sum32(float x, float y) {
    auto r = __builtin_amdgcn_permlane32_swap(__builtin_bit_cast(uint32_t, x),
                                              __builtin_bit_cast(uint32_t, y), false, false);
    return __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
}
__device__ __forceinline__ float pair_sum16(float x, float y) {
    auto r = __builtin_amdgcn_permlane16_swap(__builtin_bit_cast(uint32_t, x),
                                              __builtin_bit_cast(uint32_t, y), false, false);
    return __builtin_bit_cast(float, (uint32_t)r[0]) + __builtin_bit_cast(float, (uint32_t)r[1]);
}
__device__ __forceinline__ double pair_sum32(double x, double y) {
    const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
    auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
    auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    const double p = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]);
    const double q = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]);
    return p + q;
}
__device__ __forceinline__ double pair_sum16(double x, double y) {
    const uint64_t a = __builtin_bit_cast(uint64_t, x), b = __builtin_bit_cast(uint64_t, y);
    auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
    auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    const double p = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[0] << 32) | (uint32_t)lo[0]);
    const double q = __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi[1] << 32) | (uint32_t)lo[1]);
    return p + q;
}

// Rescaling needs only the binary exponent of a vector's largest entry.  The
// entries are >= 0, so the exponent of the largest one is that of the largest
// high word taken as an unsigned integer (the whole word in single precision,
// the upper 32 bits in double): the maximum runs on integers, without the
// quieting that floating-point max needs.
__device__ __forceinline__ uint32_t hiword(float x) { return __builtin_bit_cast(uint32_t, x); }
__device__ __forceinline__ uint32_t hiword(double x) {
    return (uint32_t)(__builtin_bit_cast(uint64_t, x) >> 32);
}
template <typename R>
__device__ __forceinline__ int hiword_exp(uint32_t u) {
    if constexpr (sizeof(R) == 4)
        return fexp(__builtin_bit_cast(float, u));
    else
        return fexp(__builtin_bit_cast(double, (uint64_t)u << 32));
}
__device__ __forceinline__ uint32_t umax(uint32_t a, uint32_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
    v = umax(v, (uint32_t)dpp_i<DPP_QP_X1>((int)v));
    v = umax(v, (uint32_t)dpp_i<DPP_QP_X2>((int)v));
    v = umax(v, (uint32_t)dpp_i<DPP_HALF_MIRROR>((int)v));
    v = umax(v, (uint32_t)dpp_i<DPP_ROW_MIRROR>((int)v));
    auto r16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    v = umax((uint32_t)r16[0], (uint32_t)r16[1]);
    auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return umax((uint32_t)r32[0], (uint32_t)r32[1]);
}
__device__ __forceinline__ uint32_t umax4(const uint32_t *g) {
    return umax(umax(g[0], g[1]), umax(g[2], g[3]));
}

// The thread's view of the sweep: tile, lane roles and LDS positions.
template <typename R, int NC>
struct SwTile {
    using C = SwCfg<R, NC>;
    using V = typename Vec16<R>::T;
    R a[C::RR][C::s];
    int w, l, q_lo, q_hi, cb, cb_hi;
    // reader role: the state this lane forms after the barrier
    int jrow, rho, ppos;
    bool rlive, writer;

    __device__ void init(const R *__restrict__ M, int N, V *alds) {
        const int tid = threadIdx.x;
        w = tid >> 6;
        l = tid & 63;
        q_lo = l >> 4;
        q_hi = w & 3;
        cb_hi = w >> 2;
        cb = 16 * cb_hi + (l & 15);
        const int row0 = (4 * q_hi + q_lo) * C::r, col0 = cb * C::s;
        // unconditional loads at clamped indices, entries outside the matrix zero
#pragma unroll
        for (int k = 0; k < C::RR; ++k)
#pragma unroll
            for (int c = 0; c < C::s; ++c) {
                const int i = row0 + k, j = col0 + c;
                const R v = M[min(i, N - 1) * N + min(j, N - 1)];
                a[k][c] = (i < N && j < N) ? v : (R)0;
            }
        if constexpr (C::RL > 0) {
            // LDS rows as 16-byte pairs of adjacent columns, wave-major: entry
            // e of lane l of wave w at ((w * EPL + e) * 64 + l), so a wave's
            // read of one entry is 1 KB contiguous and a lane's entries lie
            // 1 KB apart (all within the 16-bit LDS offset of one address)
            constexpr int EPL = C::RL * (C::s / 2);
#pragma unroll
            for (int k = 0; k < C::RL; ++k)
#pragma unroll
                for (int cp = 0; cp < C::s / 2; ++cp) {
                    const int i = row0 + C::RR + k, j = col0 + 2 * cp;
                    const R v0 = M[min(i, N - 1) * N + min(j, N - 1)];
                    const R v1 = M[min(i, N - 1) * N + min(j + 1, N - 1)];
                    V p;
                    p.x = (i < N && j < N) ? v0 : (R)0;
                    p.y = (i < N && j + 1 < N) ? v1 : (R)0;
                    alds[(w * EPL + k * (C::s / 2) + cp) * 64 + l] = p;
                }
        }
        rho = l % C::WR;
        jrow = q_hi * C::WR + rho;
        ppos = C::pos(jrow);
        rlive = jrow < N;
        writer = cb_hi == 0 && l < C::WR;
    }

    // partial products of the tile over the wave's input copy, reduced over
    // the wave's four row blocks and stored to psum[buf]
    __device__ __forceinline__ void product(SwShared<R, NC> &sh, const V *alds, int buf) const {
        R acc[C::s];
#pragma unroll
        for (int c = 0; c < C::s; ++c) acc[c] = (R)0;
        const R *xr = &sh.xw[w][q_lo * C::r];
#pragma unroll
        for (int k = 0; k < C::RR; k += C::XV) {
            const V xv = *reinterpret_cast<const V *>(xr + k);
#pragma unroll
            for (int kk = 0; kk < C::XV; ++kk) {
                const R xk = Vec16<R>::get(xv, kk);
#pragma unroll
                for (int c = 0; c < C::s; ++c) acc[c] = fma(xk, a[k + kk][c], acc[c]);
            }
        }
        if constexpr (C::RL > 0) {
            constexpr int EPL = C::RL * (C::s / 2);
            const V *base = alds + w * EPL * 64 + l;
#pragma unroll
            for (int k = 0; k < C::RL; k += C::XV) {
                const V xv = *reinterpret_cast<const V *>(xr + C::RR + k);
#pragma unroll
                for (int kk = 0; kk < C::XV; ++kk) {
                    const R xk = Vec16<R>::get(xv, kk);
#pragma unroll
                    for (int cp = 0; cp < C::s / 2; ++cp) {
                        const V av = base[((k + kk) * (C::s / 2) + cp) * 64];
                        acc[2 * cp] = fma(xk, av.x, acc[2 * cp]);
                        acc[2 * cp + 1] = fma(xk, av.y, acc[2 * cp + 1]);
                    }
                }
            }
        }
        // reduce-scatter: lane bit 5, then bit 4; lane keeps columns
        // SV * q_lo + e (e < SV) of its column block
        R v1[C::s / 2];
#pragma unroll
        for (int c = 0; c < C::s / 2; ++c) v1[c] = pair_sum32(acc[c], acc[c + C::s / 2]);
#pragma unroll
        for (int e = 0; e < C::SV; ++e) {
            const R u = pair_sum16(v1[e], v1[e + C::SV]);
            sh.psum[buf][q_hi][C::pos(C::s * cb + C::SV * q_lo + e)] = u;
        }
    }

    __device__ __forceinline__ R gather(const SwShared<R, NC> &sh, int buf) const {
        return (sh.psum[buf][0][ppos] + sh.psum[buf][1][ppos]) +
               (sh.psum[buf][2][ppos] + sh.psum[buf][3][ppos]);
    }
};

// ---------------------------------------------------------------- forward
template <typename R, int NC>
__global__ __launch_bounds__(512) void k_sw_fwd(StagedModel<R> m, const int64_t *__restrict__ offsets,
                                                const R *__restrict__ etab,
                                                const double *__restrict__ mt, R *__restrict__ alpha,
                                                int32_t *__restrict__ aexp,
                                                double *__restrict__ loglik,
                                                int32_t *__restrict__ status) {
    using C = SwCfg<R, NC>;
    using V = typename Vec16<R>::T;
    __shared__ __align__(16) SwShared<R, NC> sh;
    __shared__ __align__(16) V alds[C::RL > 0 ? C::RL * (C::s / 2) * C::NT : 1];
    const int N = m.N;
    SwTile<R, NC> tl;
    tl.init(m.A, N, alds);
    const int64_t b = blockIdx.x;
    const int64_t off = offsets[b];
    const int T = (int)(offsets[b + 1] - off);
    const int nrm = *m.nrm;
    const bool exact = nrm == 1;
    const int per = nrm >= 4 ? 2 : 1;
    const int jc = min(tl.jrow, N - 1);
    const bool lead = tl.l == 0 && tl.cb_hi == 0;
    // t = 0: pi o e_0, normalised exactly
    // row pointers are uniform; lanes add their state index
    const R *erow = etab + off * N;
    R *arow = alpha + off * N;
    R v = tl.rlive ? m.pi[jc] * erow[jc] : (R)0;
    {
        const uint32_t wm = wave_umax(hiword(v));
        if (lead) sh.gE[tl.q_hi] = wm;
    }
    __syncthreads();   // also publishes the LDS rows of the tile
    int ex = __builtin_amdgcn_readfirstlane(hiword_exp<R>(umax4(sh.gE)));
    v = fldexp(v, -ex);
    int64_t E = ex;
    if (tl.writer && tl.rlive) arow[tl.jrow] = v;
    if (threadIdx.x == 0) aexp[off] = ex;
    if (tl.l < C::WR) sh.xw[tl.w][tl.rho] = v;
    wave_lds_order();
    R ring[C::PF];
#pragma unroll
    for (int u = 0; u < C::PF; ++u) ring[u] = (etab + (off + min(1 + u, T - 1)) * N)[jc];
    for (int t0 = 1; t0 < T; t0 += C::PF) {
#pragma unroll
        for (int u = 0; u < C::PF; ++u) {
            const int t = t0 + u;
            if (t >= T) break;
            const R e = ring[u];
            ring[u] = (etab + (off + min(t + C::PF, T - 1)) * N)[jc];
            const int buf = t & 1;
            const bool resc = !exact && (t % per) == 0;
            if (resc) {
                // largest entry of this step's input vector
                const uint32_t wm = wave_umax(hiword(v));
                if (lead) sh.gmax[buf][tl.q_hi] = wm;
            }
            tl.product(sh, alds, buf);
            __syncthreads();
            R raw = tl.gather(sh, buf);
            raw = tl.rlive ? raw * e : (R)0;
            ex = 0;
            if (exact) {
                const uint32_t wm = wave_umax(hiword(raw));
                if (lead) sh.gE[tl.q_hi] = wm;
                __syncthreads();
                ex = hiword_exp<R>(umax4(sh.gE));
            } else if (resc) {
                ex = hiword_exp<R>(umax4(sh.gmax[buf]));
            }
            ex = __builtin_amdgcn_readfirstlane(ex);   // uniform: kept in scalar registers
            v = fldexp(raw, -ex);
            E += ex;
            if (tl.writer && tl.rlive) (arow + (int64_t)t * N)[tl.jrow] = v;
            if (threadIdx.x == 0) aexp[off + t] = ex;
            if (tl.l < C::WR) sh.xw[tl.w][tl.rho] = v;
            wave_lds_order();
        }
    }
    // log P(y) = sum of the per-step log shifts + E log 2 + log sum_j x_{T-1}(j)
    double ls = 0.0;
    for (int t = threadIdx.x; t < T; t += C::NT) ls += mt[off + t];
    const double lsw = wave_sum_r(ls);
    const R z = wave_sum_r((tl.cb_hi == 0 && tl.l < C::WR) ? v : (R)0);
    if (tl.l == 0) sh.red[tl.w] = lsw;
    if (lead) sh.zsum[0][tl.q_hi] = z;
    __syncthreads();
    if (threadIdx.x == 0) {
        double logS = 0.0;
        for (int k = 0; k < C::NW; ++k) logS += sh.red[k];
        const R zt = (sh.zsum[0][0] + sh.zsum[0][1]) + (sh.zsum[0][2] + sh.zsum[0][3]);
        double ll;
        int st;
        if (*m.perr) {
            ll = __builtin_nan("");
            st = 4;
        } else if (isnan(logS)) {
            ll = __builtin_nan("");
            st = 2;
        } else if (!(zt > (R)0) || isinf(logS)) {
            ll = -__builtin_inf();
            st = 1;
        } else {
            ll = logS + (double)E * 0.69314718055994530942 + log((double)zt);
            st = 0;
        }
        loglik[b] = ll;
        status[b] = st;
    }
}

// ---------------------------------------------------------------- backward
// Also forms gamma_t = a_t o b_t / Z_t and w'_t = e_t o b_t 2^{-x_t} / Z_t
// (x_t the forward exponent of step t, Z_t = sum a_t o b_t), written over
// e_t in place; row 0 of each sequence gets w' = 0.
template <typename R, int NC>
__global__ __launch_bounds__(512) void k_sw_bwd(StagedModel<R> m, const int64_t *__restrict__ offsets,
                                                R *__restrict__ etab, const R *__restrict__ alpha,
                                                const int32_t *__restrict__ aexp,
                                                const int32_t *__restrict__ status,
                                                R *__restrict__ gamma) {
    using C = SwCfg<R, NC>;
    using V = typename Vec16<R>::T;
    __shared__ __align__(16) SwShared<R, NC> sh;
    __shared__ __align__(16) V alds[C::RL > 0 ? C::RL * (C::s / 2) * C::NT : 1];
    const int N = m.N;
    SwTile<R, NC> tl;
    tl.init(m.AT, N, alds);
    const int64_t b = blockIdx.x;
    const int64_t off = offsets[b];
    const int T = (int)(offsets[b + 1] - off);
    const bool use = status[b] == 0;
    const int nrm = *m.nrm;
    const bool exact = nrm == 1;
    const int per = nrm >= 4 ? 2 : 1;
    const int jc = min(tl.jrow, N - 1);
    const bool lead = tl.l == 0 && tl.cb_hi == 0;
    R bt = tl.rlive ? (R)1 : (R)0;   // b_{T-1}
    R ra[C::PFB], re[C::PFB];
    int rx[C::PFB];
#pragma unroll
    for (int u = 0; u < C::PFB; ++u) {
        const int64_t row = off + max(T - 1 - u, 0);
        ra[u] = (alpha + row * N)[jc];
        re[u] = (etab + row * N)[jc];
        rx[u] = aexp[row];
    }
    __syncthreads();   // the LDS rows of the tile
    for (int t0 = T - 1; t0 >= 1; t0 -= C::PFB) {
#pragma unroll
        for (int u = 0; u < C::PFB; ++u) {
            const int t = t0 - u;
            if (t < 1) break;
            const R a = tl.rlive ? ra[u] : (R)0, e = tl.rlive ? re[u] : (R)0;
            const int xt = rx[u];
            {
                const int64_t row = off + max(t - C::PFB, 0);
                ra[u] = (alpha + row * N)[jc];
                re[u] = (etab + row * N)[jc];
                rx[u] = aexp[row];
            }
            const int buf = t & 1;
            const R h = a * bt, wv = e * bt;
            {
                const R zs = wave_sum_r(tl.l < C::WR ? h : (R)0);
                if (lead) sh.zsum[buf][tl.q_hi] = zs;
            }
            const bool resc = !exact && ((T - 1 - t) % per) == 0;
            if (resc) {
                const uint32_t wm = wave_umax(hiword(wv));
                if (lead) sh.gmax[buf][tl.q_hi] = wm;
            }
            if (tl.l < C::WR) {
                sh.xw[tl.w][tl.rho] = wv;
                sh.hw[tl.w][tl.rho] = h;
            }
            wave_lds_order();
            tl.product(sh, alds, buf);
            __syncthreads();
            const R Z = (sh.zsum[buf][0] + sh.zsum[buf][1]) + (sh.zsum[buf][2] + sh.zsum[buf][3]);
            const R rz = (R)1 / Z;
            if (tl.writer && tl.rlive) {
                // h and w of this lane's state, read back from the wave's own slots
                const int64_t row = off + t;
                (gamma + row * N)[tl.jrow] = use ? sh.hw[tl.w][tl.rho] * rz : (R)0;
                (etab + row * N)[tl.jrow] = use ? fldexp(sh.xw[tl.w][tl.rho] * rz, -xt) : (R)0;
            }
            R raw = tl.gather(sh, buf);
            raw = tl.rlive ? raw : (R)0;
            int ex = 0;
            if (exact) {
                const uint32_t wm = wave_umax(hiword(raw));
                if (lead) sh.gE[tl.q_hi] = wm;
                __syncthreads();
                ex = hiword_exp<R>(umax4(sh.gE));
            } else if (resc) {
                ex = hiword_exp<R>(umax4(sh.gmax[buf]));
            }
            ex = __builtin_amdgcn_readfirstlane(ex);
            bt = fldexp(raw, -ex);
        }
    }
    // t = 0: gamma_0; w'_0 = 0 (no transition into the first step)
    {
        // alpha_0 is already in the ring: slot (T - 1) % PF was last loaded
        // for row max(t - PF, 0) = 0
        R a0 = ra[0];
#pragma unroll
        for (int u = 1; u < C::PFB; ++u)
            if ((T - 1) % C::PFB == u) a0 = ra[u];
        const R a = tl.rlive ? a0 : (R)0;
        const R h = a * bt;
        const R zs = wave_sum_r(tl.l < C::WR ? h : (R)0);
        if (lead) sh.zsum[0][tl.q_hi] = zs;
        __syncthreads();
        const R Z = (sh.zsum[0][0] + sh.zsum[0][1]) + (sh.zsum[0][2] + sh.zsum[0][3]);
        if (tl.writer && tl.rlive) {
            gamma[off * N + tl.jrow] = use ? h * ((R)1 / Z) : (R)0;
            etab[off * N + tl.jrow] = (R)0;
        }
    }
}

// NC = 128 for N <= 128, else 256 (N in (128, 192] runs padded)
template <typename R>
void launch_sw_sweep(bool fwd, const StagedModel<R> &m, const int64_t *offsets, int64_t nseq,
                     R *etab, const double *mt, R *alpha, int32_t *aexp, double *loglik,
                     int32_t *status, R *gamma, hipStream_t s) {
    const bool small = m.N <= 128;
    if (fwd) {
        if (small)
            hipLaunchKernelGGL((k_sw_fwd<R, 128>), dim3((unsigned)nseq), dim3(512), 0, s, m, offsets,
                               (const R *)etab, mt, alpha, aexp, loglik, status);
        else
            hipLaunchKernelGGL((k_sw_fwd<R, 256>), dim3((unsigned)nseq), dim3(512), 0, s, m, offsets,
                               (const R *)etab, mt, alpha, aexp, loglik, status);
    } else {
        if (small)
            hipLaunchKernelGGL((k_sw_bwd<R, 128>), dim3((unsigned)nseq), dim3(512), 0, s, m, offsets,
                               etab, (const R *)alpha, (const int32_t *)aexp,
                               (const int32_t *)status, gamma);
        else
            hipLaunchKernelGGL((k_sw_bwd<R, 256>), dim3((unsigned)nseq), dim3(512), 0, s, m, offsets,
                               etab, (const R *)alpha, (const int32_t *)aexp,
                               (const int32_t *)status, gamma);
    }
}

template void launch_sw_sweep<float>(bool, const StagedModel<float> &, const int64_t *, int64_t,
                                     float *, const double *, float *, int32_t *, double *,
                                     int32_t *, float *, hipStream_t);
template void launch_sw_sweep<double>(bool, const StagedModel<double> &, const int64_t *, int64_t,
                                      double *, const double *, double *, int32_t *, double *,
                                      int32_t *, double *, hipStream_t);

}  // namespace hmmk
