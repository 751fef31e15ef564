// k_xi.hip -- the transition statistics of the large-state path on the matrix
// cores.
//
// With w'_t = e_t o b_t 2^{-x_t} / Z_t written by the backward sweep (zero on
// each sequence's first step), the pooled transition statistic of section 3.1
// is sum_t xi_t(i,j) = a_ij * C_ij with
//   C = sum_k alpha_k^T w'_{k+1}     (k over all rows of the batch but the last),
// a dense contraction over K = sum T - 1 rows.  The rows are cut into slices;
// per slice, each wave accumulates a 64 x 128 tile of C with
// v_mfma_f{64,32}_16x16x4 (32 independent 16x16 blocks), and
// the slice partials are added in a fixed order in FP64.
//
// Operand layout of the 16x16x4 instructions (lane l): A row l % 16, k = l / 16;
// B column l % 16, k = l / 16; result column l % 16 and, in register v, row
// 4 (l / 16) + v for f32 but row l / 16 + 4 v for f64 (both checked on the
// device with exact small-integer products).
// A lane loads four consecutive entries of a row (one 16-byte load in single
// precision, two in double), so tile row i = i0 + 4 m + u belongs to block u
// at block row m (and likewise for columns): the blocks hold a fixed
// permutation of the tile, undone when the partials are summed.
#include "dev_common.hpp"

namespace hmmk {

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

template <typename R>
struct XiMfma;
template <>
struct XiMfma<float> {
    typedef f32x4_t acc_t;
    __device__ static acc_t op(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};
template <>
struct XiMfma<double> {
    typedef f64x4_t acc_t;
    __device__ static acc_t op(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};

// Workgroup shape for padded state count NC: WI waves along i (64 rows each),
// WJ along j (128 columns each), HALVES workgroups per slice along j.
template <typename R, int NC>
struct XiCfg {
    static constexpr int WI = NC / 64;
    static constexpr int WJ = (sizeof(R) == 4 && NC == 256) ? 2 : 1;
    static constexpr int HALVES = NC / (128 * WJ);
    static constexpr int NT = 64 * WI * WJ;
    static constexpr int64_t PER_SLICE = (int64_t)NC * NC;   // partial entries per slice
};

// four consecutive entries of row `row` starting at column c (clamped to
// column 0 past the row's end)
template <typename R, bool VEC>
__device__ __forceinline__ void load4(const R *__restrict__ base, int64_t row, int c, int N,
                                      R (&v)[4]) {
    if constexpr (VEC) {
        // N % 4 == 0: a group of four is wholly inside or outside the row
        const R *p = base + row * N + (c < N ? c : 0);
        if constexpr (sizeof(R) == 4) {
            const float4 q = *reinterpret_cast<const float4 *>(p);
            v[0] = q.x;
            v[1] = q.y;
            v[2] = q.z;
            v[3] = q.w;
        } else {
            const double2 q0 = *reinterpret_cast<const double2 *>(p);
            const double2 q1 = *reinterpret_cast<const double2 *>(p + 2);
            v[0] = q0.x;
            v[1] = q0.y;
            v[2] = q1.x;
            v[3] = q1.y;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = base[row * N + (c + e < N ? c + e : 0)];
    }
}

// grid (HALVES, nslices); slice q covers rows [q ks, min(K, (q+1) ks)), ks a
// multiple of 4.  part[q][...] receives the slice's tile in block order.
template <typename R, int NC, bool VEC>
__global__ __launch_bounds__((XiCfg<R, NC>::NT)) void k_xi_mfma(const R *__restrict__ alpha,
                                                             const R *__restrict__ wp, int N,
                                                             int64_t K, int64_t ks,
                                                             R *__restrict__ part) {
    using C = XiCfg<R, NC>;
    using acc_t = typename XiMfma<R>::acc_t;
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    const int wi = w % C::WI, wj = w / C::WI;
    const int jh = blockIdx.x;
    const int i0 = 64 * wi + 4 * (l & 15);
    const int j0 = jh * (NC / C::HALVES) + 128 * wj + 4 * (l & 15);
    const int64_t kbeg = (int64_t)blockIdx.y * ks;
    const int64_t kend = min(K, kbeg + ks);
    acc_t acc[4][8];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) acc[u][v] = acc_t{0, 0, 0, 0};
    // No masks: columns outside the matrix only reach output entries that the
    // reduction drops, and a row at or past the slice end pairs alpha row
    // kbeg with w' row 0, which the backward sweep zeroes (no transition
    // enters a sequence's first step), so it adds nothing.
    auto fetch = [&](int64_t k0, R (&xa)[4], R (&xb)[8]) {
        const int64_t k = k0 + (l >> 4);
        const bool ok = k < kend;
        load4<R, VEC>(alpha, ok ? k : kbeg, i0, N, xa);
        R t0[4], t1[4];
        load4<R, VEC>(wp, ok ? k + 1 : 0, j0, N, t0);
        load4<R, VEC>(wp, ok ? k + 1 : 0, j0 + 64, N, t1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            xb[e] = t0[e];
            xb[4 + e] = t1[e];
        }
    };
    // NB groups of four rows in flight, each refilled right after its 32
    // products: a group's loads are issued NB - 1 groups before its use (the
    // compiler still waits for all loads once per pass over the NB groups,
    // so NB is as large as the registers allow)
    constexpr int NB = sizeof(R) == 8 ? 6 : 4;
    R ra[NB][4], rb[NB][8];
#pragma unroll
    for (int g = 0; g < NB; ++g) fetch(kbeg + 4 * g, ra[g], rb[g]);
    for (int64_t k0 = kbeg; k0 < kend; k0 += 4 * NB) {
#pragma unroll
        for (int g = 0; g < NB; ++g) {
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 8; ++v) acc[u][v] = XiMfma<R>::op(ra[g][u], rb[g][v], acc[u][v]);
            // refill this group's registers right behind its products (kept in
            // place: hoisting the loads would make the compiler rotate
            // registers and wait for every load at the end of the loop)
            __builtin_amdgcn_sched_barrier(0);
            fetch(k0 + 4 * (g + NB), ra[g], rb[g]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    // block order: ((jh WJ + wj) WI + wi) * 32 + 8 u + v, then lane, then the
    // four result rows of the lane
    R *dst = part + (int64_t)blockIdx.y * C::PER_SLICE +
             ((int64_t)((jh * C::WJ + wj) * C::WI + wi) * 32) * 256 + 4 * l;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            R *p = dst + (u * 8 + v) * 256;
            if constexpr (sizeof(R) == 4) {
                *reinterpret_cast<float4 *>(p) =
                    make_float4(acc[u][v][0], acc[u][v][1], acc[u][v][2], acc[u][v][3]);
            } else {
                *reinterpret_cast<double2 *>(p) = make_double2(acc[u][v][0], acc[u][v][1]);
                *reinterpret_cast<double2 *>(p + 2) = make_double2(acc[u][v][2], acc[u][v][3]);
            }
        }
}

// out[i N + j] = sum over slices (in slice order, FP64) of the partials
template <typename R, int NC>
__global__ __launch_bounds__(256) void k_xi_reduce(const R *__restrict__ part, int nsl, int N,
                                                    double *__restrict__ out) {
    using C = XiCfg<R, NC>;
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= C::PER_SLICE) return;
    double acc = 0.0;
    for (int q = 0; q < nsl; ++q) acc += (double)part[(int64_t)q * C::PER_SLICE + p];
    // decode the block order
    const int rv = (int)(p & 3);
    const int l = (int)((p >> 2) & 63);
    const int blk = (int)((p >> 8) & 31);
    const int wv = (int)(p >> 13);            // (jh WJ + wj) WI + wi
    const int wi = wv % C::WI, jw = wv / C::WI;
    const int u = blk >> 3, v = blk & 7;
    const int brow = sizeof(R) == 4 ? 4 * (l >> 4) + rv : (l >> 4) + 4 * rv;   // row in the block
    const int i = 64 * wi + 4 * brow + u;
    const int j = 128 * jw + 64 * (v >> 2) + 4 * (l & 15) + (v & 3);
    if (i < N && j < N) out[(int64_t)i * N + j] = acc;
}

int xi_nc(int N) { return N <= 128 ? 128 : 256; }

int xi_slices(bool f64, int N, int64_t total) {
    const int64_t K = total - 1;
    if (K <= 0) return 1;
    const int nc = xi_nc(N);
    // about one workgroup per compute unit, at least 64 rows per slice
    const int halves = nc / (128 * ((!f64 && nc == 256) ? 2 : 1));
    int target = nc == 256 ? 256 / halves : 512;
    const int64_t by_rows = (K + 63) / 64;
    return (int)(by_rows < target ? by_rows : target);
}

template <typename R, int NC>
static void launch_xi_t(const R *alpha, const R *wp, int N, int64_t K, R *part, int nsl,
                        double *out, hipStream_t s) {
    using C = XiCfg<R, NC>;
    int64_t ks = (K + nsl - 1) / nsl;
    ks = (ks + 3) / 4 * 4;
    const dim3 grid(C::HALVES, (unsigned)nsl);
    if (N % 4 == 0)
        hipLaunchKernelGGL((k_xi_mfma<R, NC, true>), grid, dim3(C::NT), 0, s, alpha, wp, N, K, ks, part);
    else
        hipLaunchKernelGGL((k_xi_mfma<R, NC, false>), grid, dim3(C::NT), 0, s, alpha, wp, N, K, ks, part);
    hipLaunchKernelGGL((k_xi_reduce<R, NC>), dim3((unsigned)(C::PER_SLICE / 256)), dim3(256), 0, s,
                       (const R *)part, nsl, N, out);
}

// out [N x N] FP64 = sum_k alpha[k]^T wp[k + 1] over k < K (K >= 1)
template <typename R>
void launch_xi_sum(const R *alpha, const R *wp, int N, int64_t K, R *part, int nsl, double *out,
                   hipStream_t s) {
    if (xi_nc(N) == 128)
        launch_xi_t<R, 128>(alpha, wp, N, K, part, nsl, out, s);
    else
        launch_xi_t<R, 256>(alpha, wp, N, K, part, nsl, out, s);
}

template void launch_xi_sum<float>(const float *, const float *, int, int64_t, float *, int,
                                   double *, hipStream_t);
template void launch_xi_sum<double>(const double *, const double *, int, int64_t, double *, int,
                                    double *, hipStream_t);

}  // namespace hmmk
