// Group forest closeness (Section 5): the greedy of Algorithm 2 on dense
// matrices in HBM.
//
// f(S) = tr((L*_{-S})^{-1}); Algorithm 2 keeps M = (L*_{-S})^{-1} and, per
// step, adds the vertex v maximising |M e_v|^2 / M_vv and downdates
// M <- M - M e_v e_v^T M / M_vv (row and column v become zero).
//
// Layout: one N x N row-major binary64 matrix, N = n rounded up to 256; the
// padding is an identity block, never read by the greedy.  It first holds
// alpha L + I, inverted in place by blocked Gauss-Jordan with 256-wide pivot
// blocks (each pivot block inverted by the same method with 64-wide blocks in
// a 256 x 256 scratch; the panels and the rank-256 trailing update are fp64
// MFMA tile products), i.e. Omega; then, in place, the inverse of L*
// grounded at the first vertex v0, with slot v0 standing for u*.
#include "fc_group_kernels.hpp"

namespace fc {

namespace {

constexpr uint32_t kT = 64;        // tile edge
constexpr uint32_t kB = 256;       // pivot block width of the outer Gauss-Jordan
constexpr uint32_t kPad = kT + 1;  // LDS row stride (doubles): rows fall on different banks
constexpr uint32_t kThreads = 256;

typedef double double4_t __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 operand layout (wave64): lane l holds A[l % 16][l / 16]
// of the 16 x 4 left operand, B[l / 16][l % 16] of the 4 x 16 right operand,
// and D[l / 16 + 4 r][l % 16] in item r of the 16 x 16 result.
__device__ __forceinline__ uint32_t d_row(uint32_t lane, uint32_t r) { return (lane >> 4) + 4u * r; }
__device__ __forceinline__ uint32_t d_col(uint32_t lane) { return lane & 15u; }

// acc += X * Y over one wave's 32 x 32 quadrant (qr, qc) of a 64 x 64 tile,
// X 64 x K (row stride XS) and Y K x 64 (row stride kPad) in LDS.
template <uint32_t K = kT, uint32_t XS = kPad>
__device__ __forceinline__ void tile_mma(const double *X, const double *Y, uint32_t qr,
                                         uint32_t qc, uint32_t lane, double4_t (&acc)[2][2]) {
    const uint32_t li = lane & 15u, lk = lane >> 4;
#pragma unroll 4
    for (uint32_t k0 = 0; k0 < K; k0 += 4) {
        double a[2], b[2];
#pragma unroll
        for (uint32_t s = 0; s < 2; ++s) {
            a[s] = X[(qr + 16u * s + li) * XS + k0 + lk];
            b[s] = Y[(k0 + lk) * kPad + qc + 16u * s + li];
        }
#pragma unroll
        for (uint32_t s = 0; s < 2; ++s)
#pragma unroll
            for (uint32_t t = 0; t < 2; ++t)
                acc[s][t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[s], b[t], acc[s][t], 0, 0, 0);
    }
}

// Stage the 64 x 64 tile at (r0, c0) of a row-major N x N matrix into LDS,
// optionally negated.
__device__ __forceinline__ void stage(const double *__restrict__ A, uint32_t N, uint32_t r0,
                                      uint32_t c0, double *S, bool negate) {
    for (uint32_t e = threadIdx.x; e < kT * kT; e += kThreads) {
        const uint32_t r = e / kT, c = e % kT;
        const double x = A[static_cast<size_t>(r0 + r) * N + c0 + c];
        S[r * kPad + c] = negate ? -x : x;
    }
}

// The wave's quadrant and the global element of (s, t, item r) of it.
struct Quad {
    uint32_t qr, qc, lane;
};
__device__ __forceinline__ Quad quad() {
    const uint32_t w = threadIdx.x >> 6;
    return {32u * (w >> 1), 32u * (w & 1u), threadIdx.x & 63u};
}

// Pivot block inverse: D = A[p0.., p0..] (64 x 64, SPD) inverted by
// Gauss-Jordan without pivoting, written to Dinv (64 x 64, row-major).  The
// 256 threads hold the block in registers, a 4 x 4 sub-block each (thread
// (ty, tx) = rows 4 ty.., columns 4 tx..); step p publishes row p and column p
// (the multipliers, read before any row changes them) through LDS, double
// buffered by the step's parity so that one barrier per step suffices, and row
// p is scaled by the pivot's reciprocal.
__global__ __launch_bounds__(kThreads) void gj_pivot_kernel(const double *__restrict__ A, uint32_t N,
                                                            uint32_t p0, double *__restrict__ Dinv) {
    __shared__ double rowp[2][kT], colp[2][kT];
    const uint32_t tx = threadIdx.x & 15u, ty = threadIdx.x >> 4;
    double d[4][4];
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r)
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c)
            d[r][c] = A[static_cast<size_t>(p0 + 4u * ty + r) * N + p0 + 4u * tx + c];
    for (uint32_t p = 0; p < kT; ++p) {
        const uint32_t b = p & 1u, band = p >> 2, lp = p & 3u;
        if (tx == band)
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) colp[b][4u * ty + r] = d[r][lp];
        if (ty == band)
#pragma unroll
            for (uint32_t c = 0; c < 4; ++c) rowp[b][4u * tx + c] = d[lp][c];
        __syncthreads();
        const double inv = 1.0 / rowp[b][p];
        double rp[4];
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) {
            const uint32_t j = 4u * tx + c;
            rp[c] = (j == p ? 1.0 : rowp[b][j]) * inv;  // row p of the result
        }
#pragma unroll
        for (uint32_t r = 0; r < 4; ++r) {
            const uint32_t i = 4u * ty + r;
            const double f = colp[b][i];
#pragma unroll
            for (uint32_t c = 0; c < 4; ++c) {
                const uint32_t j = 4u * tx + c;
                // column p of row i becomes -f / piv; the others subtract f * row p
                d[r][c] = i == p ? rp[c] : (j == p ? 0.0 : d[r][c]) - f * rp[c];
            }
        }
    }
#pragma unroll
    for (uint32_t r = 0; r < 4; ++r)
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) Dinv[(4u * ty + r) * kT + 4u * tx + c] = d[r][c];
}

// Row panel: A[p-rows, j-tile] <- Dinv A[p-rows, j-tile] (j-tile != p);
// column panel: A[i-tile, p-cols] <- -A[i-tile, p-cols] Dinv (i-tile != p).
__global__ __launch_bounds__(kThreads) void gj_panel_kernel(double *__restrict__ A, uint32_t N,
                                                            uint32_t pt,
                                                            const double *__restrict__ Dinv,
                                                            uint32_t column) {
    const uint32_t t = blockIdx.x;
    if (t == pt) return;
    __shared__ double X[kT * kPad], Y[kT * kPad];
    const uint32_t p0 = pt * kT, t0 = t * kT;
    if (!column) {
        for (uint32_t e = threadIdx.x; e < kT * kT; e += kThreads)
            X[(e / kT) * kPad + e % kT] = Dinv[e];
        stage(A, N, p0, t0, Y, false);
    } else {
        stage(A, N, t0, p0, X, true);
        for (uint32_t e = threadIdx.x; e < kT * kT; e += kThreads)
            Y[(e / kT) * kPad + e % kT] = Dinv[e];
    }
    __syncthreads();
    const Quad q = quad();
    double4_t acc[2][2] = {};
    tile_mma(X, Y, q.qr, q.qc, q.lane, acc);
    const uint32_t r0 = column ? t0 : p0, c0 = column ? p0 : t0;
#pragma unroll
    for (uint32_t s = 0; s < 2; ++s)
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r) {
                const uint32_t row = q.qr + 16u * s + d_row(q.lane, r);
                const uint32_t col = q.qc + 16u * u + d_col(q.lane);
                A[static_cast<size_t>(r0 + row) * N + c0 + col] = acc[s][u][r];
            }
}

// Trailing update: A[i, j] -= A[i, p] A[p, j] for tiles i, j != p (A[i, p]
// still the old column panel, A[p, j] the new row panel).
__global__ __launch_bounds__(kThreads) void gj_update_kernel(double *__restrict__ A, uint32_t N,
                                                             uint32_t pt) {
    const uint32_t ti = blockIdx.y, tj = blockIdx.x;
    if (ti == pt || tj == pt) return;
    __shared__ double X[kT * kPad], Y[kT * kPad];
    const uint32_t p0 = pt * kT, i0 = ti * kT, j0 = tj * kT;
    stage(A, N, i0, p0, X, true);  // -A[i, p]
    stage(A, N, p0, j0, Y, false);
    __syncthreads();
    const Quad q = quad();
    double4_t acc[2][2];
#pragma unroll
    for (uint32_t s = 0; s < 2; ++s)
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                acc[s][u][r] = A[static_cast<size_t>(i0 + q.qr + 16u * s + d_row(q.lane, r)) * N + j0 +
                                 q.qc + 16u * u + d_col(q.lane)];
    tile_mma(X, Y, q.qr, q.qc, q.lane, acc);
#pragma unroll
    for (uint32_t s = 0; s < 2; ++s)
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                A[static_cast<size_t>(i0 + q.qr + 16u * s + d_row(q.lane, r)) * N + j0 + q.qc +
                  16u * u + d_col(q.lane)] = acc[s][u][r];
}

// Tile product over K = kchunks x kK: out[ti, tj] = (load_c ? out[ti, tj] : 0)
// + (negate_x ? -X : X)[ti, :] Y[:, tj], the K dimension streamed through LDS
// kK at a time (the accumulators stay in registers; 32-deep chunks keep the
// LDS tiles and the prefetch registers small enough for four workgroups per CU).  Tiles whose row tile is
// in [si0, si1) or whose column tile is in [sj0, sj1) are skipped.
constexpr uint32_t kK = 32;         // K chunk of gemm_kernel
constexpr uint32_t kPadK = kK + 1;  // its X tile's row stride (doubles)
struct GemmArgs {
    const double *X;
    const double *Y;
    double *out;
    uint32_t ldx, ldy, ldo, kchunks;
    uint32_t si0, si1, sj0, sj1;
    uint32_t load_c, negate_x;
};

__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void gemm_kernel(GemmArgs g) {
    const uint32_t ti = blockIdx.y, tj = blockIdx.x;
    if ((ti >= g.si0 && ti < g.si1) || (tj >= g.sj0 && tj < g.sj1)) return;
    __shared__ double X[kT * kPadK], Y[kK * kPad];
    const Quad q = quad();
    double4_t acc[2][2];
    const uint32_t i0 = ti * kT, j0 = tj * kT;
#pragma unroll
    for (uint32_t s = 0; s < 2; ++s)
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                acc[s][u][r] = g.load_c ? g.out[static_cast<size_t>(i0 + q.qr + 16u * s + d_row(q.lane, r)) *
                                                    g.ldo + j0 + q.qc + 16u * u + d_col(q.lane)]
                                        : 0.0;
    // software pipeline: chunk c + 1 is loaded into registers while the
    // matrix cores work on chunk c from LDS
    constexpr uint32_t kPer = kT * kK / kThreads;  // elements of a chunk per thread
    double xr[kPer], yr[kPer];
    const double sx = g.negate_x ? -1.0 : 1.0;
    auto load = [&](uint32_t c) {
#pragma unroll
        for (uint32_t q2 = 0; q2 < kPer; ++q2) {
            const uint32_t e = q2 * kThreads + threadIdx.x;
            xr[q2] = g.X[static_cast<size_t>(i0 + e / kK) * g.ldx + c * kK + e % kK];
            yr[q2] = g.Y[static_cast<size_t>(c * kK + e / kT) * g.ldy + j0 + e % kT];
        }
    };
    load(0);
    for (uint32_t c = 0; c < g.kchunks; ++c) {
        __syncthreads();
#pragma unroll
        for (uint32_t q2 = 0; q2 < kPer; ++q2) {
            const uint32_t e = q2 * kThreads + threadIdx.x;
            X[(e / kK) * kPadK + e % kK] = sx * xr[q2];
            Y[(e / kT) * kPad + e % kT] = yr[q2];
        }
        __syncthreads();
        if (c + 1 < g.kchunks) load(c + 1);
        tile_mma<kK, kPadK>(X, Y, q.qr, q.qc, q.lane, acc);
    }
#pragma unroll
    for (uint32_t s = 0; s < 2; ++s)
#pragma unroll
        for (uint32_t u = 0; u < 2; ++u)
#pragma unroll
            for (uint32_t r = 0; r < 4; ++r)
                g.out[static_cast<size_t>(i0 + q.qr + 16u * s + d_row(q.lane, r)) * g.ldo + j0 + q.qc +
                      16u * u + d_col(q.lane)] = acc[s][u][r];
}

// dst[r][c] = src[r][c] for a rows x cols block (row strides lds, ldd).
__global__ __launch_bounds__(kThreads) void copy_block_kernel(const double *__restrict__ src,
                                                              uint32_t lds, double *__restrict__ dst,
                                                              uint32_t ldd, uint32_t cols) {
    const uint32_t r = blockIdx.y;
    for (uint32_t c = blockIdx.x * kThreads + threadIdx.x; c < cols; c += gridDim.x * kThreads)
        dst[static_cast<size_t>(r) * ldd + c] = src[static_cast<size_t>(r) * lds + c];
}

__global__ __launch_bounds__(kThreads) void gj_put_kernel(double *__restrict__ A, uint32_t N,
                                                          uint32_t pt,
                                                          const double *__restrict__ Dinv) {
    const uint32_t p0 = pt * kT;
    for (uint32_t e = threadIdx.x; e < kT * kT; e += kThreads)
        A[static_cast<size_t>(p0 + e / kT) * N + p0 + e % kT] = Dinv[e];
}

// alpha L + I of the first n rows (weighted when w is not null), identity on
// the padding, zeros elsewhere; one thread per row, after the matrix was zeroed.
__global__ __launch_bounds__(kThreads) void dense_build_kernel(const int32_t *__restrict__ row_ptr,
                                                               const int32_t *__restrict__ col_idx,
                                                               const double *__restrict__ w,
                                                               uint32_t n, uint32_t N, double alpha,
                                                               double *__restrict__ A) {
    const uint32_t v = blockIdx.x * kThreads + threadIdx.x;
    if (v >= N) return;
    double *row = A + static_cast<size_t>(v) * N;
    if (v >= n) {
        row[v] = 1.0;
        return;
    }
    double deg = 0.0;
    for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        const double we = w ? w[e] : 1.0;
        row[col_idx[e]] = -(alpha * we);
        deg += we;
    }
    row[v] = alpha * deg + 1.0;
}

// Diagonal (n entries) into out, for the argmin of the first vertex.
__global__ __launch_bounds__(kThreads) void diag_kernel(const double *__restrict__ A, uint32_t n,
                                                        uint32_t N, double *__restrict__ out) {
    const uint32_t v = blockIdx.x * kThreads + threadIdx.x;
    if (v < n) out[v] = A[static_cast<size_t>(v) * N + v];
}

// First vertex: the smallest id of minimal diagonal (Omega_vv >= 0, so the
// binary64 bits order as uint64).  sel[0] = min bits, then sel[1] = min id.
__global__ __launch_bounds__(kThreads) void argmin_bits_kernel(const double *__restrict__ x, uint32_t n,
                                                               unsigned long long *sel) {
    const uint32_t v = blockIdx.x * kThreads + threadIdx.x;
    if (v < n) atomicMin(&sel[0], static_cast<unsigned long long>(__double_as_longlong(x[v])));
}
__global__ __launch_bounds__(kThreads) void argmin_id_kernel(const double *__restrict__ x, uint32_t n,
                                                             unsigned long long *sel) {
    const uint32_t v = blockIdx.x * kThreads + threadIdx.x;
    if (v < n && static_cast<unsigned long long>(__double_as_longlong(x[v])) == sel[0])
        atomicMin(&sel[1], static_cast<unsigned long long>(v));
}

// Change of ground from u* to v0: with c = column v0 of Omega and Omega(u*, .)
// = 0 (slot v0 stands for u*), M[i][j] = O(i, j) - c^(i) - c^(j) + c[v0],
// O(i, j) = Omega[i][j] off row and column v0 and 0 on them, c^ = c with
// c^[v0] = 0 (identity of grounded inverses of one Laplacian:
// G_r(i, j) = P(i, j) - P(i, r) - P(r, j) + P(r, r) for any pseudo-inverse P).
__global__ __launch_bounds__(kThreads) void reground_kernel(double *__restrict__ A, uint32_t n,
                                                            uint32_t N, uint32_t v0,
                                                            const double *__restrict__ c) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t i = blockIdx.y;
    if (j >= n) return;
    const double cvv = c[v0];
    const double ci = i == v0 ? 0.0 : c[i], cj = j == v0 ? 0.0 : c[j];
    double *p = A + static_cast<size_t>(i) * N + j;
    const double o = (i == v0 || j == v0) ? 0.0 : *p;
    *p = (o - ci - cj) + cvv;
}

// The vertex of a greedy step: the host's v, or the device's choice *vsel
// (n when there is none: the step then changes nothing).
__device__ __forceinline__ uint32_t step_vertex(uint32_t v, const unsigned long long *vsel, uint32_t n) {
    if (!vsel) return v;
    const unsigned long long x = *vsel;
    return x < n ? static_cast<uint32_t>(x) : n;
}

__global__ __launch_bounds__(kThreads) void copy_col_kernel(const double *__restrict__ A, uint32_t n,
                                                            uint32_t N, uint32_t v0,
                                                            const unsigned long long *vsel,
                                                            double *__restrict__ col,
                                                            double *__restrict__ row) {
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t v = step_vertex(v0, vsel, n);
    if (i >= n || v >= n) return;
    col[i] = A[static_cast<size_t>(i) * N + v];
    if (row) row[i] = A[static_cast<size_t>(v) * N + i];
}

// Column sums of squares over row chunks of kChunk rows (part[chunk * N + j]),
// optionally after the downdate M[i][j] -= cv[i] rv[j] / piv of vertex v,
// whose row and column become zero.
constexpr uint32_t kChunk = 64;
__global__ __launch_bounds__(kThreads) void colsq_kernel(double *__restrict__ A, uint32_t n, uint32_t N,
                                                         uint32_t v0, const unsigned long long *vsel,
                                                         const double *__restrict__ cv,
                                                         const double *__restrict__ rv,
                                                         const double *__restrict__ pivp,
                                                         double *__restrict__ part) {
    const uint32_t j = blockIdx.x * kThreads + threadIdx.x;
    const uint32_t c = blockIdx.y;
    if (j >= n) return;
    const uint32_t v = step_vertex(v0, vsel, n);
    const uint32_t i0 = c * kChunk, i1 = min(n, i0 + kChunk);
    double s = 0.0;
    if (cv && v < n) {
        const double piv = *pivp;
        const double f = rv[j] / piv;
        for (uint32_t i = i0; i < i1; ++i) {
            double *p = A + static_cast<size_t>(i) * N + j;
            const double x = (i == v || j == v) ? 0.0 : *p - cv[i] * f;
            *p = x;
            s += x * x;
        }
    } else {
        for (uint32_t i = i0; i < i1; ++i) {
            const double x = A[static_cast<size_t>(i) * N + j];
            s += x * x;
        }
    }
    part[static_cast<size_t>(c) * N + j] = s;
}

// Order-preserving 64-bit key of a non-NaN binary64 value (-0 taken as +0):
// keys compare as the values do, and every key is above 0, the key of "no
// candidate".
__device__ __forceinline__ unsigned long long gain_key(double g) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(g + 0.0));
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// gain[j] = |M e_j|^2 / M_jj for candidates (not taken, not the u* slot),
// the chunk sums added in chunk order; per block, the largest candidate
// gain's key (0 with no candidate) in bmax[b], the smallest id of a
// candidate with that key (none: all ones) in bid[b], and the sum of its
// diagonal entries (in a fixed order) in bdiag[b].  Gains are >= 0 in exact
// arithmetic; a rounded negative one still competes by its value.  A NaN gain
// (non-finite entries in M) sets bit 1 of *bad.
__global__ __launch_bounds__(kThreads) void gain_kernel(const double *__restrict__ A, uint32_t n,
                                                        uint32_t N, uint32_t chunks,
                                                        const double *__restrict__ part,
                                                        const uint8_t *__restrict__ taken,
                                                        unsigned long long *__restrict__ bmax,
                                                        uint32_t *__restrict__ bid,
                                                        double *__restrict__ bdiag, uint32_t *bad) {
    __shared__ unsigned long long sk[kThreads];
    __shared__ uint32_t si[kThreads];
    __shared__ double sd[kThreads];
    const uint32_t t = threadIdx.x, j = blockIdx.x * kThreads + t;
    unsigned long long key = 0ull;
    bool ok = false;
    const double djj = j < n ? A[static_cast<size_t>(j) * N + j] : 0.0;
    if (j < n && !taken[j]) {
        double sum = 0.0;
        for (uint32_t c = 0; c < chunks; ++c) sum += part[static_cast<size_t>(c) * N + j];
        const double g = sum / djj;
        if (g == g) {
            key = gain_key(g);
            ok = true;
        } else {
            atomicOr(bad, 2u);
        }
    }
    sk[t] = key;
    sd[t] = djj;
    __syncthreads();
    for (uint32_t h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h) {
            sk[t] = max(sk[t], sk[t + h]);
            sd[t] += sd[t + h];
        }
        __syncthreads();
    }
    const unsigned long long top = sk[0];
    si[t] = ok && key == top ? j : ~0u;
    __syncthreads();
    for (uint32_t h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h) si[t] = min(si[t], si[t + h]);
        __syncthreads();
    }
    if (t == 0) {
        bmax[blockIdx.x] = top;
        bid[blockIdx.x] = si[0];
        bdiag[blockIdx.x] = sd[0];
    }
}

// The step's vertex from the gain blocks' results (every block of the next
// kernel reduces them the same way): the smallest id among the largest
// pattern, or n when there is none.
__device__ uint32_t reduce_choice(const unsigned long long *__restrict__ bmax,
                                  const uint32_t *__restrict__ bid, uint32_t nb, uint32_t n) {
    __shared__ unsigned long long sk[kThreads];
    __shared__ uint32_t si[kThreads];
    const uint32_t t = threadIdx.x;
    unsigned long long k = 0ull;
    for (uint32_t b = t; b < nb; b += kThreads) k = max(k, bmax[b]);
    sk[t] = k;
    __syncthreads();
    for (uint32_t h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h) sk[t] = max(sk[t], sk[t + h]);
        __syncthreads();
    }
    const unsigned long long top = sk[0];
    uint32_t id = ~0u;
    for (uint32_t b = t; b < nb; b += kThreads)
        if (bmax[b] == top) id = min(id, bid[b]);
    si[t] = id;
    __syncthreads();
    for (uint32_t h = kThreads / 2; h > 0; h >>= 1) {
        if (t < h) si[t] = min(si[t], si[t + h]);
        __syncthreads();
    }
    const uint32_t v = si[0];
    __syncthreads();  // the arrays are reused by a later call
    return v < n ? v : n;
}

// Column v of the chosen vertex (and its row) copied out before the downdate,
// v reduced from the gain blocks; block 0 also does the step's bookkeeping:
// taken[v] = 1, gout[s] = v, *piv = M[v][v], *vout = v for the downdate
// (all ones and bit 0 of *bad set when there is no candidate), and, when fout is not
// null, fout[s - 1] = the sum of the blocks' diagonal sums (f(S) of step s - 1).
__global__ __launch_bounds__(kThreads) void choose_copy_kernel(
    const double *__restrict__ A, uint32_t n, uint32_t N, const unsigned long long *__restrict__ bmax,
    const uint32_t *__restrict__ bid, const double *__restrict__ bdiag, uint32_t nb,
    uint8_t *__restrict__ taken, int32_t *gout, uint32_t s, double *piv, unsigned long long *vout,
    uint32_t *bad, double *__restrict__ fout, double *__restrict__ col, double *__restrict__ row) {
    const uint32_t v = reduce_choice(bmax, bid, nb, n);
    if (fout && blockIdx.x == 0 && threadIdx.x == 0) {
        // tr M before this step's downdate: f(S) after the previous step
        double tr = 0.0;
        for (uint32_t b = 0; b < nb; ++b) tr += bdiag[b];
        fout[s - 1] = tr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (v < n) {
            taken[v] = 1u;
            gout[s] = static_cast<int32_t>(v);
            *piv = A[static_cast<size_t>(v) * N + v];
            *vout = v;
        } else {
            gout[s] = -1;
            atomicOr(bad, 1u);
            *vout = ~0ull;
        }
    }
    const uint32_t i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n || v >= n) return;
    col[i] = A[static_cast<size_t>(i) * N + v];
    row[i] = A[static_cast<size_t>(v) * N + i];
}

// tr(M) over the first n slots (one block, fixed order), into *out; also
// stores M[v][v] into *piv when v < n.
__global__ __launch_bounds__(kThreads) void trace_kernel(const double *__restrict__ A, uint32_t n,
                                                         uint32_t N, uint32_t v,
                                                         double *__restrict__ out,
                                                         double *__restrict__ piv) {
    __shared__ double s[kThreads];
    double t = 0.0;
    for (uint32_t i = threadIdx.x; i < n; i += kThreads) t += A[static_cast<size_t>(i) * N + i];
    s[threadIdx.x] = t;
    __syncthreads();
    for (uint32_t h = kThreads / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out = s[0];
        if (v < n) *piv = A[static_cast<size_t>(v) * N + v];
    }
}

inline unsigned int blocks_for(uint32_t items) { return (items + kThreads - 1) / kThreads; }

}  // namespace

uint32_t group_dim(uint32_t n) { return (n + kB - 1) / kB * kB; }
size_t group_scratch_doubles(uint32_t N) {
    return static_cast<size_t>(kB) * kB + 2 * static_cast<size_t>(kB) * N + kT * kT;
}
uint32_t group_chunks(uint32_t n) { return (n + kChunk - 1) / kChunk; }

hipError_t launch_group_build(const int32_t *row_ptr, const int32_t *col_idx, const double *w,
                              uint32_t n, double alpha, double *A, hipStream_t stream) {
    const uint32_t N = group_dim(n);
    hipError_t e = hipMemsetAsync(A, 0, sizeof(double) * N * N, stream);
    if (e != hipSuccess) return e;
    dense_build_kernel<<<blocks_for(N), kThreads, 0, stream>>>(row_ptr, col_idx, w, n, N, alpha, A);
    return hipGetLastError();
}

namespace {

// In-place Gauss-Jordan inverse with 64-wide pivot blocks (N a multiple of 64).
void invert_64(double *A, uint32_t N, double *Dinv, hipStream_t stream) {
    const uint32_t nt = N / kT;
    for (uint32_t pt = 0; pt < nt; ++pt) {
        gj_pivot_kernel<<<1, kThreads, 0, stream>>>(A, N, pt * kT, Dinv);
        gj_panel_kernel<<<nt, kThreads, 0, stream>>>(A, N, pt, Dinv, 0u);
        gj_update_kernel<<<dim3(nt, nt), kThreads, 0, stream>>>(A, N, pt);
        gj_panel_kernel<<<nt, kThreads, 0, stream>>>(A, N, pt, Dinv, 1u);
        gj_put_kernel<<<1, kThreads, 0, stream>>>(A, N, pt, Dinv);
    }
}

}  // namespace

// Outer Gauss-Jordan over 256-wide pivot blocks P (rows and columns [p0, p0 + 256)):
//   W = A[P, P]^{-1}                    (copy, then invert_64 on the 256 x 256 copy)
//   R = W A[P, :]                       (row panel, out of place: 256 x N)
//   A[i, j] -= A[i, P] R[:, j]          (i, j outside P; A[i, P] still the old panel)
//   C = -A[:, P] W                      (column panel, out of place: N x 256)
//   A[P, :] = R, A[:, P] = C, A[P, P] = W
// Scratch: W (256 x 256), R (256 x N), C (N x 256), then a 64 x 64 block.
hipError_t launch_group_invert(double *A, uint32_t N, double *scratch, hipStream_t stream) {
    double *W = scratch, *R = W + kB * kB, *C = R + static_cast<size_t>(kB) * N;
    double *D64 = C + static_cast<size_t>(N) * kB;
    const uint32_t nt = N / kT, pb = kB / kT;
    for (uint32_t p0 = 0; p0 < N; p0 += kB) {
        const uint32_t pt0 = p0 / kT, pt1 = pt0 + pb;
        copy_block_kernel<<<dim3(1, kB), kThreads, 0, stream>>>(A + static_cast<size_t>(p0) * N + p0, N,
                                                                W, kB, kB);
        invert_64(W, kB, D64, stream);
        GemmArgs row{W, A + static_cast<size_t>(p0) * N, R, kB, N, N, kB / kK, 0u, 0u, pt0, pt1, 0u, 0u};
        gemm_kernel<<<dim3(nt, pb), kThreads, 0, stream>>>(row);
        GemmArgs upd{A + p0, R, A, N, N, N, kB / kK, pt0, pt1, pt0, pt1, 1u, 1u};
        gemm_kernel<<<dim3(nt, nt), kThreads, 0, stream>>>(upd);
        GemmArgs col{A + p0, W, C, N, kB, kB, kB / kK, pt0, pt1, 0u, 0u, 0u, 1u};
        gemm_kernel<<<dim3(pb, nt), kThreads, 0, stream>>>(col);
        // write back: rows of P from R (outside P's columns), columns of P from C
        // (outside P's rows), and W on the diagonal block
        if (p0 > 0)
            copy_block_kernel<<<dim3(4, kB), kThreads, 0, stream>>>(R, N, A + static_cast<size_t>(p0) * N,
                                                                    N, p0);
        if (p0 + kB < N)
            copy_block_kernel<<<dim3(4, kB), kThreads, 0, stream>>>(
                R + p0 + kB, N, A + static_cast<size_t>(p0) * N + p0 + kB, N, N - p0 - kB);
        if (p0 > 0)
            copy_block_kernel<<<dim3(1, p0), kThreads, 0, stream>>>(C, kB, A + p0, N, kB);
        if (p0 + kB < N)
            copy_block_kernel<<<dim3(1, N - p0 - kB), kThreads, 0, stream>>>(
                C + static_cast<size_t>(p0 + kB) * kB, kB, A + static_cast<size_t>(p0 + kB) * N + p0, N,
                kB);
        copy_block_kernel<<<dim3(1, kB), kThreads, 0, stream>>>(W, kB, A + static_cast<size_t>(p0) * N + p0,
                                                                N, kB);
    }
    return hipGetLastError();
}

hipError_t launch_group_first(const double *A, uint32_t n, uint32_t N, double *diag,
                              unsigned long long *sel, hipStream_t stream) {
    diag_kernel<<<blocks_for(n), kThreads, 0, stream>>>(A, n, N, diag);
    argmin_bits_kernel<<<blocks_for(n), kThreads, 0, stream>>>(diag, n, sel);
    argmin_id_kernel<<<blocks_for(n), kThreads, 0, stream>>>(diag, n, sel);
    return hipGetLastError();
}

hipError_t launch_group_reground(double *A, uint32_t n, uint32_t N, uint32_t v0, double *c,
                                 hipStream_t stream) {
    copy_col_kernel<<<blocks_for(n), kThreads, 0, stream>>>(A, n, N, v0, nullptr, c, nullptr);
    reground_kernel<<<dim3(blocks_for(n), n), kThreads, 0, stream>>>(A, n, N, v0, c);
    return hipGetLastError();
}

hipError_t launch_group_trace(const double *A, uint32_t n, uint32_t N, uint32_t v, double *out,
                              double *piv, hipStream_t stream) {
    trace_kernel<<<1, kThreads, 0, stream>>>(A, n, N, v, out, piv);
    return hipGetLastError();
}

hipError_t launch_group_colsq(double *A, uint32_t n, uint32_t N, uint32_t v, double *cv, double *rv,
                              const double *piv, double *part, hipStream_t stream) {
    const bool down = v < n;
    if (down) copy_col_kernel<<<blocks_for(n), kThreads, 0, stream>>>(A, n, N, v, nullptr, cv, rv);
    colsq_kernel<<<dim3(blocks_for(n), group_chunks(n)), kThreads, 0, stream>>>(
        A, n, N, v, nullptr, down ? cv : nullptr, down ? rv : nullptr, piv, part);
    return hipGetLastError();
}

hipError_t launch_group_step(double *A, uint32_t n, uint32_t N, double *part, uint8_t *taken,
                             unsigned long long *bmax, uint32_t *bid, double *bdiag,
                             unsigned long long *vsel, double *cv, double *rv, double *piv,
                             int32_t *gout, double *fout, uint32_t s, uint32_t *bad,
                             hipStream_t stream) {
    const uint32_t nb = blocks_for(n);
    gain_kernel<<<nb, kThreads, 0, stream>>>(A, n, N, group_chunks(n), part, taken, bmax, bid,
                                             bdiag, bad);
    choose_copy_kernel<<<nb, kThreads, 0, stream>>>(A, n, N, bmax, bid, bdiag, nb, taken, gout, s,
                                                    piv, vsel, bad, fout, cv, rv);
    colsq_kernel<<<dim3(nb, group_chunks(n)), kThreads, 0, stream>>>(A, n, N, n, vsel, cv, rv, piv,
                                                                    part);
    return hipGetLastError();
}

}  // namespace fc
