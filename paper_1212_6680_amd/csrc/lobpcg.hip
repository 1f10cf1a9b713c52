// LOBPCG (Section 4) on gfx950 with the SMG V-cycle as preconditioner.
//
// The locally optimal block preconditioned conjugate gradient method
// (Knyazev 2001) for the m smallest eigenpairs.  Per iteration:
//   R = A X - X diag(theta); active columns J have relative residual > rtol;
//   W = T R_J (one batched SMG V-cycle over |J| right-hand sides);
//   S = [X, W, P_J] with W and P columns scaled to unit length;
//   S, A S <- Cholesky QR, twice (drop P, then fall back to an eigen-based
//   orthonormalisation of S^T S when the Gram matrix is numerically singular);
//   Rayleigh-Ritz on S^T A S; X = S C_m, P = S_{W,P} C_{W,P; m}.
// The only dense contractions are the tall-skinny Gram products S^T Y and
// the block updates S C, which run on FP64 MFMA (v_mfma_f64_16x16x4f64);
// the k x k (k <= 3m) Cholesky and eigen-decompositions run on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "dense_host.hpp"
#include "smg_internal.h"

using namespace smg;

typedef double v4d __attribute__((ext_vector_type(4)));

namespace {

constexpr int kT = 64;      // output tile edge of the MFMA kernels
constexpr int kNarrow = 8;  // bases of at most this many columns use the streaming kernels
constexpr int kK = 16;      // reduction slice staged in LDS per step
constexpr int kLdsPad = 4;  // LDS row padding (doubles)

// Partial Gram products over a slice of rows:
//   part[z][i][j] = sum_{n in slice z} U[n + i*ldu] * V[n + j*ldv],  i < p, j < q.
// Block: 4 waves; tile 128(i) x 128(j); wave w owns rows i in [32w, 32w+32)
// (two 16-row MFMA blocks) and all 128 columns (eight 16-column blocks), so
// each step of 4 in n costs 10 LDS reads for 16 MFMAs.
// MFMA 16x16x4 f64 operand layout: A[i][k] from lane i + 16k, B[k][j] from
// lane j + 16k, D[i][j] in lane j + 16*(i%4), element i/4.
constexpr int kGT = 128;    // Gram output tile edge

// Gram slices (blocks along N per output tile): about 1024 blocks in all,
// two rounds of two resident blocks per CU
inline int gram_slices(int tiles) { return std::max(1, 1024 / std::max(1, tiles)); }

__global__ __launch_bounds__(256) void k_gram_partial(const double *U, long long ldu, int p, const double *V,
                                                      long long ldv, int q, long long n, long long slice,
                                                      double *part, int sym)
{
    // sym: the product is symmetric (p == q); tiles below the diagonal are
    // left out and read mirrored by the reduction
    if (sym && blockIdx.x > blockIdx.y) return;
    constexpr int TILE = kGT;
    constexpr int RB = TILE / 64;      // 16-row MFMA blocks per wave (4 waves)
    constexpr int CB = TILE / 16;      // 16-column MFMA blocks
    constexpr int R = TILE / 16;       // values per thread per slice and operand
    // two LDS stages: the next slice is read into registers while the MFMAs
    // run on this one, then stored into the other stage (one barrier a slice)
    __shared__ double Us[2][kK][TILE + kLdsPad];
    __shared__ double Vs[2][kK][TILE + kLdsPad];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int i0 = blockIdx.x * TILE, j0 = blockIdx.y * TILE;
    const long long n_beg = static_cast<long long>(blockIdx.z) * slice;
    const long long n_end = n_beg + slice < n ? n_beg + slice : n;
    v4d acc[RB][CB];
#pragma unroll
    for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < CB; ++b) acc[a][b] = v4d{0, 0, 0, 0};
    // 16 x 16 blocks inside p x q only (the tile is padded)
    bool in[RB];
#pragma unroll
    for (int a = 0; a < RB; ++a) in[a] = i0 + 16 * (RB * w + a) < p;
    const int jn = (q - j0 + 15) / 16;
    // thread e of a slice holds row e % 16 of tile column e / 16
    double ru[R], rv[R];
    auto fetch = [&](long long n0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + 256 * r;
            const int ii = e & 15, col = e >> 4;
            const long long nn = n0 + ii;
            const bool inn = nn < n_end;
            ru[r] = (inn && i0 + col < p) ? U[nn + (i0 + col) * ldu] : 0.0;
            rv[r] = (inn && j0 + col < q) ? V[nn + (j0 + col) * ldv] : 0.0;
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + 256 * r;
            Us[st][e & 15][e >> 4] = ru[r];
            Vs[st][e & 15][e >> 4] = rv[r];
        }
    };
    if (n_beg < n_end) {
        fetch(n_beg);
        stash(0);
    }
    __syncthreads();
    int st = 0;
    for (long long n0 = n_beg; n0 < n_end; n0 += kK) {
        const bool more = n0 + kK < n_end;
        if (more) fetch(n0 + kK);
#pragma unroll
        for (int kk = 0; kk < kK / 4; ++kk) {
            const int kr = 4 * kk + (lane >> 4);
            double a[RB];
#pragma unroll
            for (int ra = 0; ra < RB; ++ra) a[ra] = Us[st][kr][16 * (RB * w + ra) + (lane & 15)];
#pragma unroll
            for (int jt = 0; jt < CB; ++jt) {
                if (jt >= jn) break;            // 16-column blocks past q
                const double b = Vs[st][kr][16 * jt + (lane & 15)];
#pragma unroll
                for (int ra = 0; ra < RB; ++ra)
                    if (in[ra]) acc[ra][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ra], b, acc[ra][jt], 0, 0, 0);
            }
        }
        // the other stage was last read before the previous barrier
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
    double *out = part + static_cast<long long>(blockIdx.z) * p * q;
#pragma unroll
    for (int ra = 0; ra < RB; ++ra)
#pragma unroll
        for (int jt = 0; jt < CB; ++jt) {
            const int j = j0 + 16 * jt + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = i0 + 16 * (RB * w + ra) + 4 * r + (lane >> 4);
                if (i < p && j < q) out[static_cast<long long>(i) * q + j] = acc[ra][jt][r];
            }
        }
}

// Symmetric Gram products of narrow blocks (k <= kTriMax) without tiles: each
// block takes a slice of rows and ALL 16 x 16 output blocks on or above the
// diagonal (nb (nb + 1) / 2 of them, nb = ceil(k / 16)), dealt round-robin to
// its 8 waves, so every block does the same work and no MFMA is spent on
// padding beyond the last 16-block.  Slices of 16 rows (of both operands when
// U != V) are staged in two LDS stages with the next slice read into
// registers meanwhile.  Writes part[z][i][j] for the upper
// blocks only (the reduction mirrors).  An instance takes k <= 16 NB: its
// accumulators and LDS scale with NB, so narrow products run more blocks per CU.
constexpr int kTriMax = 224;                  // 14 blocks of 16
constexpr int kTriWaves = 8;                  // waves per block (two per SIMD)

template <bool SAME, int NB>
__global__ __launch_bounds__(64 * kTriWaves) void k_gram_tri(const double *U, const double *V, long long ld, int k, long long n,
                                                  long long slice, double *part)
{
    constexpr int KS = 16;                               // rows per stage
    constexpr int NT = 64 * kTriWaves;
    constexpr int TM = 16 * NB;                          // widest k of this instance
    constexpr int PW = (NB * (NB + 1) / 2 + kTriWaves - 1) / kTriWaves;   // output blocks per wave
    constexpr int R = (KS * TM + NT - 1) / NT;           // staged values per thread and operand
    // stages: U in Ls[0], Ls[1]; V (when it differs) in Ls[2], Ls[3]
    __shared__ double Ls[SAME ? 2 : 4][KS][TM + kLdsPad];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int nb = (k + 15) / 16, T = nb * (nb + 1) / 2;
    const long long n_beg = static_cast<long long>(blockIdx.x) * slice;
    const long long n_end = n_beg + slice < n ? n_beg + slice : n;
    // this wave's output blocks: t = w, w + 8, ... in row-major order of the
    // upper triangle (uniform values)
    int bi[PW], bj[PW];
#pragma unroll
    for (int b = 0; b < PW; ++b) {
        const int t = w + kTriWaves * b;
        int i = 0, rem = t;
        while (i < nb && rem >= nb - i) {
            rem -= nb - i;
            ++i;
        }
        bi[b] = t < T ? i : -1;
        bj[b] = t < T ? i + rem : -1;
    }
    v4d acc[PW];
#pragma unroll
    for (int b = 0; b < PW; ++b) acc[b] = v4d{0, 0, 0, 0};
    const int kp = nb * 16;   // staged columns (zero past k)
    double ru[R], rv[SAME ? 1 : R];
    auto fetch = [&](long long n0) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + NT * r;
            const int ii = e % KS, col = e / KS;
            const long long nn = n0 + ii;
            const bool in = col < k && nn < n_end;
            ru[r] = in ? U[nn + col * ld] : 0.0;
            if constexpr (!SAME) rv[r] = in ? V[nn + col * ld] : 0.0;
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int e = tid + NT * r;
            const int ii = e % KS, col = e / KS;
            if (col < kp) {
                Ls[st][ii][col] = ru[r];
                if constexpr (!SAME) Ls[2 + st][ii][col] = rv[r];
            }
        }
    };
    if (n_beg < n_end) {
        fetch(n_beg);
        stash(0);
    }
    __syncthreads();
    int st = 0;
    for (long long n0 = n_beg; n0 < n_end; n0 += KS) {
        const bool more = n0 + KS < n_end;
        if (more) fetch(n0 + KS);
        const double(*Ua)[TM + kLdsPad] = Ls[st];
        const double(*Vb)[TM + kLdsPad] = Ls[SAME ? st : 2 + st];
#pragma unroll
        for (int kk = 0; kk < KS / 4; ++kk) {
            const int kr = 4 * kk + (lane >> 4);
#pragma unroll
            for (int b = 0; b < PW; ++b) {
                if (bi[b] < 0) break;
                const double a = Ua[kr][16 * bi[b] + (lane & 15)];
                const double v = Vb[kr][16 * bj[b] + (lane & 15)];
                acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, v, acc[b], 0, 0, 0);
            }
        }
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
    double *out = part + static_cast<long long>(blockIdx.x) * k * k;
#pragma unroll
    for (int b = 0; b < PW; ++b) {
        if (bi[b] < 0) break;
        const int j = 16 * bj[b] + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * bi[b] + 4 * r + (lane >> 4);
            if (i < k && j < k) out[static_cast<long long>(i) * k + j] = acc[b][r];
        }
    }
}

// G[i][j] = sum_z part[z][i][j] in a fixed order (deterministic); with sym,
// entries of tiles below the diagonal come from the mirrored entry.  A block
// takes 64 entries; its 4 waves sum the slices z = w, w + 4, ... and wave 0
// adds the four sums in order.
constexpr int kRedGroups = 4;

__global__ __launch_bounds__(64 * kRedGroups) void k_gram_reduce(const double *part, int nz, int p, int q, int tile,
                                                                 int sym, double *G)
{
    __shared__ double sums[kRedGroups][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + lane;
    double s = 0.0;
    if (e < p * q) {
        const int i = e / q, j = e % q;
        const int src = sym && i / tile > j / tile ? j * q + i : e;
        for (int z = w; z < nz; z += kRedGroups) s += part[static_cast<long long>(z) * p * q + src];
    }
    sums[w][lane] = s;
    __syncthreads();
    if (w == 0 && e < p * q) {
        double t = sums[0][lane];
#pragma unroll
        for (int g = 1; g < kRedGroups; ++g) t += sums[g][lane];
        G[e] = t;
    }
}

// Y[n + j*ldy] = sum_{i<k} U[n + i*ldu] * C[i*mo + j]  for j < mo (C row-major k x mo).
// Computed as the transposed tile Y^T = C^T U^T so that each MFMA output row
// is a contiguous run of 16 n: wave w owns n in [16w, 16w+16) of the tile;
// 16-column blocks past mo are skipped.
__global__ __launch_bounds__(256) void k_block_update(const double *U, long long ldu, int k, const double *C, int mo,
                                                      double *Y, long long ldy, long long n, double *Y2, int jsplit)
{
    // two LDS stages: the next 16 rows of C and U are read into registers
    // while the MFMAs run on these (one barrier per step)
    __shared__ double Ut[2][kK][kT + kLdsPad];
    __shared__ double Ct[2][kK][kT + kLdsPad];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long long n0 = static_cast<long long>(blockIdx.x) * kT;
    const int j0 = blockIdx.y * kT;
    const int jn = (mo - j0 + 15) / 16;
    v4d acc[4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    // U[n0 .. n0+63][i0 .. i0+15] as Ut[i][n] and C[i0..][j0..j0+63] as Ct[i][j]
    double ru[4], rc[4];
    auto fetch = [&](int i0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;         // 0 .. 1023
            const int ii = e >> 6, nn = e & 63;  // 16 x 64
            const long long ng = n0 + nn;
            ru[r] = (i0 + ii < k && ng < n) ? U[ng + (i0 + ii) * ldu] : 0.0;
            rc[r] = (i0 + ii < k && j0 + nn < mo) ? C[static_cast<long long>(i0 + ii) * mo + j0 + nn] : 0.0;
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            Ut[st][e >> 6][e & 63] = ru[r];
            Ct[st][e >> 6][e & 63] = rc[r];
        }
    };
    fetch(0);
    stash(0);
    __syncthreads();
    int st = 0;
    for (int i0 = 0; i0 < k; i0 += kK) {
        const bool more = i0 + kK < k;
        if (more) fetch(i0 + kK);
#pragma unroll
        for (int kk = 0; kk < kK / 4; ++kk) {
            const int kr = 4 * kk + (lane >> 4);
            const double b = Ut[st][kr][16 * w + (lane & 15)];
#pragma unroll
            for (int jt = 0; jt < 4; ++jt) {
                if (jt >= jn) break;
                const double a = Ct[st][kr][16 * jt + (lane & 15)];
                acc[jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[jt], 0, 0, 0);
            }
        }
        // the other stage was last read before the previous barrier
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
    const long long nn = n0 + 16 * w + (lane & 15);
    if (nn >= n) return;
#pragma unroll
    for (int jt = 0; jt < 4; ++jt) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = j0 + 16 * jt + 4 * r + (lane >> 4);
            if (j < mo) (j < jsplit ? Y + j * ldy : Y2 + (j - jsplit) * ldy)[nn] = acc[jt][r];
        }
    }
}

// Y (N x mo) = U (N x k) C (k x mo) for mo <= 16 JB with every output
// column in one block: a block owns 64 rows (wave w: rows 16w .. 16w + 15)
// and all ceil(mo/16) 16-column blocks, so U is read once (the 64-column
// tiles of k_block_update read it once per tile) and C comes from cache.
// Same transposed MFMA form (Y^T = C^T U^T) and two LDS stages with the next
// 16 rows of C and U read into registers meanwhile. Rows of C that are zero
// for a whole 16-column block (a triangular factor, a coefficient block with
// zeroed rows) are skipped: column block jt only takes the 16-row stages that
// meet [lo[jt], hi[jt]), and the stage loop runs over their union.
struct RowSpan {
    int lo[kTriMax / 16];
    int hi[kTriMax / 16];
};

// RG: 16-row groups per wave; a block owns 64 RG rows, so each staged slice of
// C serves RG times as many rows.
template <int JB, int RG = 1>
__global__ __launch_bounds__(256, 2) void k_block_update_wide(
    const double *U, long long ldu, int i_begin, int i_end,
                                                           const double *C, int mo, RowSpan span, double *Y,
                                                           long long ldy, long long n, double *Y2, int jsplit)
{
    constexpr int W = 16 * JB;
    constexpr int RC = (kK * W + 255) / 256;     // C values per thread and stage
    __shared__ double Ct[2][kK][W + kLdsPad];
    constexpr int TR = kT * RG;                  // rows per block
    __shared__ double Ut[2][kK][TR + kLdsPad];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const long long n0 = static_cast<long long>(blockIdx.x) * TR;
    const int jn = (mo + 15) / 16;
    const int mp = jn * 16;
    v4d acc[RG][JB];
#pragma unroll
    for (int g = 0; g < RG; ++g)
#pragma unroll
        for (int jt = 0; jt < JB; ++jt) acc[g][jt] = v4d{0, 0, 0, 0};
    double ru[4 * RG], rc[RC];
    auto fetch = [&](int i0) {
#pragma unroll
        for (int r = 0; r < 4 * RG; ++r) {
            const int e = tid + 256 * r;          // 16 x TR
            const int ii = e / TR, nn = e % TR;
            const long long ng = n0 + nn;
            ru[r] = (i0 + ii < i_end && ng < n) ? U[ng + (i0 + ii) * ldu] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int e = tid + 256 * r;          // 16 x W
            const int ii = e / W, jj = e % W;
            rc[r] = (ii < kK && i0 + ii < i_end && jj < mo) ? C[static_cast<long long>(i0 + ii) * mo + jj] : 0.0;
        }
    };
    auto stash = [&](int st) {
#pragma unroll
        for (int r = 0; r < 4 * RG; ++r) {
            const int e = tid + 256 * r;
            Ut[st][e / TR][e % TR] = ru[r];
        }
#pragma unroll
        for (int r = 0; r < RC; ++r) {
            const int e = tid + 256 * r;
            const int ii = e / W, jj = e % W;
            if (ii < kK && jj < mp) Ct[st][ii][jj] = rc[r];
        }
    };
    fetch(i_begin);
    stash(0);
    __syncthreads();
    int st = 0;
    for (int i0 = i_begin; i0 < i_end; i0 += kK) {
        const bool more = i0 + kK < i_end;
        if (more) fetch(i0 + kK);
#pragma unroll
        for (int kk = 0; kk < kK / 4; ++kk) {
            const int kr = 4 * kk + (lane >> 4);
            double b[RG];
#pragma unroll
            for (int g = 0; g < RG; ++g) b[g] = Ut[st][kr][kT * g + 16 * w + (lane & 15)];
#pragma unroll
            for (int jt = 0; jt < JB; ++jt) {
                if (jt < jn && i0 < span.hi[jt] && i0 + kK > span.lo[jt]) {
                    const double a = Ct[st][kr][16 * jt + (lane & 15)];
#pragma unroll
                    for (int g = 0; g < RG; ++g)
                        acc[g][jt] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[g], acc[g][jt], 0, 0, 0);
                }
            }
        }
        if (more) stash(st ^ 1);
        __syncthreads();
        st ^= 1;
    }
#pragma unroll
    for (int g = 0; g < RG; ++g) {
        const long long nn = n0 + kT * g + 16 * w + (lane & 15);
        if (nn >= n) continue;
#pragma unroll
        for (int jt = 0; jt < JB; ++jt) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * jt + 4 * r + (lane >> 4);
                if (j < mo) (j < jsplit ? Y + j * ldy : Y2 + (j - jsplit) * ldy)[nn] = acc[g][jt][r];
            }
        }
    }
}

// Narrow bases (k <= K <= 8 columns: LOBPCG with m <= 2).  A product over a
// few columns moves 8 N k bytes per operand and does ~k flops per byte read,
// far from the matrix cores' regime: plain streaming kernels whose threads
// keep every column of a row in registers run at the memory's pace, where the
// 16-column MFMA tiles would spend most of their work on padding.
//
// part[z][i][j] = sum over rows of slice z of U[n, i] V[n, j], i, j < k (with
// SYM, V = U and the lower triangle mirrored); fixed slices and a fixed
// reduction order, like the tiled Gram kernels.
template <int K, bool SYM>
__global__ __launch_bounds__(256) void k_gram_narrow(const double *U, const double *V, long long ld, int k, long long n,
                                                     long long slice, double *part)
{
    __shared__ double sums[4][K * K];
    const int z = blockIdx.x, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long beg = static_cast<long long>(z) * slice;
    const long long end = beg + slice < n ? beg + slice : n;
    double acc[K][K];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) acc[i][j] = 0.0;
    for (long long e = beg + threadIdx.x; e < end; e += blockDim.x) {
        double u[K], v[K];
#pragma unroll
        for (int i = 0; i < K; ++i) {
            u[i] = i < k ? U[e + i * ld] : 0.0;
            if (!SYM) v[i] = i < k ? V[e + i * ld] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < K; ++i)
#pragma unroll
            for (int j = 0; j < K; ++j)
                if (!SYM || j >= i) acc[i][j] += u[i] * (SYM ? u[j] : v[j]);
    }
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (SYM && j < i) continue;
            double t = acc[i][j];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
            if (lane == 0) sums[w][i * K + j] = t;
        }
    __syncthreads();
    for (int t = threadIdx.x; t < k * k; t += blockDim.x) {
        const int i = t / k, j = t % k;
        const int src = SYM && j < i ? j * K + i : i * K + j;
        part[static_cast<long long>(z) * k * k + t] = ((sums[0][src] + sums[1][src]) + sums[2][src]) + sums[3][src];
    }
}

// Y[:, j] = sum_{i<k} U[:, i] C[i][j] for j < mo (C row-major k x mo, k <= K,
// mo <= 16); columns from jsplit on go to Y2 (column jsplit + c to Y2[:, c]).
template <int K>
__global__ __launch_bounds__(256) void k_update_narrow(const double *U, long long ld, int k, const double *C, int mo,
                                                       double *Y, double *Y2, int jsplit, long long n)
{
    __shared__ double Cs[K * 16];
    for (int t = threadIdx.x; t < k * mo; t += blockDim.x) Cs[(t / mo) * 16 + t % mo] = C[t];
    __syncthreads();
    for (long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; e < n;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        double u[K];
#pragma unroll
        for (int i = 0; i < K; ++i) u[i] = i < k ? U[e + i * ld] : 0.0;
        for (int j = 0; j < mo; ++j) {
            double y = 0.0;
#pragma unroll
            for (int i = 0; i < K; ++i)
                if (i < k) y += u[i] * Cs[i * 16 + j];
            (j < jsplit ? Y + j * ld : Y2 + (j - jsplit) * ld)[e] = y;
        }
    }
}

// part[c][z] = sum over slice z of U[:, c] .* V[:, c]
__global__ __launch_bounds__(256) void k_coldot_partial(const double *U, const double *V, long long ld, long long n,
                                                        long long slice, double *part, int nslices)
{
    __shared__ double lds[4];
    const int c = blockIdx.y, z = blockIdx.x;
    const long long beg = static_cast<long long>(z) * slice;
    const long long end = beg + slice < n ? beg + slice : n;
    double s = 0.0;
    for (long long e = beg + threadIdx.x; e < end; e += blockDim.x) s += U[e + c * ld] * V[e + c * ld];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[c * nslices + z] = lds[0] + lds[1] + lds[2] + lds[3];
}

// R = AX - X diag(theta) with the column sums of R^2 and X^2 in one pass
// (the slicing and summation order of k_coldot_partial): part[c][z] for R,
// part[m + c][z] for X.
__global__ __launch_bounds__(256) void k_block_resid_dots(const double *AX, const double *X, const double *theta,
                                                          double *R, long long ld, long long n, long long slice,
                                                          double *part, int nslices, int m)
{
    __shared__ double lds[2][4];
    const int c = blockIdx.y, z = blockIdx.x;
    const long long beg = static_cast<long long>(z) * slice;
    const long long end = beg + slice < n ? beg + slice : n;
    const double th = theta[c];
    double sr = 0.0, sx = 0.0;
    for (long long e = beg + threadIdx.x; e < end; e += blockDim.x) {
        const double xv = X[e + c * ld];
        const double rv = AX[e + c * ld] - th * xv;
        R[e + c * ld] = rv;
        sr += rv * rv;
        sx += xv * xv;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_down(sr, off, 64);
        sx += __shfl_down(sx, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = sr;
        lds[1][threadIdx.x >> 6] = sx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        part[c * nslices + z] = lds[0][0] + lds[0][1] + lds[0][2] + lds[0][3];
        part[(m + c) * nslices + z] = lds[1][0] + lds[1][1] + lds[1][2] + lds[1][3];
    }
}

// out[c] = sum_z part[c][z]: one block per column, its threads summing the
// slices z = t, t + 256, ... and the block combining them in a fixed order
__global__ __launch_bounds__(256) void k_coldot_reduce(const double *part, int nslices, double *out)
{
    __shared__ double lds[4];
    const int c = blockIdx.x;
    double s = 0.0;
    for (int z = threadIdx.x; z < nslices; z += blockDim.x) s += part[static_cast<long long>(c) * nslices + z];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) out[c] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// G[e] = sum_z part[z][e] for a small product (the narrow bases): one block
// per entry, reduced like k_coldot_reduce
__global__ __launch_bounds__(256) void k_gram_reduce_narrow(const double *part, int nz, int pq, double *G)
{
    __shared__ double lds[4];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int z = threadIdx.x; z < nz; z += blockDim.x) s += part[static_cast<long long>(z) * pq + e];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) G[e] = ((lds[0] + lds[1]) + lds[2]) + lds[3];
}

// X[:, c] *= 1/sqrt(nrm2[c]) (and the same for AX when given)
__global__ void k_scale_cols(double *X, double *AX, const double *nrm2, long long ld, long long n, int m)
{
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= n || c >= m) return;
    const double f = 1.0 / sqrt(nrm2[c]);
    X[e + c * ld] *= f;
    if (AX) AX[e + c * ld] *= f;
}

// dst[:, c] = src[:, idx[c]]
// dst[:, c] = src[:, idx[c]] (times scale[c] when scale is given)
__global__ void k_gather_cols(const double *src, double *dst, const int *idx, const double *scale, long long ld,
                              long long n, int m)
{
    const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (e >= n || c >= m) return;
    const double v = src[e + static_cast<long long>(idx[c]) * ld];
    dst[e + c * ld] = scale ? scale[c] * v : v;
}

inline unsigned nblk(long long n, int bs) { return static_cast<unsigned>((n + bs - 1) / bs); }

struct LobLayout {
    size_t S, AS, T, AT, P, AP, R, part, G, C, theta, cpart, cout, idx, gscale, total;
    int nslices_gram, nslices_col;
};

size_t al(size_t v) { return (v + 255) / 256 * 256; }

LobLayout lob_layout(size_t N, int m)
{
    LobLayout L{};
    const size_t k3 = 3 * static_cast<size_t>(m);
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t r = off;
        off = al(off + b);
        return r;
    };
    L.S = take(N * k3 * 8);
    L.AS = take(N * k3 * 8);
    L.T = take(N * k3 * 8);
    L.AT = take(N * k3 * 8);
    L.P = take(N * m * 8);
    L.AP = take(N * m * 8);
    L.R = take(N * m * 8);
    // enough partial products for any product taken (one output tile at least)
    long long ns = gram_slices(1);
    const long long maxs = static_cast<long long>((N + 1023) / 1024);
    if (ns > maxs) ns = maxs < 1 ? 1 : maxs;
    L.nslices_gram = static_cast<int>(ns);
    L.part = take(static_cast<size_t>(ns) * k3 * k3 * 8);
    L.G = take(k3 * k3 * 8);
    L.C = take(k3 * 2 * m * 8 + k3 * k3 * 8);
    L.theta = take(k3 * 8);
    // column passes: enough slices to fill the chip when the block is narrow
    L.nslices_col = static_cast<int>(
        std::min<long long>(std::max<long long>(256, 2048 / m), static_cast<long long>((N + 4095) / 4096)));
    if (L.nslices_col < 1) L.nslices_col = 1;
    L.cpart = take(k3 * L.nslices_col * 8 * 2);
    L.cout = take(k3 * 8 * 2);
    L.idx = take(k3 * 4);
    L.gscale = take(k3 * 8);
    L.total = off;
    return L;
}

struct Lob {
    smg_handle *h;
    hipStream_t st;
    size_t N;
    int m;
    char *ws;
    LobLayout L;
    template <typename X> X *at(size_t off) const { return reinterpret_cast<X *>(ws + off); }

    bool ok() { return hipGetLastError() == hipSuccess; }

    // device G (p x q row-major) = U^T V; sym: the product is symmetric (p == q)
    void gram_launch(const double *U, int p, const double *V, int q, bool sym)
    {
        const int s = sym && p == q ? 1 : 0;
        if (s && p <= kNarrow) {   // a few columns: streaming kernel
            const long long ln = static_cast<long long>(N);
            const long long want = std::min<long long>(1024, L.nslices_gram);
            const long long sl = (ln + want - 1) / want;
            const int nz = static_cast<int>((ln + sl - 1) / sl);
            double *pt = at<double>(L.part);
            if (U == V) {
                if (p <= 4)
                    hipLaunchKernelGGL((k_gram_narrow<4, true>), dim3(nz), dim3(256), 0, st, U, V, ln, p, ln, sl, pt);
                else
                    hipLaunchKernelGGL((k_gram_narrow<kNarrow, true>), dim3(nz), dim3(256), 0, st, U, V, ln, p, ln, sl,
                                       pt);
            } else {
                if (p <= 4)
                    hipLaunchKernelGGL((k_gram_narrow<4, false>), dim3(nz), dim3(256), 0, st, U, V, ln, p, ln, sl,
                                       pt);
                else
                    hipLaunchKernelGGL((k_gram_narrow<kNarrow, false>), dim3(nz), dim3(256), 0, st, U, V, ln, p, ln,
                                       sl, pt);
            }
            hipLaunchKernelGGL(k_gram_reduce_narrow, dim3(p * q), dim3(256), 0, st, pt, nz, p * q, at<double>(L.G));
            return;
        }
        if (s && p <= kTriMax) {   // narrow: all upper 16-blocks per block, slices of N
            // one block per CU for the widest instance; the narrower ones fit
            // two and four per CU
            const int nbk = (p + 15) / 16;
            const long long want = std::min<long long>(nbk <= 4 ? 1024 : nbk <= 8 ? 512 : 256, L.nslices_gram);
            const long long slice = (static_cast<long long>(N) + want - 1) / want;
            const long long sl = (slice + 15) / 16 * 16;
            const int nz = static_cast<int>((static_cast<long long>(N) + sl - 1) / sl);
            // instances by the widest k they take (registers and LDS scale with it)
            const long long ln = static_cast<long long>(N);
            double *pt = at<double>(L.part);
            const dim3 g(nz), b(64 * kTriWaves);
            if (U == V) {
                if (nbk <= 4)
                    hipLaunchKernelGGL((k_gram_tri<true, 4>), g, b, 0, st, U, V, ln, p, ln, sl, pt);
                else if (nbk <= 8)
                    hipLaunchKernelGGL((k_gram_tri<true, 8>), g, b, 0, st, U, V, ln, p, ln, sl, pt);
                else
                    hipLaunchKernelGGL((k_gram_tri<true, kTriMax / 16>), g, b, 0, st, U, V, ln, p, ln, sl, pt);
            } else {
                if (nbk <= 4)
                    hipLaunchKernelGGL((k_gram_tri<false, 4>), g, b, 0, st, U, V, ln, p, ln, sl, pt);
                else if (nbk <= 8)
                    hipLaunchKernelGGL((k_gram_tri<false, 8>), g, b, 0, st, U, V, ln, p, ln, sl, pt);
                else
                    hipLaunchKernelGGL((k_gram_tri<false, kTriMax / 16>), g, b, 0, st, U, V, ln, p, ln, sl, pt);
            }
            hipLaunchKernelGGL(k_gram_reduce, dim3(nblk(static_cast<long long>(p) * q, 64)), dim3(64 * kRedGroups), 0, st,
                               at<double>(L.part), nz, p, q, 16, 1, at<double>(L.G));
            return;
        }
        const int tp = nblk(p, kGT), tq = nblk(q, kGT);
        // slices by the full tile grid: the diagonal tiles bound the time, and
        // more, shorter slices only add partial products
        const long long want = std::min<long long>(gram_slices(tp * tq), L.nslices_gram);
        const long long slice = (static_cast<long long>(N) + want - 1) / want;
        const long long sl = (slice + kK - 1) / kK * kK;
        const int nz = static_cast<int>((static_cast<long long>(N) + sl - 1) / sl);
        hipLaunchKernelGGL(k_gram_partial, dim3(tp, tq, nz), dim3(256), 0, st, U, static_cast<long long>(N), p, V,
                           static_cast<long long>(N), q, static_cast<long long>(N), sl, at<double>(L.part), s);
        hipLaunchKernelGGL(k_gram_reduce, dim3(nblk(static_cast<long long>(p) * q, 64)), dim3(64 * kRedGroups), 0, st,
                           at<double>(L.part), nz, p, q, kGT, s, at<double>(L.G));
    }

    // host G (p x q row-major) = U^T V (every product taken here is symmetric:
    // S^T S and S^T A S)
    bool gram(const double *U, int p, const double *V, int q, std::vector<double> &G)
    {
        gram_launch(U, p, V, q, true);
        G.resize(static_cast<size_t>(p) * q);
        if (hipMemcpyAsync(G.data(), at<double>(L.G), G.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
            return false;
        return hipStreamSynchronize(st) == hipSuccess && ok();
    }

    // Y (N x mo) = U (N x k) C (k x mo, host row-major); with Y2, columns
    // from jsplit on go to Y2 instead (column jsplit + c to Y2[:, c])
    bool update(const double *U, int k, const std::vector<double> &C, int mo, double *Y, double *Y2 = nullptr,
                int jsplit = -1)
    {
        if (!Y2) jsplit = mo;
        if (hipMemcpyAsync(at<double>(L.C), C.data(), C.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
            return false;
        if (k <= kNarrow && mo <= 16) {   // a few columns: streaming kernel
            const long long ln = static_cast<long long>(N);
            const unsigned nb = std::min<unsigned>(nblk(ln, 256), 4096);
            if (k <= 4)
                hipLaunchKernelGGL(k_update_narrow<4>, dim3(nb), dim3(256), 0, st, U, ln, k, at<double>(L.C), mo, Y,
                                   Y2, jsplit, ln);
            else
                hipLaunchKernelGGL(k_update_narrow<kNarrow>, dim3(nb), dim3(256), 0, st, U, ln, k, at<double>(L.C), mo,
                                   Y, Y2, jsplit, ln);
            return hipStreamSynchronize(st) == hipSuccess && ok();
        }
        // one 64-column tile of k_block_update reads U once already; it is
        // kept for 49..64 columns, where the 4-block instance needs 195 VGPRs
        if (mo <= kTriMax && (mo <= 48 || mo > kT)) {
            // rows of C that are nonzero per 16-column block; all-zero row spans are skipped
            RowSpan sp{};
            const int jn = (mo + 15) / 16;
            int i_begin = k, i_end = 0;
            for (int jt = 0; jt < jn; ++jt) {
                int lo = k, hi = 0;
                for (int i = 0; i < k; ++i)
                    for (int j = 16 * jt; j < std::min(mo, 16 * jt + 16); ++j)
                        if (C[static_cast<size_t>(i) * mo + j] != 0.0) {
                            lo = std::min(lo, i);
                            hi = i + 1;
                            break;
                        }
                sp.lo[jt] = lo;
                sp.hi[jt] = hi;
                if (lo < hi) {
                    i_begin = std::min(i_begin, lo);
                    i_end = std::max(i_end, hi);
                }
            }
            if (i_end <= i_begin) i_begin = i_end = 0;   // C == 0: the kernel writes zeros
            i_begin -= i_begin % kK;
            const dim3 grid(nblk(static_cast<long long>(N), kT));
            const dim3 grid2(nblk(static_cast<long long>(N), 2 * kT));
            const long long ln = static_cast<long long>(N);
            const double *Cd = at<double>(L.C);
            if (mo <= 32)
                hipLaunchKernelGGL((k_block_update_wide<2, 2>), grid2, dim3(256), 0, st, U, ln, i_begin, i_end, Cd, mo,
                                   sp, Y, ln, ln, Y2, jsplit);
            else if (mo <= 48)
                hipLaunchKernelGGL((k_block_update_wide<3, 2>), grid2, dim3(256), 0, st, U, ln, i_begin, i_end, Cd, mo,
                                   sp, Y, ln, ln, Y2, jsplit);
            else if (mo <= 128)
                hipLaunchKernelGGL((k_block_update_wide<8, 2>), grid2, dim3(256), 0, st, U, ln, i_begin, i_end, Cd, mo,
                                   sp, Y, ln, ln, Y2, jsplit);
            else if (mo <= 144)
                hipLaunchKernelGGL((k_block_update_wide<9, 2>), grid2, dim3(256), 0, st, U, ln, i_begin, i_end, Cd, mo,
                                   sp, Y, ln, ln, Y2, jsplit);
            else if (mo <= 208)
                hipLaunchKernelGGL(k_block_update_wide<13>, grid, dim3(256), 0, st, U, ln, i_begin, i_end, Cd, mo, sp,
                                   Y, ln, ln, Y2, jsplit);
            else
                hipLaunchKernelGGL(k_block_update_wide<kTriMax / 16>, grid, dim3(256), 0, st, U, ln, i_begin, i_end,
                                   Cd, mo, sp, Y, ln, ln, Y2, jsplit);
        } else {
            hipLaunchKernelGGL(k_block_update, dim3(nblk(static_cast<long long>(N), kT), nblk(mo, kT)), dim3(256), 0,
                               st, U, static_cast<long long>(N), k, at<double>(L.C), mo, Y, static_cast<long long>(N),
                               static_cast<long long>(N), Y2, jsplit);
        }
        // C is reused by the next call: wait before the host buffer changes
        return hipStreamSynchronize(st) == hipSuccess && ok();
    }

    // out[c] = (U[:, c], V[:, c]) for c < mcols (device out)
    void coldots(const double *U, const double *V, int mcols, double *out, double *part)
    {
        const int ns = L.nslices_col;
        const long long slice = (static_cast<long long>(N) + ns - 1) / ns;
        hipLaunchKernelGGL(k_coldot_partial, dim3(ns, mcols), dim3(256), 0, st, U, V, static_cast<long long>(N),
                           static_cast<long long>(N), slice, part, ns);
        hipLaunchKernelGGL(k_coldot_reduce, dim3(mcols), dim3(256), 0, st, part, ns, out);
    }

    void normalize(double *X, double *AX, int mcols)
    {
        double *nrm = at<double>(L.cout);
        coldots(X, X, mcols, nrm, at<double>(L.cpart));
        hipLaunchKernelGGL(k_scale_cols, dim3(nblk(static_cast<long long>(N), 256), mcols), dim3(256), 0, st, X, AX,
                           nrm, static_cast<long long>(N), static_cast<long long>(N), mcols);
    }

    // dst[:, t] = src[:, idx[t]], times scale[t] (host) when given
    bool gather(const double *src, double *dst, const std::vector<int> &idx, const double *scale = nullptr)
    {
        if (idx.empty()) return true;
        if (hipMemcpyAsync(at<int>(L.idx), idx.data(), idx.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess)
            return false;
        if (scale && hipMemcpyAsync(at<double>(L.gscale), scale, idx.size() * 8, hipMemcpyHostToDevice, st) !=
                         hipSuccess)
            return false;
        hipLaunchKernelGGL(k_gather_cols, dim3(nblk(static_cast<long long>(N), 256), static_cast<int>(idx.size())),
                           dim3(256), 0, st, src, dst, at<int>(L.idx), scale ? at<double>(L.gscale) : nullptr,
                           static_cast<long long>(N), static_cast<long long>(N), static_cast<int>(idx.size()));
        return hipStreamSynchronize(st) == hipSuccess && ok();
    }

    // Y = A X for cols columns (the grid operator; stream-ordered)
    bool apply_a(const double *X, double *Y, int cols)
    {
        return cols == 0 || smg_matvec(h, X, Y, cols, static_cast<int64_t>(N), st) == SMG_OK;
    }

    // A S after S <- S C (C k x mo): from the operator when the basis is wide
    // (a stencil pass over the mo new columns moves 16 N mo bytes, while the
    // k x mo update is bound by its N k mo MFMA flops), else by the same update
    // of A S.  Y receives the new A S; AS itself is only read.
    static constexpr int kStencilK = 96;
    bool new_as(const double *AS, int k, const std::vector<double> &C, int mo, const double *Snew, double *Y)
    {
        return k >= kStencilK ? apply_a(Snew, Y, mo) : update(AS, k, C, mo, Y);
    }

    // Cholesky QR twice of S (N x k). S and the scratch T swap roles, so after
    // two passes the result is back in S; A S follows the two (upper
    // triangular) factors at once: by their product, or for a wide basis by
    // the operator.
    int cholqr2(double *&S, double *&AS, double *&T, double *&AT, int k)
    {
        const size_t kk = static_cast<size_t>(k) * k;
        std::vector<double> G, C1(kk), C2(kk);
        for (int pass = 0; pass < 2; ++pass) {
            if (!gram(S, k, S, k, G)) return -1;
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < i; ++j) G[i * k + j] = G[j * k + i] = 0.5 * (G[i * k + j] + G[j * k + i]);
            if (!dense::cholesky(k, G.data())) {
                if (pass == 0) return 0;
                // keep A S in step with the once-factored S
                if (!new_as(AS, k, C1, k, S, AT)) return -1;
                std::swap(AS, AT);
                return 0;
            }
            std::vector<double> &C = pass == 0 ? C1 : C2;
            dense::inv_lower_transpose(k, G.data(), C.data());
            if (!update(S, k, C, k, T)) return -1;
            std::swap(S, T);
        }
        std::vector<double> Cp;
        if (k < kStencilK) {
            Cp.assign(kk, 0.0);
            for (int i = 0; i < k; ++i)
                for (int l = i; l < k; ++l) {
                    const double c = C1[i * k + l];
                    for (int j = l; j < k; ++j) Cp[i * k + j] += c * C2[l * k + j];
                }
        }
        if (!new_as(AS, k, Cp, k, S, AT)) return -1;
        std::swap(AS, AT);
        return 1;
    }

    // eigen-based orthonormalisation of S (N x k); returns the kept count
    int svqb(double *&S, double *&AS, double *&T, double *&AT, int k)
    {
        std::vector<double> G;
        if (!gram(S, k, S, k, G)) return -1;
        std::vector<double> dinv(k), Gs(static_cast<size_t>(k) * k), V(static_cast<size_t>(k) * k), w(k);
        for (int i = 0; i < k; ++i) {
            const double d = std::sqrt(std::fabs(G[i * k + i]));
            dinv[i] = d > 0 ? 1.0 / d : 1.0;
        }
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < k; ++j)
                Gs[i * k + j] = 0.5 * (G[i * k + j] + G[j * k + i]) * dinv[i] * dinv[j];
        if (!dense::sym_eig(k, Gs.data(), V.data(), w.data())) return -1;
        const double wmax = w[k - 1];
        std::vector<int> keep;
        for (int j = 0; j < k; ++j)
            if (w[j] > 1e-12 * wmax) keep.push_back(j);
        const int kk = static_cast<int>(keep.size());
        std::vector<double> Cm(static_cast<size_t>(k) * kk);
        for (int i = 0; i < k; ++i)
            for (int jj = 0; jj < kk; ++jj)
                Cm[i * kk + jj] = dinv[i] * V[i * k + keep[jj]] / std::sqrt(w[keep[jj]]);
        if (!update(S, k, Cm, kk, T) || !new_as(AS, k, Cm, kk, T, AT)) return -1;
        std::swap(S, T);
        std::swap(AS, AT);
        return kk;
    }
};

}  // namespace

extern "C" {

int lobpcg_workspace_bytes(smg_handle *h, int32_t m, size_t *bytes)
{
    if (!h || m < 1 || !bytes) return SMG_EINVAL;
    size_t N = 0;
    if (smg_handle_size(h, &N) != SMG_OK) return SMG_EINVAL;
    *bytes = lob_layout(N, m).total;
    return SMG_OK;
}

int lobpcg_profile_gram(smg_handle *h, int32_t m, int32_t k, void *ws, size_t ws_bytes, int32_t reps, void *stream,
                        double *ms)
{
    if (!h || !ws || !ms || m < 1 || k < 1 || k > 3 * m || reps < 1) return SMG_EINVAL;
    size_t N = 0;
    if (smg_handle_size(h, &N) != SMG_OK) return SMG_EINVAL;
    Lob lb{h, reinterpret_cast<hipStream_t>(stream), N, m, static_cast<char *>(ws), lob_layout(N, m)};
    if (ws_bytes < lb.L.total) return SMG_EWORKSPACE;
    hipStream_t st = lb.st;
    double *S = lb.at<double>(lb.L.S);
    launch_fill(S, 1.0 / 1024.0, N * static_cast<size_t>(k), st);
    auto one = [&]() { lb.gram_launch(S, k, S, k, true); };
    one();   // warm-up
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SMG_EHIP;
    int rc = SMG_OK;
    float t = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess) rc = SMG_EHIP;
    for (int i = 0; rc == SMG_OK && i < reps; ++i) one();
    if (rc == SMG_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                         hipEventElapsedTime(&t, e0, e1) != hipSuccess || !lb.ok()))
        rc = SMG_EHIP;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = static_cast<double>(t) / reps;
    return rc;
}

int lobpcg_solve(smg_handle *h, int32_t m, double *X, double *lambda, double *resnorms, void *ws, size_t ws_bytes,
                 const lobpcg_opts *o, lobpcg_info *info, void *stream)
{
    if (!h || !X || !lambda || !ws || !o || m < 1 || o->max_iter < 0 || !(o->rtol >= 0.0)) return SMG_EINVAL;
    if (o->precond != SMG_PRECOND_SMG && o->precond != SMG_PRECOND_NONE) return SMG_EINVAL;
    if (o->guard < 0) return SMG_EINVAL;
    const int mw = m;     // wanted pairs; the block also carries the guard columns
    m += o->guard;
    size_t N = 0;
    int32_t max_nrhs = 0;
    if (smg_handle_size(h, &N) != SMG_OK || smg_handle_max_nrhs(h, &max_nrhs) != SMG_OK) return SMG_EINVAL;
    if (o->precond == SMG_PRECOND_SMG && max_nrhs < m) return SMG_EINVAL;
    if (static_cast<size_t>(m) > N) return SMG_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    Lob lb{h, reinterpret_cast<hipStream_t>(stream), N, m, static_cast<char *>(ws), lob_layout(N, m)};
    if (ws_bytes < lb.L.total) return SMG_EWORKSPACE;
    hipStream_t st = lb.st;
    lobpcg_info inf{};
    auto finish = [&](int status) {
        inf.status = status;
        inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (info) *info = inf;
        return status;
    };
    const long long ld = static_cast<long long>(N);
    double *S = lb.at<double>(lb.L.S), *AS = lb.at<double>(lb.L.AS);
    double *T = lb.at<double>(lb.L.T), *AT = lb.at<double>(lb.L.AT);
    double *P = lb.at<double>(lb.L.P), *AP = lb.at<double>(lb.L.AP), *R = lb.at<double>(lb.L.R);
    double *theta_d = lb.at<double>(lb.L.theta);

    if (hipMemcpyAsync(S, X, N * m * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) return finish(SMG_EHIP);
    if (smg_matvec(h, S, AS, m, ld, stream) != SMG_OK) return finish(SMG_EHIP);
    {
        int rc = lb.cholqr2(S, AS, T, AT, m);
        if (rc < 0) return finish(SMG_EHIP);
        if (rc == 0) {
            const int kk = lb.svqb(S, AS, T, AT, m);
            if (kk < 0) return finish(SMG_EHIP);
            if (kk < m) return finish(SMG_EBREAKDOWN);   // initial block is rank deficient
        }
    }
    std::vector<double> G, V, w, theta(m);
    // initial Rayleigh-Ritz on span(X)
    if (!lb.gram(S, m, AS, m, G)) return finish(SMG_EHIP);
    for (int i = 0; i < m; ++i)
        for (int j = 0; j < i; ++j) G[i * m + j] = G[j * m + i] = 0.5 * (G[i * m + j] + G[j * m + i]);
    V.resize(static_cast<size_t>(m) * m);
    w.resize(m);
    if (!dense::sym_eig(m, G.data(), V.data(), w.data())) return finish(SMG_EBREAKDOWN);
    if (!lb.update(S, m, V, m, T) || !lb.new_as(AS, m, V, m, T, AT)) return finish(SMG_EHIP);
    std::swap(S, T);
    std::swap(AS, AT);
    for (int i = 0; i < m; ++i) theta[i] = w[i];

    bool have_p = false;
    std::vector<double> rr(m), xx(m), res(m), pinv(m, 1.0);
    std::vector<int> active, all(m);
    for (int i = 0; i < m; ++i) all[i] = i;
    int it = 0;
    int status = SMG_NOT_CONVERGED;
    for (;; ++it) {
        // residuals and their relative norms
        if (hipMemcpyAsync(theta_d, theta.data(), m * 8, hipMemcpyHostToDevice, st) != hipSuccess)
            return finish(SMG_EHIP);
        double *cout = lb.at<double>(lb.L.cout);
        {
            // R and the column norms of R and X in one pass
            const int ns = lb.L.nslices_col;
            const long long slice = (ld + ns - 1) / ns;
            double *cp = lb.at<double>(lb.L.cpart);
            hipLaunchKernelGGL(k_block_resid_dots, dim3(ns, m), dim3(256), 0, st, AS, S, theta_d, R, ld, ld, slice, cp,
                               ns, m);
            hipLaunchKernelGGL(k_coldot_reduce, dim3(2 * m), dim3(256), 0, st, cp, ns, cout);
        }
        std::vector<double> nr(2 * m);
        if (hipMemcpyAsync(nr.data(), cout, 2 * m * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess || !lb.ok())
            return finish(SMG_EHIP);
        active.clear();
        int wanted_left = 0;
        for (int i = 0; i < m; ++i) {
            res[i] = std::sqrt(nr[i]) / (std::fabs(theta[i]) * std::sqrt(nr[m + i]));
            if (!std::isfinite(res[i])) return finish(SMG_EBREAKDOWN);
            if (res[i] > o->rtol) {
                active.push_back(i);
                if (i < mw) ++wanted_left;
            }
        }
        inf.nconv = mw - wanted_left;
        if (wanted_left == 0) {
            status = SMG_OK;
            break;
        }
        if (it >= o->max_iter) break;
        const int nj = static_cast<int>(active.size());
        // W = T R_J into S[:, m : m+nj]
        double *W = S + static_cast<size_t>(m) * N, *AW = AS + static_cast<size_t>(m) * N;
        // R_J: R itself while every column is active, else gathered into T
        const double *RJ = R;
        if (nj < m) {
            if (!lb.gather(R, T, active)) return finish(SMG_EHIP);
            RJ = T;
        }
        if (o->precond == SMG_PRECOND_SMG) {
            if (smg_apply(h, RJ, W, nj, ld, stream) != SMG_OK) return finish(SMG_EHIP);
        } else if (hipMemcpyAsync(W, RJ, N * nj * 8, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            return finish(SMG_EHIP);
        }
        lb.normalize(W, nullptr, nj);
        if (smg_matvec(h, W, AW, nj, ld, stream) != SMG_OK) return finish(SMG_EHIP);
        int k = m + nj;
        if (have_p) {
            // P's columns come out of the last Rayleigh-Ritz step with norms
            // known from its coefficients (S was orthonormal), so the gather
            // normalises them itself
            double *Pj = S + static_cast<size_t>(k) * N, *APj = AS + static_cast<size_t>(k) * N;
            std::vector<double> sc(nj);
            for (int t = 0; t < nj; ++t) sc[t] = pinv[active[t]];
            if (!lb.gather(P, Pj, active, sc.data()) || !lb.gather(AP, APj, active, sc.data()))
                return finish(SMG_EHIP);
            k += nj;
        }
        int rc = lb.cholqr2(S, AS, T, AT, k);
        if (rc < 0) return finish(SMG_EHIP);
        if (rc == 0 && have_p) {
            k = m + nj;
            rc = lb.cholqr2(S, AS, T, AT, k);
            if (rc < 0) return finish(SMG_EHIP);
        }
        if (rc == 0) {
            k = lb.svqb(S, AS, T, AT, k);
            if (k < 0) return finish(SMG_EHIP);
            if (k < m) return finish(SMG_EBREAKDOWN);
        }
        // Rayleigh-Ritz on S^T A S
        if (!lb.gram(S, k, AS, k, G)) return finish(SMG_EHIP);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < i; ++j) G[i * k + j] = G[j * k + i] = 0.5 * (G[i * k + j] + G[j * k + i]);
        V.resize(static_cast<size_t>(k) * k);
        w.resize(k);
        if (!dense::sym_eig(k, G.data(), V.data(), w.data())) return finish(SMG_EBREAKDOWN);
        for (int i = 0; i < m; ++i) theta[i] = w[i];
        // [X_new | P_new] = S [C_m | C_m with the X rows zeroed]
        std::vector<double> Ce(static_cast<size_t>(k) * 2 * m, 0.0);
        for (int i = 0; i < k; ++i)
            for (int j = 0; j < m; ++j) {
                Ce[static_cast<size_t>(i) * 2 * m + j] = V[static_cast<size_t>(i) * k + j];
                if (i >= m) Ce[static_cast<size_t>(i) * 2 * m + m + j] = V[static_cast<size_t>(i) * k + j];
            }
        // 1 / ||P_new[:, j]|| = 1 / ||C_P[:, j]|| for orthonormal S (1 for a zero column)
        for (int j = 0; j < m; ++j) {
            double q = 0.0;
            for (int i = m; i < k; ++i) {
                const double c = Ce[static_cast<size_t>(i) * 2 * m + m + j];
                q += c * c;
            }
            pinv[j] = q > 0.0 ? 1.0 / std::sqrt(q) : 1.0;
        }
        // X into the scratch (then swapped in), P straight into its own buffer
        // (the gathered copy in S is what is read); AX and AP likewise, by the
        // operator for a wide basis
        if (!lb.update(S, k, Ce, 2 * m, T, P, m)) return finish(SMG_EHIP);
        const bool ok_as = k >= Lob::kStencilK ? lb.apply_a(T, AT, m) && lb.apply_a(P, AP, m)
                                               : lb.update(AS, k, Ce, 2 * m, AT, AP, m);
        if (!ok_as) return finish(SMG_EHIP);
        std::swap(S, T);
        std::swap(AS, AT);
        have_p = true;
    }
    if (hipMemcpyAsync(X, S, N * m * 8, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return finish(SMG_EHIP);
    for (int i = 0; i < m; ++i) {
        lambda[i] = theta[i];
        if (resnorms) resnorms[i] = res[i];
    }
    inf.iters = it;
    return finish(status);
}

}  // extern "C"
