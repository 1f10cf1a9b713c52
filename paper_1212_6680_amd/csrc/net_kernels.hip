// Kernels of the learned post-smoother network: four 3x3x3 convolutions with
// zero padding (1 -> 16 -> 16 -> 16 -> 1 channels, ReLU after the first
// three), their input and weight gradients, the mean-squared-error loss and
// the Adam update.
//
// Activations are channels-last (voxel-major, 16 channels of one voxel
// contiguous), voxel index x + nx*(y + ny*z).  Storage type T is bf16 (FP32
// arithmetic, FP32 master weights) or double (FP64 check mode).
// Weights of a layer: W[tap][ci][co], tap = 9*dz + 3*dy + dx, then the bias.
//
// The 16 -> 16 layers in bf16 run on MFMA (v_mfma_f32_16x16x32_bf16): one
// instruction contracts 16 output channels x 16 voxels over 32 = two taps x
// 16 input channels.  Operand layout (gfx950, measured): A[i][k] in lane
// i + 16*(k/8), element k%8; B[k][j] in lane j + 16*(k/8), element k%8;
// D[i][j] in lane j + 16*(i/4), element i%4.  With A = weights (i = output
// channel) and B = input voxels (j = voxel), each lane ends up holding four
// consecutive output channels of one voxel, which is one 8-byte store.
#include "net_internal.h"

namespace smg {
namespace net {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ inline float lo_bf(unsigned int u) { return __uint_as_float(u << 16); }
__device__ inline float hi_bf(unsigned int u) { return __uint_as_float(u & 0xffff0000u); }
__device__ inline unsigned int pack2(float a, float b)
{
    return static_cast<unsigned int>(f_to_bf16(a).bits) | (static_cast<unsigned int>(f_to_bf16(b).bits) << 16);
}

template <typename T> __device__ inline typename Arith<T>::type load_a(const T *p) { return ldv(p); }

// ---------------------------------------------------------------------------
// MFMA convolution 16 -> 16 (bf16 storage, FP32 accumulation)
// ---------------------------------------------------------------------------
constexpr int MTX = 64, MTY = 8;                 // output tile per z step
constexpr int MHX = MTX + 2, MHY = MTY + 2;      // with halo
constexpr int MPLANE = MHX * MHY;                // voxels per staged plane
constexpr int MITEMS = 2 * MPLANE;               // 16-byte chunks per plane
constexpr int MPER = (MITEMS + 255) / 256;       // chunks per thread

__device__ inline void mfma_fetch(const u32x4 *in, int x0, int y0, int zi, int nx, int ny, int nz, u32x4 *reg)
{
#pragma unroll
    for (int m = 0; m < MPER; ++m) {
        const int it = threadIdx.x + 256 * m;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (it < MITEMS) {
            const int h = it & 1, rest = it >> 1;
            const int lx = rest % MHX, ly = rest / MHX;
            const int gx = x0 + lx - 1, gy = y0 + ly - 1;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && zi >= 0 && zi < nz)
                v = in[((static_cast<long long>(zi) * ny + gy) * nx + gx) * 2 + h];
        }
        reg[m] = v;
    }
}

__device__ inline void mfma_stage(u32x4 *lds, int slot, const u32x4 *reg)
{
#pragma unroll
    for (int m = 0; m < MPER; ++m) {
        const int it = threadIdx.x + 256 * m;
        if (it < MITEMS) {
            const int h = it & 1, rest = it >> 1;
            lds[(slot * 2 + h) * MPLANE + rest] = reg[m];
        }
    }
}

// EPI: 0 = bias + ReLU, 1 = multiply by (mask > 0)
template <int EPI>
__global__ __launch_bounds__(256) void k_conv16_mfma(Conv16Args a)
{
    __shared__ u32x4 lds[3 * 2 * MPLANE];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x0 = blockIdx.x * MTX, y0 = blockIdx.y * MTY;
    const int z0 = blockIdx.z * a.zc;
    const int z1 = min(z0 + a.zc, a.nz);
    const u32x4 *in = reinterpret_cast<const u32x4 *>(a.in);

    bf16x8 wf[14];
#pragma unroll
    for (int p = 0; p < 14; ++p) wf[p] = __builtin_bit_cast(bf16x8, reinterpret_cast<const u32x4 *>(a.frag)[p * 64 + lane]);
    const int q = lane >> 4, j = lane & 15, hh = (lane >> 4) & 1, tp = lane >> 5;
    float bias[4] = {0.f, 0.f, 0.f, 0.f};
    if (EPI == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[e] = a.bias[4 * q + e];
    }
    // per pair: LDS offset of this lane's tap relative to the tile origin
    int toff[14], tz[14];
#pragma unroll
    for (int p = 0; p < 14; ++p) {
        int t = 2 * p + tp;
        t = t > 26 ? 26 : t;
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        tz[p] = dz;
        toff[p] = hh * MPLANE + dy * MHX + dx;
    }

    u32x4 reg[MPER];
    mfma_fetch(in, x0, y0, z0 - 1, a.nx, a.ny, a.nz, reg);
    mfma_stage(lds, 0, reg);
    mfma_fetch(in, x0, y0, z0, a.nx, a.ny, a.nz, reg);
    mfma_stage(lds, 1, reg);
    mfma_fetch(in, x0, y0, z0 + 1, a.nx, a.ny, a.nz, reg);
    for (int z = z0; z < z1; ++z) {
        const int base = z - z0;                  // plane z-1 sits in slot base % 3
        mfma_stage(lds, (base + 2) % 3, reg);
        __syncthreads();
        if (z + 2 <= z1) mfma_fetch(in, x0, y0, z + 2, a.nx, a.ny, a.nz, reg);
        f32x4 acc[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int p = 0; p < 14; ++p) {
            const int slot = (base + tz[p]) % 3;
            const int o = slot * 2 * MPLANE + toff[p] + (2 * w) * MHX + j;
#pragma unroll
            for (int r = 0; r < 2; ++r)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const bf16x8 bv = __builtin_bit_cast(bf16x8, lds[o + r * MHX + 16 * s]);
                    acc[r * 4 + s] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[p], bv, acc[r * 4 + s], 0, 0, 0);
                }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            const int gy = y0 + 2 * w + r;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int gx = x0 + 16 * s + j;
                if (gx < a.nx && gy < a.ny) {
                    const long long v = (static_cast<long long>(z) * a.ny + gy) * a.nx + gx;
                    float o4[4];
#pragma unroll
                    for (int e = 0; e < 4; ++e) o4[e] = acc[r * 4 + s][e];
                    if (EPI == 0) {
#pragma unroll
                        for (int e = 0; e < 4; ++e) o4[e] = fmaxf(o4[e] + bias[e], 0.f);
                    } else {
                        const u32x2 mk = reinterpret_cast<const u32x2 *>(a.mask)[v * 4 + q];
                        if (!(lo_bf(mk.x) > 0.f)) o4[0] = 0.f;
                        if (!(hi_bf(mk.x) > 0.f)) o4[1] = 0.f;
                        if (!(lo_bf(mk.y) > 0.f)) o4[2] = 0.f;
                        if (!(hi_bf(mk.y) > 0.f)) o4[3] = 0.f;
                    }
                    u32x2 st;
                    st.x = pack2(o4[0], o4[1]);
                    st.y = pack2(o4[2], o4[3]);
                    reinterpret_cast<u32x2 *>(a.out)[v * 4 + q] = st;
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// bf16 single-channel layers on vector ALUs with packed bf16 dot products
// (v_dot2_f32_bf16: two bf16 products added to an FP32 accumulator).
// Block: 64 x 4 output voxels per z step, marching through zc planes with a
// ring of three staged input planes; weights are read with uniform addresses.
// ---------------------------------------------------------------------------
typedef __attribute__((__vector_size__(2 * sizeof(__bf16)))) __bf16 bf16x2;
constexpr int SRY = 2;                                   // output rows per thread
constexpr int STX = 64, STY = 4 * SRY, SHX = STX + 2, SHY = STY + 2, SPLANE = SHX * SHY;

__device__ inline float dot2(unsigned int a, unsigned int b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a), __builtin_bit_cast(bf16x2, b), c, false);
}

// 1 -> 16 (layer 0 forward; input gradient of layer 3) on the matrix cores:
// out[co][voxel] = sum_t W[t][co] in[voxel + off_t] is one
// v_mfma_f32_16x16x32_bf16 per 16 voxels (A = the 16 x 32 weight matrix, taps
// 27..31 zero; B = each voxel's 27 neighbours gathered from the staged
// planes).  INM 0: bf16 input; INM 1: FP64 input times ns->in_scale, rounded
// to bf16.  EPI 0: bias + ReLU; EPI 1: mask.  w: the [27][16] bf16 weights.
template <int INM, int EPI>
__global__ __launch_bounds__(256) void k_in16_bf16(In16Args a)
{
    constexpr int PER = (SPLANE + 255) / 256;
    __shared__ uint16_t lds[3 * SPLANE];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int x0 = blockIdx.x * STX, y0 = blockIdx.y * STY;
    const int z0 = blockIdx.z * a.zc, z1 = min(z0 + a.zc, a.nz);
    const double in_scale = INM == 1 ? a.ns->in_scale : 1.0;
    const int j = lane & 15, q = lane >> 4;
    // A fragment: lane (co = j, taps 8q .. 8q+7)
    bf16x8 wf;
    int toff[8], slot_of[8][3];
    unsigned int keep[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int t = 8 * q + e;
        wf[e] = t < 27 ? __builtin_bit_cast(__bf16, a.w[t * 16 + j].bits) : static_cast<__bf16>(0.0f);
        const int tc = t < 27 ? t : 26;
        toff[e] = ((tc / 3) % 3) * SHX + tc % 3;
        keep[e] = t < 27 ? 0xffffu : 0u;
        // LDS offset of the plane z + dz - 1 for each ring position of plane z - 1
#pragma unroll
        for (int b3 = 0; b3 < 3; ++b3) slot_of[e][b3] = ((b3 + tc / 9) % 3) * SPLANE;
    }
    float bias[4] = {0.f, 0.f, 0.f, 0.f};
    if (EPI == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) bias[e] = a.bias[4 * q + e];
    }
    auto fetch = [&](int zi, uint16_t *reg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int it = threadIdx.x + 256 * m;
            uint16_t v = 0;
            if (it < SPLANE) {
                const int lx = it % SHX, ly = it / SHX;
                const int gx = x0 + lx - 1, gy = y0 + ly - 1;
                if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && zi >= 0 && zi < a.nz) {
                    const long long g = (static_cast<long long>(zi) * a.ny + gy) * a.nx + gx;
                    if (INM == 0)
                        v = a.in[g].bits;
                    else
                        v = f_to_bf16(static_cast<float>(a.in64[g] * in_scale)).bits;
                }
            }
            reg[m] = v;
        }
    };
    auto stage = [&](int slot, const uint16_t *reg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int it = threadIdx.x + 256 * m;
            if (it < SPLANE) lds[slot * SPLANE + it] = reg[m];
        }
    };
    uint16_t reg[PER];
    fetch(z0 - 1, reg);
    stage(0, reg);
    fetch(z0, reg);
    stage(1, reg);
    fetch(z0 + 1, reg);
    for (int z = z0; z < z1; ++z) {
        const int base = z - z0;
        stage((base + 2) % 3, reg);
        __syncthreads();
        if (z + 2 <= z1) fetch(z + 2, reg);
        // wave w: rows 2w, 2w+1 of the tile, four 16-voxel segments each
#pragma unroll
        for (int sg = 0; sg < 8; ++sg) {
            const int row = 2 * w + (sg >> 2), xs = 16 * (sg & 3) + j;
            // every gather reads a valid location (taps past 26 alias tap 26);
            // the missing taps are then zeroed without branching
            unsigned int pk[4];
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const unsigned int lo = lds[slot_of[2 * h][base % 3] + row * SHX + xs + toff[2 * h]];
                const unsigned int hi = lds[slot_of[2 * h + 1][base % 3] + row * SHX + xs + toff[2 * h + 1]];
                pk[h] = (lo & keep[2 * h]) | ((hi & keep[2 * h + 1]) << 16);
            }
            u32x4 pv = {pk[0], pk[1], pk[2], pk[3]};
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf, __builtin_bit_cast(bf16x8, pv), acc, 0, 0, 0);
            const int gy = y0 + row, gx = x0 + xs;
            if (gx < a.nx && gy < a.ny) {
                const long long v = (static_cast<long long>(z) * a.ny + gy) * a.nx + gx;
                float o4[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) o4[e] = acc[e];
                if (EPI == 0) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) o4[e] = fmaxf(o4[e] + bias[e], 0.f);
                } else {
                    const u32x2 mk = reinterpret_cast<const u32x2 *>(a.mask)[v * 4 + q];
                    if (!(lo_bf(mk.x) > 0.f)) o4[0] = 0.f;
                    if (!(hi_bf(mk.x) > 0.f)) o4[1] = 0.f;
                    if (!(lo_bf(mk.y) > 0.f)) o4[2] = 0.f;
                    if (!(hi_bf(mk.y) > 0.f)) o4[3] = 0.f;
                }
                u32x2 st;
                st.x = pack2(o4[0], o4[1]);
                st.y = pack2(o4[2], o4[3]);
                reinterpret_cast<u32x2 *>(a.out)[v * 4 + q] = st;
            }
        }
        __syncthreads();
    }
}

// 16 -> 1 (layer 3 forward).  EPI 2: outA = acc + b; EPI 3: s_out = s_in +
// out_scale * (acc + b).  w: the layer's bf16 weights W[t][ci] as channel
// pairs, kept in LDS; each thread computes SRY voxels along y.
template <int EPI>
__global__ __launch_bounds__(256) void k_out16_bf16(Out16Args a, const u32x4 *__restrict__ wg)
{
    __shared__ u32x4 lds[3 * 2 * SPLANE];
    constexpr int ITEMS = 2 * SPLANE, PER = (ITEMS + 255) / 256;
    const int tx = threadIdx.x % STX, ty = threadIdx.x / STX;
    const int x0 = blockIdx.x * STX, y0 = blockIdx.y * STY;
    const int z0 = blockIdx.z * a.zc, z1 = min(z0 + a.zc, a.nz);
    const u32x4 *in = reinterpret_cast<const u32x4 *>(a.in);
    // the weights are the same for every lane: read per tap plane through the
    // scalar cache (wg is a read-only kernel argument) rather than from LDS,
    // which the activations need
    auto fetch = [&](int zi, u32x4 *reg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int it = threadIdx.x + 256 * m;
            u32x4 v = {0u, 0u, 0u, 0u};
            if (it < ITEMS) {
                const int h = it & 1, rest = it >> 1;
                const int lx = rest % SHX, ly = rest / SHX;
                const int gx = x0 + lx - 1, gy = y0 + ly - 1;
                if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && zi >= 0 && zi < a.nz)
                    v = in[((static_cast<long long>(zi) * a.ny + gy) * a.nx + gx) * 2 + h];
            }
            reg[m] = v;
        }
    };
    auto stage = [&](int slot, const u32x4 *reg) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int it = threadIdx.x + 256 * m;
            if (it < ITEMS) lds[(slot * 2 + (it & 1)) * SPLANE + (it >> 1)] = reg[m];
        }
    };
    const float b = a.bias[0];
    const double out_scale = EPI == 3 ? a.ns->out_scale : 0.0;
    u32x4 reg[PER];
    fetch(z0 - 1, reg);
    stage(0, reg);
    fetch(z0, reg);
    stage(1, reg);
    fetch(z0 + 1, reg);
    const int gx = x0 + tx;
    for (int z = z0; z < z1; ++z) {
        const int base = z - z0;
        stage((base + 2) % 3, reg);
        __syncthreads();
        if (z + 2 <= z1) fetch(z + 2, reg);
        float acc[SRY];
#pragma unroll
        for (int r = 0; r < SRY; ++r) acc[r] = 0.f;
#pragma unroll 1
        for (int dz = 0; dz < 3; ++dz) {
            u32x4 wz[9][2];
#pragma unroll
            for (int t9 = 0; t9 < 9; ++t9) {
                wz[t9][0] = wg[2 * (9 * dz + t9)];
                wz[t9][1] = wg[2 * (9 * dz + t9) + 1];
            }
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
#pragma unroll
                for (int yy = 0; yy < SRY + 2; ++yy) {
                    // input row SRY*ty + yy feeds output rows r = yy - dy for dy = 0..2
                    const int o = ((base + dz) % 3) * 2 * SPLANE + (SRY * ty + yy) * SHX + tx + dx;
                    const u32x4 v0 = lds[o], v1 = lds[o + SPLANE];
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy) {
                        const int r = yy - dy;
                        if (r >= 0 && r < SRY) {
                            const u32x4 w0 = wz[3 * dy + dx][0], w1 = wz[3 * dy + dx][1];
#pragma unroll
                            for (int e = 0; e < 4; ++e) {
                                acc[r] = dot2(v0[e], w0[e], acc[r]);
                                acc[r] = dot2(v1[e], w1[e], acc[r]);
                            }
                        }
                    }
                }
        }
#pragma unroll
        for (int r = 0; r < SRY; ++r) {
            const int gy = y0 + SRY * ty + r;
            if (gx < a.nx && gy < a.ny) {
                const long long v = (static_cast<long long>(z) * a.ny + gy) * a.nx + gx;
                if (EPI == 2)
                    a.outA[v] = acc[r] + b;
                else
                    a.s_out[v] = a.s_in[v] + out_scale * static_cast<double>(acc[r] + b);
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Direct convolution on vector ALUs (the FP64 check mode, and any layer
// shape without a bf16 kernel).  One output voxel per thread.
// ---------------------------------------------------------------------------
template <typename A> struct VecTile;
template <> struct VecTile<double> { static constexpr int TX = 16, TY = 4, TZ = 2; };

// INM: 0 = storage input with CIN channels; 1 = FP64 single channel times
// the device in_scale, rounded to the storage type first.
// EPI: 0 = bias + ReLU -> T; 1 = mask -> T; 2 = bias -> A (single channel);
//      3 = s_out = s_in + out_scale * (acc + bias) (single channel, FP64).
template <typename T, typename A, int CIN, int COUT, int INM, int EPI>
__global__ __launch_bounds__(VecTile<A>::TX * VecTile<A>::TY * VecTile<A>::TZ) void k_conv_vec(ConvVecArgs<T, A> a)
{
    constexpr int TX = VecTile<A>::TX, TY = VecTile<A>::TY, TZ = VecTile<A>::TZ;
    constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, HV = HX * HY * HZ;
    constexpr int NT = TX * TY * TZ;
    constexpr int NW = 27 * CIN * COUT;
    constexpr bool WLDS = NW <= 432;
    __shared__ A tile[HV * CIN];
    __shared__ A wl[WLDS ? NW : 1];
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY, z0 = blockIdx.z * TZ;
    double in_scale = 0.0;
    if (INM == 1) in_scale = a.ns->in_scale;
    for (int it = threadIdx.x; it < HV * CIN; it += NT) {
        const int c = it % CIN, hv = it / CIN;
        const int lx = hv % HX, ly = (hv / HX) % HY, lz = hv / (HX * HY);
        const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + lz - 1;
        A v = A(0);
        if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz) {
            const long long g = (static_cast<long long>(gz) * a.ny + gy) * a.nx + gx;
            if (INM == 0) {
                v = load_a(a.in + g * CIN + c);
            } else {
                T q;
                stv(&q, static_cast<A>(a.in64[g] * in_scale));
                v = load_a(&q);
            }
        }
        tile[it] = v;
    }
    if (WLDS)
        for (int i = threadIdx.x; i < NW; i += NT) wl[i] = load_a(a.W + i);
    __syncthreads();
    const int tx = threadIdx.x % TX, ty = (threadIdx.x / TX) % TY, tz = threadIdx.x / (TX * TY);
    const int gx = x0 + tx, gy = y0 + ty, gz = z0 + tz;
    if (gx >= a.nx || gy >= a.ny || gz >= a.nz) return;
    A acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = A(0);
    for (int t = 0; t < 27; ++t) {
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        const A *src = tile + (((tz + dz) * HY + (ty + dy)) * HX + (tx + dx)) * CIN;
#pragma unroll
        for (int ci = 0; ci < CIN; ++ci) {
            const A xv = src[ci];
#pragma unroll
            for (int co = 0; co < COUT; ++co) {
                const int wi = (t * CIN + ci) * COUT + co;
                const A wv = WLDS ? wl[wi] : load_a(a.W + wi);
                acc[co] += xv * wv;
            }
        }
    }
    const long long v = (static_cast<long long>(gz) * a.ny + gy) * a.nx + gx;
    if (EPI == 0) {
#pragma unroll
        for (int co = 0; co < COUT; ++co) {
            const A o = acc[co] + a.bias[co];
            stv(a.out + v * COUT + co, o > A(0) ? o : A(0));
        }
    } else if (EPI == 1) {
#pragma unroll
        for (int co = 0; co < COUT; ++co) {
            const A m = load_a(a.mask + v * COUT + co);
            stv(a.out + v * COUT + co, m > A(0) ? acc[co] : A(0));
        }
    } else if (EPI == 2) {
        a.outA[v] = acc[0] + a.bias[0];
    } else {
        a.s_out[v] = a.s_in[v] + a.ns->out_scale * static_cast<double>(acc[0] + a.bias[0]);
    }
}

// ---------------------------------------------------------------------------
// Weight and bias gradients: dW[t][ci][co] = sum_v in[v + t - 1][ci] g[v][co],
// db[co] = sum_v g[v][co].  A fixed grid of blocks strides over voxel tiles
// and writes one partial per block; k_wgrad_reduce adds them in block order.
// ---------------------------------------------------------------------------
constexpr int WTX = 8, WTY = 4, WTZ = 4, WNV = WTX * WTY * WTZ;
constexpr int WHX = WTX + 2, WHY = WTY + 2, WHZ = WTZ + 2, WHV = WHX * WHY * WHZ;

template <typename T, typename A, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs<T, A> a)
{
    constexpr int NW = 27 * CIN * COUT;
    constexpr int MW = (NW + 255) / 256;
    __shared__ A tin[WHV * CIN];
    __shared__ A tg[WNV * COUT];
    const int gxn = (a.nx + WTX - 1) / WTX, gyn = (a.ny + WTY - 1) / WTY, gzn = (a.nz + WTZ - 1) / WTZ;
    const long long ntiles = static_cast<long long>(gxn) * gyn * gzn;
    A acc[MW];
    int toff[MW], tci[MW], tco[MW];
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        acc[m] = A(0);
        const int wi = threadIdx.x + 256 * m;
        const int wcl = wi < NW ? wi : 0;
        const int co = wcl % COUT, ci = (wcl / COUT) % CIN, t = wcl / (COUT * CIN);
        const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;
        toff[m] = (dz * WHY + dy) * WHX + dx;
        tci[m] = ci;
        tco[m] = co;
    }
    A bacc = A(0);
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const int bx = static_cast<int>(tile % gxn), by = static_cast<int>((tile / gxn) % gyn),
                  bz = static_cast<int>(tile / (static_cast<long long>(gxn) * gyn));
        const int x0 = bx * WTX, y0 = by * WTY, z0 = bz * WTZ;
        __syncthreads();
        for (int it = threadIdx.x; it < WHV * CIN; it += 256) {
            const int c = it % CIN, hv = it / CIN;
            const int lx = hv % WHX, ly = (hv / WHX) % WHY, lz = hv / (WHX * WHY);
            const int gx = x0 + lx - 1, gy = y0 + ly - 1, gz = z0 + lz - 1;
            A v = A(0);
            if (gx >= 0 && gx < a.nx && gy >= 0 && gy < a.ny && gz >= 0 && gz < a.nz)
                v = load_a(a.in + ((static_cast<long long>(gz) * a.ny + gy) * a.nx + gx) * CIN + c);
            tin[it] = v;
        }
        for (int it = threadIdx.x; it < WNV * COUT; it += 256) {
            const int c = it % COUT, lv = it / COUT;
            const int lx = lv % WTX, ly = (lv / WTX) % WTY, lz = lv / (WTX * WTY);
            const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
            A v = A(0);
            if (gx < a.nx && gy < a.ny && gz < a.nz)
                v = load_a(a.g + ((static_cast<long long>(gz) * a.ny + gy) * a.nx + gx) * COUT + c);
            tg[it] = v;
        }
        __syncthreads();
        for (int lv = 0; lv < WNV; ++lv) {
            const int lx = lv % WTX, ly = (lv / WTX) % WTY, lz = lv / (WTX * WTY);
            const int hb = (lz * WHY + ly) * WHX + lx;
#pragma unroll
            for (int m = 0; m < MW; ++m) acc[m] += tin[(hb + toff[m]) * CIN + tci[m]] * tg[lv * COUT + tco[m]];
            if (threadIdx.x < COUT) bacc += tg[lv * COUT + threadIdx.x];
        }
    }
    A *dst = a.part + static_cast<long long>(blockIdx.x) * (NW + COUT);
#pragma unroll
    for (int m = 0; m < MW; ++m) {
        const int wi = threadIdx.x + 256 * m;
        if (wi < NW) dst[wi] = acc[m];
    }
    if (threadIdx.x < COUT) dst[NW + threadIdx.x] = bacc;
}

template <typename A>
__global__ void k_wgrad_reduce(const A *part, int nblk, int len, A *grad)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= len) return;
    A s = A(0);
    for (int b = 0; b < nblk; ++b) s += part[static_cast<long long>(b) * len + i];
    grad[i] = s;
}

// ---------------------------------------------------------------------------
// Loss, scalars, Adam, weight packing, pair assembly, random right-hand sides
// ---------------------------------------------------------------------------
constexpr int kRB = 256;

template <typename V>
__device__ inline V block_sum_t(V v, V *lds)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (l == 0) lds[w] = v;
    __syncthreads();
    V s = V(0);
    if (threadIdx.x == 0)
        for (int i = 0; i < static_cast<int>(blockDim.x >> 6); ++i) s += lds[i];
    __syncthreads();
    return s;   // valid in thread 0
}

// g = (2/n)(y - t) in the storage type; partial sums of (y - t)^2 (in double)
template <typename T, typename A>
__global__ __launch_bounds__(kRB) void k_mse(const A *y, const A *t, T *g, long long n, double *partials)
{
    __shared__ double lds[kRB / 64];
    double s = 0.0;
    const A sc = static_cast<A>(2.0 / static_cast<double>(n));
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const A d = y[c] - t[c];
        stv(g + c, sc * d);
        s += static_cast<double>(d) * static_cast<double>(d);
    }
    s = block_sum_t(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// energy norm of the unit stencil: loss partials of d.(L d), g = (2/n) L d
template <typename T, typename A>
__global__ __launch_bounds__(kRB) void k_energy(const A *y, const A *t, T *g, int nx, int ny, int nz,
                                                double *partials)
{
    __shared__ double lds[kRB / 64];
    const long long n = static_cast<long long>(nx) * ny * nz;
    const long long pl = static_cast<long long>(nx) * ny;
    double s = 0.0;
    const A sc = static_cast<A>(2.0 / static_cast<double>(n));
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int i = static_cast<int>(c % nx);
        const long long rest = c / nx;
        const int j = static_cast<int>(rest % ny), k = static_cast<int>(rest / ny);
        const A d = y[c] - t[c];
        A nb = A(0);
        if (i > 0) nb += y[c - 1] - t[c - 1];
        if (i + 1 < nx) nb += y[c + 1] - t[c + 1];
        if (j > 0) nb += y[c - nx] - t[c - nx];
        if (j + 1 < ny) nb += y[c + nx] - t[c + nx];
        if (k > 0) nb += y[c - pl] - t[c - pl];
        if (k + 1 < nz) nb += y[c + pl] - t[c + pl];
        const A ld = A(6) * d - nb;
        stv(g + c, sc * ld);
        s += static_cast<double>(d) * static_cast<double>(ld);
    }
    s = block_sum_t(s, lds);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

__global__ __launch_bounds__(kRB) void k_sum_partials(const double *partials, int np, double scale, double *out)
{
    __shared__ double lds[kRB / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += partials[i];
    s = block_sum_t(s, lds);
    if (threadIdx.x == 0) *out = s * scale;
}

// sigma = rms(r'/cbar) from the partial sums of r'^2
__global__ __launch_bounds__(kRB) void k_net_scalars(const double *partials, int np, double cbar, double n,
                                                     NetScalars *ns)
{
    __shared__ double lds[kRB / 64];
    double s = 0.0;
    for (int i = threadIdx.x; i < np; i += blockDim.x) s += partials[i];
    s = block_sum_t(s, lds);
    if (threadIdx.x == 0) {
        const double sigma = sqrt(s / n) / cbar;
        ns->sigma = sigma;
        ns->in_scale = sigma > 0.0 ? 1.0 / (cbar * sigma) : 0.0;
        ns->out_scale = sigma;
        ns->inv_sigma = sigma > 0.0 ? 1.0 / sigma : 0.0;
    }
}

template <typename A>
__global__ void k_adam(A *p, A *m, A *v, const A *g, int n, double lr, double b1, double b2, double eps,
                       double bc1, double bc2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const A gi = g[i];
    const A mi = static_cast<A>(b1) * m[i] + static_cast<A>(1.0 - b1) * gi;
    const A vi = static_cast<A>(b2) * v[i] + static_cast<A>(1.0 - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const A mh = mi / static_cast<A>(bc1), vh = vi / static_cast<A>(bc2);
    p[i] -= static_cast<A>(lr) * mh / (sqrt(vh) + static_cast<A>(eps));
}

// Storage copies of the master weights: plain (wst), flipped and transposed
// for the input gradient (wtr[t'][co][ci] = W[26-t'][ci][co]).
template <typename T, typename A>
__global__ void k_pack(const A *p, T *wst, T *wtr, LayerTable lt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= lt.total) return;
    stv(wst + i, p[i]);
    int l = 0;
    while (l < 3 && i >= lt.off[l + 1]) ++l;
    const int li = i - lt.off[l];
    const int cin = lt.cin[l], cout = lt.cout[l], nw = 27 * cin * cout;
    if (li >= nw) {
        stv(wtr + i, p[i]);
        return;
    }
    // wtr index li = (t' * cout + co) * cin + ci
    const int ci = li % cin, co = (li / cin) % cout, tq = li / (cin * cout);
    stv(wtr + i, p[lt.off[l] + ((26 - tq) * cin + ci) * cout + co]);
}

// MFMA A-operand fragments of a 16 -> 16 layer: fragment p, lane L, element e
// holds A[i][k] with i = L%16, k = 8*(L/16) + e, where row i is the output
// channel and k runs over (tap 2p + k/16, input channel k%16).  bwd = 1 builds
// the fragments of the flipped, transposed weights used by the input gradient.
__global__ void k_pack_frag(const float *p, int off, int bwd, uint16_t *frag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 14 * 64 * 8) return;
    const int e = i & 7, L = (i >> 3) & 63, pp = i >> 9;
    const int row = L & 15, kq = L >> 4;
    const int t = 2 * pp + (kq >> 1), c = 8 * (kq & 1) + e;
    float v = 0.f;
    if (t < 27) v = bwd ? p[off + ((26 - t) * 16 + row) * 16 + c] : p[off + (t * 16 + c) * 16 + row];
    frag[i] = f_to_bf16(v).bits;
}

// Pair assembly: input = T(r' * in_scale), target = (x* - x') / sigma.
template <typename T, typename A>
__global__ void k_pair_store(const double *rp, const double *xs, const double *xp, const NetScalars *ns, T *input,
                             A *target, long long n)
{
    const double is = ns->in_scale, ivs = ns->inv_sigma;
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        stv(input + c, static_cast<A>(rp[c] * is));
        target[c] = static_cast<A>((xs[c] - xp[c]) * ivs);
    }
}

// Uniform [-1, 1) doubles: SplitMix64 (Steele, Lea and Flood 2014) taken
// counter-style, value i = mix(seed + (i+1)*golden), top 53 bits.
__global__ void k_uniform_pm1(unsigned long long seed, long long n, double *out)
{
    for (long long c = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x; c < n;
         c += static_cast<long long>(gridDim.x) * blockDim.x) {
        unsigned long long z = seed + static_cast<unsigned long long>(c + 1) * 0x9E3779B97F4A7C15ull;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z = z ^ (z >> 31);
        out[c] = 2.0 * (static_cast<double>(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
void launch_conv16_mfma(const Conv16Args &a0, int epi, hipStream_t st)
{
    Conv16Args a = a0;
    const int gx = (a.nx + MTX - 1) / MTX, gy = (a.ny + MTY - 1) / MTY;
    int nzb = (2048 + gx * gy - 1) / (gx * gy);
    nzb = nzb < 1 ? 1 : nzb;
    int zc = (a.nz + nzb - 1) / nzb;
    zc = zc < 4 ? 4 : zc;
    zc = zc > a.nz ? a.nz : zc;
    a.zc = zc;
    const dim3 grid(gx, gy, (a.nz + zc - 1) / zc);
    if (epi == 0)
        hipLaunchKernelGGL(k_conv16_mfma<0>, grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_conv16_mfma<1>, grid, dim3(256), 0, st, a);
}

static int single_zc(int nx, int ny, int nz, int *gz)
{
    const int gx = (nx + STX - 1) / STX, gy = (ny + STY - 1) / STY;
    int nzb = (4096 + gx * gy - 1) / (gx * gy);
    nzb = nzb < 1 ? 1 : nzb;
    int zc = (nz + nzb - 1) / nzb;
    zc = zc < 4 ? 4 : zc;
    zc = zc > nz ? nz : zc;
    *gz = (nz + zc - 1) / zc;
    return zc;
}

void launch_in16_bf16(const In16Args &a0, int inm, int epi, hipStream_t st)
{
    In16Args a = a0;
    int gz = 1;
    a.zc = single_zc(a.nx, a.ny, a.nz, &gz);
    const dim3 grid((a.nx + STX - 1) / STX, (a.ny + STY - 1) / STY, gz);
    if (inm == 1)
        hipLaunchKernelGGL((k_in16_bf16<1, 0>), grid, dim3(256), 0, st, a);
    else if (epi == 0)
        hipLaunchKernelGGL((k_in16_bf16<0, 0>), grid, dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL((k_in16_bf16<0, 1>), grid, dim3(256), 0, st, a);
}

void launch_out16_bf16(const Out16Args &a0, int epi, hipStream_t st)
{
    Out16Args a = a0;
    int gz = 1;
    a.zc = single_zc(a.nx, a.ny, a.nz, &gz);
    const dim3 grid((a.nx + STX - 1) / STX, (a.ny + STY - 1) / STY, gz);
    if (epi == 2)
        hipLaunchKernelGGL(k_out16_bf16<2>, grid, dim3(256), 0, st, a, reinterpret_cast<const u32x4 *>(a.w));
    else
        hipLaunchKernelGGL(k_out16_bf16<3>, grid, dim3(256), 0, st, a, reinterpret_cast<const u32x4 *>(a.w));
}

template <typename T, typename A, int CIN, int COUT, int INM, int EPI>
void launch_conv_vec(const ConvVecArgs<T, A> &a, hipStream_t st)
{
    constexpr int TX = VecTile<A>::TX, TY = VecTile<A>::TY, TZ = VecTile<A>::TZ;
    const dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY, (a.nz + TZ - 1) / TZ);
    hipLaunchKernelGGL((k_conv_vec<T, A, CIN, COUT, INM, EPI>), grid, dim3(TX * TY * TZ), 0, st, a);
}

int wgrad_blocks(int nx, int ny, int nz)
{
    const long long nt = static_cast<long long>((nx + WTX - 1) / WTX) * ((ny + WTY - 1) / WTY) * ((nz + WTZ - 1) / WTZ);
    return static_cast<int>(nt < kWgradBlocks ? nt : kWgradBlocks);
}

template <typename T, typename A, int CIN, int COUT>
void launch_wgrad(const WgradArgs<T, A> &a, A *grad, hipStream_t st)
{
    const int nb = wgrad_blocks(a.nx, a.ny, a.nz);
    hipLaunchKernelGGL((k_wgrad<T, A, CIN, COUT>), dim3(nb), dim3(256), 0, st, a);
    const int len = 27 * CIN * COUT + COUT;
    hipLaunchKernelGGL(k_wgrad_reduce<A>, dim3((len + 255) / 256), dim3(256), 0, st, a.part, nb, len, grad);
}

template <typename T, typename A>
void launch_loss(int kind, const A *y, const A *t, T *g, int nx, int ny, int nz, double *partials, double *loss_out,
                 hipStream_t st)
{
    const long long n = static_cast<long long>(nx) * ny * nz;
    if (kind == NET_LOSS_ENERGY)
        hipLaunchKernelGGL((k_energy<T, A>), dim3(kLossBlocks), dim3(kRB), 0, st, y, t, g, nx, ny, nz, partials);
    else
        hipLaunchKernelGGL((k_mse<T, A>), dim3(kLossBlocks), dim3(kRB), 0, st, y, t, g, n, partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kRB), 0, st, partials, kLossBlocks,
                       1.0 / static_cast<double>(n), loss_out);
}

void launch_net_scalars(const double *partials, int np, double cbar, double n, NetScalars *ns, hipStream_t st)
{
    hipLaunchKernelGGL(k_net_scalars, dim3(1), dim3(kRB), 0, st, partials, np, cbar, n, ns);
}

template <typename A>
void launch_adam(A *p, A *m, A *v, const A *g, int n, double lr, double b1, double b2, double eps, double bc1,
                 double bc2, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam<A>, dim3((n + 255) / 256), dim3(256), 0, st, p, m, v, g, n, lr, b1, b2, eps, bc1, bc2);
}

template <typename T, typename A>
void launch_pack(const A *p, T *wst, T *wtr, const LayerTable &lt, hipStream_t st)
{
    hipLaunchKernelGGL((k_pack<T, A>), dim3((lt.total + 255) / 256), dim3(256), 0, st, p, wst, wtr, lt);
}

void launch_pack_frag(const float *p, int off, int bwd, uint16_t *frag, hipStream_t st)
{
    hipLaunchKernelGGL(k_pack_frag, dim3((14 * 64 * 8 + 255) / 256), dim3(256), 0, st, p, off, bwd, frag);
}

template <typename T, typename A>
void launch_pair_store(const double *rp, const double *xs, const double *xp, const NetScalars *ns, T *input,
                       A *target, long long n, hipStream_t st)
{
    hipLaunchKernelGGL((k_pair_store<T, A>), dim3(1024), dim3(256), 0, st, rp, xs, xp, ns, input, target, n);
}

void launch_uniform_pm1(unsigned long long seed, long long n, double *out, hipStream_t st)
{
    hipLaunchKernelGGL(k_uniform_pm1, dim3(1024), dim3(256), 0, st, seed, n, out);
}

// Instantiations ----------------------------------------------------------
#define NET_INST(T, A)                                                                                     \
    template void launch_wgrad<T, A, 1, 16>(const WgradArgs<T, A> &, A *, hipStream_t);                   \
    template void launch_wgrad<T, A, 16, 16>(const WgradArgs<T, A> &, A *, hipStream_t);                  \
    template void launch_wgrad<T, A, 16, 1>(const WgradArgs<T, A> &, A *, hipStream_t);                   \
    template void launch_loss<T, A>(int, const A *, const A *, T *, int, int, int, double *, double *,     \
                                    hipStream_t);                                                          \
    template void launch_adam<A>(A *, A *, A *, const A *, int, double, double, double, double, double,    \
                                 double, hipStream_t);                                                     \
    template void launch_pack<T, A>(const A *, T *, T *, const LayerTable &, hipStream_t);                 \
    template void launch_pair_store<T, A>(const double *, const double *, const double *, const NetScalars *, \
                                          T *, A *, long long, hipStream_t);
NET_INST(bf16, float)
NET_INST(double, double)
template void launch_conv_vec<double, double, 1, 16, 0, 0>(const ConvVecArgs<double, double> &, hipStream_t);
template void launch_conv_vec<double, double, 1, 16, 1, 0>(const ConvVecArgs<double, double> &, hipStream_t);
template void launch_conv_vec<double, double, 1, 16, 0, 1>(const ConvVecArgs<double, double> &, hipStream_t);
template void launch_conv_vec<double, double, 16, 1, 0, 2>(const ConvVecArgs<double, double> &, hipStream_t);
template void launch_conv_vec<double, double, 16, 1, 0, 3>(const ConvVecArgs<double, double> &, hipStream_t);
template void launch_conv_vec<double, double, 16, 16, 0, 0>(const ConvVecArgs<double, double> &, hipStream_t);
template void launch_conv_vec<double, double, 16, 16, 0, 1>(const ConvVecArgs<double, double> &, hipStream_t);

}  // namespace net
}  // namespace smg
