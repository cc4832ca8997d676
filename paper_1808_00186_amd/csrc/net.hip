// Learned initial guess for the Krylov solve (not in the paper): a small 3D
// U-Net on a 32^3 voxel grid over the mesh's bounding box maps
//   [log10 sigma, (x - x_s)/L, (y - y_s)/L, (z - z_s)/L, log10 f]
// to the secondary field E_s (Re/Im of x, y, z) at the voxel centres, scaled by
// 1 / (g |b|). The prediction is interpolated trilinearly to the edge
// midpoints and projected on the edge tangents (a DOF is the tangential
// component of E, Section 3) to give x0. The plain zero guess remains the
// fallback (petgem_solve rejects an x0 with |b - A x0| >= |b|).
//
// Layers (channels-last NDHWC, BF16 activations, FP32 accumulation):
//   c1 16->16 @32^3 relu | pool | c2 16->32 @16^3 relu | pool |
//   c3 32->64 @8^3 relu | c4 64->64 @8^3 relu | up, concat c2 |
//   c5 96->32 @16^3 relu | up, concat c1 | c6 48->16 @32^3 relu |
//   c7 16->16 @32^3 (linear; channels 0..5 are the output)
// Every convolution is 3x3x3, stride 1, zero padding 1, computed as an
// implicit GEMM on v_mfma_f32_16x16x32_bf16: M = voxels, N = output channels,
// K = 27 taps x input channels (each lane's 8 K values of a 32-wide chunk are
// 8 channels of one tap, 16 contiguous bytes). The backward data pass is the
// same kernel with the taps mirrored and the channel roles swapped; the
// backward weight pass is an MFMA reduction over voxels (v_mfma_f32_16x16x16_bf16,
// 4 voxels per lane) on voxel-quad interleaved copies of the layer input and
// its output gradient.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "device.h"
#include "internal.h"

namespace petgem {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
using bf16 = uint16_t;

constexpr int kSide = 32;
constexpr int kVox = kSide * kSide * kSide;
constexpr int kIn = 16, kOut = 16, kOutUsed = 6;

namespace {

__device__ __forceinline__ bf16 f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return 0x7fc0;   // NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                        // round to nearest even
    return (bf16)(u >> 16);
}

// 8 bf16 from LDS at a 16-byte aligned address (one 16-byte read), as the
// operand type of v_mfma_f32_16x16x32_bf16
__device__ __forceinline__ bf16x8 lds8(const bf16* p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const s16x8*>(p));
}

// ---------------------------------------------------------------- conv
// out[v][co] = sum_tap sum_ci in[v + off(tap)][ci] W[tap][ci][co] (+ bias, relu)
// in bf16 [B][D^3][CIN], wt bf16 [COUT][27*CIN] (K-contiguous per output
// channel), out bf16 or f32 [B][D^3][COUT].
// A block owns TY full x rows of one z plane (TY*D voxels, 16-voxel M tiles,
// MT per wave) and NTB 16-wide output tiles. For each of the three z offsets
// it stages in LDS the input rows y0-1 .. y0+TY of that plane (x padded by a
// zero column on both sides) and the nine taps of weights of that plane; the
// MFMA operands are then 8-byte LDS reads, each A fragment feeding NTB MFMAs
// and each weight fragment MT.
template <int CIN, int COUT, int D, int TY, int NTB>
struct ConvTile {
    static constexpr int MT = TY * D / 64;           // M tiles per wave
    static constexpr int HC = CIN + 8;               // halo voxel stride (bf16; 16-byte aligned rows)
    static constexpr int WK = 9 * CIN + 8;           // weight row stride (bf16; 16-byte aligned rows)
    static constexpr int HALO = (TY + 2) * (D + 2) * HC;
    static constexpr int WTS = 16 * NTB * WK;
    static_assert(TY * D % 64 == 0 && D % TY == 0 && COUT % (16 * NTB) == 0 && CIN % 16 == 0, "tile shape");
};

template <int CIN, int COUT, int D, int TY, int NTB, bool RELU, bool OUTF32>
__global__ void __launch_bounds__(256)
k_conv(const bf16* __restrict__ in, const bf16* __restrict__ wt, const float* __restrict__ bias,
       void* __restrict__ out) {
    using T = ConvTile<CIN, COUT, D, TY, NTB>;
    constexpr int MT = T::MT, HC = T::HC, WK = T::WK, K = 27 * CIN, Vs = D * D * D;
    __shared__ __align__(16) bf16 halo[T::HALO];
    __shared__ __align__(16) bf16 wl[T::WTS];
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
    const long v0 = (long)blockIdx.x * TY * D;
    const int b = (int)(v0 / Vs), r0 = (int)(v0 % Vs);
    const int z = r0 / (D * D), y0 = (r0 / D) % D;
    const int co0 = blockIdx.y * 16 * NTB;
    // LDS offsets of this lane's voxel in each of its M tiles (tile wave + 4 i)
    int aoff[MT];
#pragma unroll
    for (int i = 0; i < MT; ++i) {
        const int vb = (wave + 4 * i) * 16 + m;
        aoff[i] = ((vb / D) * (D + 2) + vb % D) * HC;
    }
    f32x4 acc[MT][NTB];
#pragma unroll
    for (int i = 0; i < MT; ++i)
#pragma unroll
        for (int t = 0; t < NTB; ++t) acc[i][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Staging of one z plane: the input rows y0-1 .. y0+TY of plane z+pz-1
    // (4 channels per uint2) and the weights of taps 9 pz .. 9 pz + 8 for this
    // block's output channels. The next plane's loads are issued into
    // registers before the current plane's MFMAs, so their latency overlaps
    // the compute; they go to LDS after the barrier that ends it.
    constexpr int Q = CIN / 4, HQ = (TY + 2) * (D + 2) * Q, NH = (HQ + 255) / 256;
    constexpr int WQ = 9 * CIN / 4, WQT = 16 * NTB * WQ, NW = (WQT + 255) / 256;
    uint2 hreg[NH], wreg[NW];
    auto fetch = [&](int pz) {
        const int zz = z + pz - 1;
#pragma unroll
        for (int j = 0; j < NH; ++j) {
            const int e = threadIdx.x + 256 * j;
            const int q = e % Q, vx = e / Q;
            const int rx = vx % (D + 2), ry = vx / (D + 2);
            const int yy = y0 - 1 + ry, xx = rx - 1;
            hreg[j] = make_uint2(0u, 0u);
            if (e < HQ && zz >= 0 && zz < D && yy >= 0 && yy < D && xx >= 0 && xx < D)
                hreg[j] = *reinterpret_cast<const uint2*>(in + ((long)b * Vs + ((long)zz * D + yy) * D + xx) * CIN + 4 * q);
        }
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const int e = threadIdx.x + 256 * j;
            if (e < WQT)
                wreg[j] = *reinterpret_cast<const uint2*>(wt + (long)(co0 + e / WQ) * K + pz * 9 * CIN + 4 * (e % WQ));
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int j = 0; j < NH; ++j) {
            const int e = threadIdx.x + 256 * j;
            if (e < HQ) *reinterpret_cast<uint2*>(halo + (e / Q) * HC + 4 * (e % Q)) = hreg[j];
        }
#pragma unroll
        for (int j = 0; j < NW; ++j) {
            const int e = threadIdx.x + 256 * j;
            if (e < WQT) *reinterpret_cast<uint2*>(wl + (e / WQ) * WK + 4 * (e % WQ)) = wreg[j];
        }
    };
    fetch(0);
    stage();
    __syncthreads();
    for (int pz = 0; pz < 3; ++pz) {
        if (pz < 2) fetch(pz + 1);
        // The plane's reduction index runs over its 9 taps x CIN channels,
        // tap-major (the order of a weight row), 32 at a time on
        // v_mfma_f32_16x16x32_bf16: lane kq takes indices 8 kq .. 8 kq + 7 of
        // the chunk, 8 channels of one tap (CIN is a multiple of 16), for both
        // operands; 9 CIN that is an odd multiple of 16 leaves 16, taken by
        // v_mfma_f32_16x16x16_bf16 (4 per lane).
        constexpr int KP = 9 * CIN, NK32 = KP / 32;
        constexpr int UNR = CIN >= 48 ? 1 : 3;   // wider inputs: keep two waves per SIMD
#pragma unroll UNR
        for (int kk = 0; kk < NK32; ++kk) {
            const int idx = 32 * kk + 8 * kq, tap = idx / CIN, ch = idx % CIN;
            const int sh = ((tap / 3) * (D + 2) + tap % 3) * HC + ch;   // (dy, dx) shift and channel in the halo
            bf16x8 a[MT], w[NTB];
#pragma unroll
            for (int i = 0; i < MT; ++i) a[i] = lds8(halo + aoff[i] + sh);
#pragma unroll
            for (int t = 0; t < NTB; ++t) w[t] = lds8(wl + (t * 16 + m) * WK + idx);
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int t = 0; t < NTB; ++t)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], w[t], acc[i][t], 0, 0, 0);
        }
        if constexpr (KP % 32 != 0) {
            const int idx = 32 * NK32 + 4 * kq, tap = idx / CIN, ch = idx % CIN;
            const int sh = ((tap / 3) * (D + 2) + tap % 3) * HC + ch;
            bf16x4 a[MT], w[NTB];
#pragma unroll
            for (int i = 0; i < MT; ++i) a[i] = *reinterpret_cast<const bf16x4*>(halo + aoff[i] + sh);
#pragma unroll
            for (int t = 0; t < NTB; ++t) w[t] = *reinterpret_cast<const bf16x4*>(wl + (t * 16 + m) * WK + idx);
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int t = 0; t < NTB; ++t)
                    acc[i][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], w[t], acc[i][t], 0, 0, 0);
        }
        __syncthreads();
        if (pz < 2) {
            stage();
            __syncthreads();
        }
    }
    // lane holds D[row voxel 4 kq + j][col co m] of every (M tile, output tile)
#pragma unroll
    for (int t = 0; t < NTB; ++t) {
        const int co = co0 + t * 16 + m;
        const float bb = bias ? bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < MT; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const long vo = v0 + (wave + 4 * i) * 16 + 4 * kq + j;
                float val = acc[i][t][j] + bb;
                if (RELU) val = fmaxf(val, 0.f);
                if (OUTF32) reinterpret_cast<float*>(out)[vo * COUT + co] = val;
                else reinterpret_cast<bf16*>(out)[vo * COUT + co] = f2bf(val);
            }
    }
}

// Voxel-quad interleaved copy of an activation: out[((v/4) C + c) 4 + v%4] =
// in[v][c]. A lane of the weight pass then reads 4 consecutive voxels of one
// channel as 8 contiguous bytes, and the 16 channels of a wave's fragment
// are adjacent. One thread moves 4 voxels x 4 channels.
template <int C>
__global__ void __launch_bounds__(256)
k_to_quads(const bf16* __restrict__ in, int nvox, bf16* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= nvox / 4 * (C / 4)) return;
    const int q = e / (C / 4), c = 4 * (e % (C / 4));
    uint2 w[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) w[j] = *reinterpret_cast<const uint2*>(in + (size_t)(4 * q + j) * C + c);
    // channel c + i of voxel 4q + j is half (i & 1) of word (i >> 1) of w[j]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t h[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const uint32_t word = (i >> 1) ? w[j].y : w[j].x;
            h[j] = (i & 1) ? (word >> 16) : (word & 0xffffu);
        }
        *reinterpret_cast<uint2*>(out + ((size_t)q * C + c + i) * 4) = make_uint2(h[0] | (h[1] << 16), h[2] | (h[3] << 16));
    }
}

// Backward weights and bias from voxel-quad interleaved copies inQ
// [B D^3 / 4][CIN][4] and dzQ [B D^3 / 4][COUT][4]:
//   partial[s][tap * CIN + ci][co] = sum over the voxels of split s of
//                                    in[v + off(tap)][ci] dz[v][co]
//   partial[s][27 CIN][co]         = sum over the same voxels of dz[v][co].
// The reduction index of v_mfma_f32_16x16x16_bf16 runs over voxels: a K step
// is 16 consecutive voxels, 4 per lane, all in one x row (D % 4 == 0). A
// block is one (16-channel input group, z offset) unit and one voxel split;
// its 4 waves take alternate K steps and are summed through LDS in wave
// order, so the result does not depend on timing. A wave keeps the 9 (y, x)
// offsets x all output tiles in registers: one 16-byte load per input row
// (x0-2 .. x0+5 of one channel) yields the three x shifts by funnel shifts.
template <int CIN, int COUT, int D>
__global__ void __launch_bounds__(256)
k_conv_bwdw(const bf16* __restrict__ inQ, const bf16* __restrict__ dzQ, float* __restrict__ partial,
            int nvox, int nsplit) {
    constexpr int NT = COUT / 16, KW = 27 * CIN, Vs = D * D * D;
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
    const int s = blockIdx.x % nsplit, unit = blockIdx.x / nsplit;
    const int g = unit / 3, pz = unit % 3;
    const bool bias_unit = unit == 1;   // g = 0, z offset 0
    const int nK = nvox / 16, chunk = (nK + nsplit - 1) / nsplit;
    const int k0 = s * chunk, k1 = min(nK, k0 + chunk);
    f32x4 acc[3][3][NT], accb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        accb[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[a][c][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const bf16x4 ones = {0x3f80, 0x3f80, 0x3f80, 0x3f80};
    // operands of one K step: dz fragments and, per y offset, the row words
    // x0-2 .. x0+5 of this lane's input channel
    struct Step {
        bf16x4 w[NT];
        uint32_t dp[3], d0[3], d1[3], dn[3];
    };
    auto load = [&](int k, Step& st) {
        const int v = 16 * k + 4 * kq;
        const int b = v / Vs, r = v % Vs;
        const int z = r / (D * D), y = (r / D) % D, x0 = r % D;
#pragma unroll
        for (int t = 0; t < NT; ++t)
            st.w[t] = *reinterpret_cast<const bf16x4*>(dzQ + ((long)(v / 4) * COUT + t * 16 + m) * 4);
        const int zz = z + pz - 1, ci = g * 16 + m;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const int yy = y + dy - 1;
            st.dp[dy] = st.d0[dy] = st.d1[dy] = st.dn[dy] = 0;
            if (zz >= 0 && zz < D && yy >= 0 && yy < D) {
                const long q = ((long)b * Vs + ((long)zz * D + yy) * D + x0) / 4;   // quad of x0 .. x0+3
                const uint2 c = *reinterpret_cast<const uint2*>(inQ + (q * CIN + ci) * 4);
                st.d0[dy] = c.x;
                st.d1[dy] = c.y;
                if (x0 > 0) st.dp[dy] = *reinterpret_cast<const uint32_t*>(inQ + ((q - 1) * CIN + ci) * 4 + 2);
                if (x0 + 4 < D) st.dn[dy] = *reinterpret_cast<const uint32_t*>(inQ + ((q + 1) * CIN + ci) * 4);
            }
        }
    };
    auto compute = [&](const Step& st) {
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            const uint32_t dp = st.dp[dy], d0 = st.d0[dy], d1 = st.d1[dy], dn = st.dn[dy];
            // voxels x0-1..x0+2, x0..x0+3, x0+1..x0+4 of this row
            const uint32_t lo[3] = {(dp >> 16) | (d0 << 16), d0, (d0 >> 16) | (d1 << 16)};
            const uint32_t hi[3] = {(d0 >> 16) | (d1 << 16), d1, (d1 >> 16) | (dn << 16)};
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                const bf16x4 a = __builtin_bit_cast(bf16x4, (u32x2{lo[dx], hi[dx]}));
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    acc[dy][dx][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, st.w[t], acc[dy][dx][t], 0, 0, 0);
            }
        }
        if (bias_unit) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
                accb[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ones, st.w[t], accb[t], 0, 0, 0);
        }
    };
    // the loads of the next two K steps are in flight during the MFMAs of this one
    Step s0, s1;
    int k = k0 + wave;
    if (k < k1) load(k, s0);
    if (k + 4 < k1) load(k + 4, s1);
    for (; k < k1; k += 4) {
        Step s2 = s1;
        if (k + 8 < k1) load(k + 8, s2);
        compute(s0);
        s0 = s1;
        s1 = s2;
    }
    // wave-ordered sum of the 4 waves, one output tile column at a time;
    // lane holds D[row ci = 4 kq + j][col co = m]
    __shared__ float red[4][10][256];
    float* base = partial + (long)s * (KW + 1) * COUT;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[wave][3 * a + c][4 * l + j] = acc[a][c][t][j];
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wave][9][4 * l + j] = accb[t][j];
        __syncthreads();
        for (int e = threadIdx.x; e < 10 * 256; e += 256) {
            const int tile = e / 256, ln = (e / 4) % 64, j = e % 4;
            const float val = red[0][tile][e % 256] + red[1][tile][e % 256] + red[2][tile][e % 256] +
                              red[3][tile][e % 256];
            const int co = t * 16 + (ln & 15), ci = g * 16 + 4 * (ln >> 4) + j;
            if (tile < 9) {
                const int tap = pz * 9 + tile;   // (z, y, x) offsets in row-major order
                base[(long)(tap * CIN + ci) * COUT + co] = val;
            } else if (bias_unit && ci == 0) {
                base[(long)KW * COUT + co] = val;
            }
        }
        __syncthreads();
    }
}

// The same weight and bias partials at side 32, with input rows reused
// along y. A column is (sample, z, 16-voxel x segment); a wave walks a
// column's D output rows and keeps the input rows y-1, y, y+1 of its z plane
// in registers, so each step loads one new input row (and the next row of
// dz) instead of three. Same units, splits, LDS reduction and partial layout
// as k_conv_bwdw; the bias unit adds the ones-operand MFMA.
template <int CIN, int COUT, int D>
__global__ void __launch_bounds__(256)
k_conv_bwdw_col(const bf16* __restrict__ inQ, const bf16* __restrict__ dzQ, float* __restrict__ partial,
                int ncol, int nsplit, int chunk) {
    constexpr int NT = COUT / 16, KW = 27 * CIN, Vs = D * D * D, XS = D / 16;
    static_assert(D % 16 == 0, "a column step is 16 voxels of one x row");
    const int wave = threadIdx.x >> 6, l = threadIdx.x & 63, m = l & 15, kq = l >> 4;
    const int s = blockIdx.x % nsplit, unit = blockIdx.x / nsplit;
    const int g = unit / 3, pz = unit % 3, ci = g * 16 + m;
    const bool bias_unit = unit == 1;   // g = 0, z offset 0
    const int c0 = s * chunk, c1 = min(ncol, c0 + chunk);   // chunk: columns per split, a multiple of 4
    f32x4 acc[3][3][NT], accb[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        accb[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c) acc[a][c][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    const bf16x4 ones = {0x3f80, 0x3f80, 0x3f80, 0x3f80};
    struct Row { uint32_t dp, d0, d1, dn; };   // x0-2 .. x0+5 of this lane's channel
    struct Frag { bf16x4 w[NT]; };
    for (int col = c0 + wave; col < c1; col += 4) {
        const int xs = col % XS, bz = col / XS, z = bz % D, b = bz / D;
        const int x0 = xs * 16 + 4 * kq, zz = z + pz - 1;
        const bool zok = zz >= 0 && zz < D;
        auto row = [&](int yy) {
            Row r{0u, 0u, 0u, 0u};
            if (zok && yy >= 0 && yy < D) {
                const long q = ((long)b * Vs + ((long)zz * D + yy) * D + x0) / 4;   // quad of x0 .. x0+3
                const uint2 c = *reinterpret_cast<const uint2*>(inQ + (q * CIN + ci) * 4);
                r.d0 = c.x;
                r.d1 = c.y;
                if (x0 > 0) r.dp = *reinterpret_cast<const uint32_t*>(inQ + ((q - 1) * CIN + ci) * 4 + 2);
                if (x0 + 4 < D) r.dn = *reinterpret_cast<const uint32_t*>(inQ + ((q + 1) * CIN + ci) * 4);
            }
            return r;
        };
        auto frag = [&](int y) {
            Frag f;
            const long q = ((long)b * Vs + ((long)z * D + y) * D + x0) / 4;
#pragma unroll
            for (int t = 0; t < NT; ++t) f.w[t] = *reinterpret_cast<const bf16x4*>(dzQ + (q * COUT + t * 16 + m) * 4);
            return f;
        };
        Row ra{0u, 0u, 0u, 0u}, rb = row(0), rc = row(1);
        Frag fc = frag(0);
        for (int y = 0; y < D; ++y) {
            const Row rn = row(y + 2);                        // zero past the last row
            const Frag fn = y + 1 < D ? frag(y + 1) : fc;
            const Row* rows[3] = {&ra, &rb, &rc};             // input rows y-1, y, y+1
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const uint32_t dp = rows[dy]->dp, d0 = rows[dy]->d0, d1 = rows[dy]->d1, dn = rows[dy]->dn;
                const uint32_t lo[3] = {(dp >> 16) | (d0 << 16), d0, (d0 >> 16) | (d1 << 16)};
                const uint32_t hi[3] = {(d0 >> 16) | (d1 << 16), d1, (d1 >> 16) | (dn << 16)};
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
                    const bf16x4 a = __builtin_bit_cast(bf16x4, (u32x2{lo[dx], hi[dx]}));
#pragma unroll
                    for (int t = 0; t < NT; ++t)
                        acc[dy][dx][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, fc.w[t], acc[dy][dx][t], 0, 0, 0);
                }
            }
            if (bias_unit) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    accb[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ones, fc.w[t], accb[t], 0, 0, 0);
            }
            ra = rb;
            rb = rc;
            rc = rn;
            fc = fn;
        }
    }
    __shared__ float red[4][10][256];
    float* base = partial + (long)s * (KW + 1) * COUT;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int j = 0; j < 4; ++j) red[wave][3 * a + c][4 * l + j] = acc[a][c][t][j];
#pragma unroll
        for (int j = 0; j < 4; ++j) red[wave][9][4 * l + j] = accb[t][j];
        __syncthreads();
        for (int e = threadIdx.x; e < 10 * 256; e += 256) {
            const int tile = e / 256, ln = (e / 4) % 64, j = e % 4;
            const float val = red[0][tile][e % 256] + red[1][tile][e % 256] + red[2][tile][e % 256] +
                              red[3][tile][e % 256];
            const int co = t * 16 + (ln & 15), cr = g * 16 + 4 * (ln >> 4) + j;
            if (tile < 9) {
                base[(long)((pz * 9 + tile) * CIN + cr) * COUT + co] = val;
            } else if (bias_unit && cr == 0) {
                base[(long)KW * COUT + co] = val;
            }
        }
        __syncthreads();
    }
}

// out[i] = sum over the nsplit partials of entry i: 16 interleaved groups of
// splits summed in split order, then the groups in a fixed tree order
// (deterministic). A block covers 64 entries with 1024 threads.
__global__ void __launch_bounds__(1024)
k_sum_splits(const float* __restrict__ partial, int nsplit, int n, float* __restrict__ out) {
    __shared__ float red[16][64];
    const int e = threadIdx.x & 63, q = threadIdx.x >> 6, i = blockIdx.x * 64 + e;
    float sum = 0.f;
    if (i < n)
        for (int k = q; k < nsplit; k += 16) sum += partial[(long)k * n + i];
    red[q][e] = sum;
    __syncthreads();
    for (int h = 8; h > 0; h >>= 1) {
        if (q < h) red[q][e] += red[q + h][e];
        __syncthreads();
    }
    if (q == 0 && i < n) out[i] = red[0][e];
}

// Elementwise kernels move 4 channels (8 bytes of bf16, 16 of f32) per
// thread; every channel count and offset is a multiple of 4.
__device__ __forceinline__ float4 ld_bf4(const bf16* p) {
    const uint2 w = *reinterpret_cast<const uint2*>(p);
    return make_float4(__uint_as_float(w.x << 16), __uint_as_float(w.x & 0xffff0000u), __uint_as_float(w.y << 16),
                       __uint_as_float(w.y & 0xffff0000u));
}
__device__ __forceinline__ void st_bf4(bf16* p, float4 v) {
    *reinterpret_cast<uint2*>(p) = make_uint2((uint32_t)f2bf(v.x) | ((uint32_t)f2bf(v.y) << 16),
                                              (uint32_t)f2bf(v.z) | ((uint32_t)f2bf(v.w) << 16));
}
// parent (coarse) voxel of fine voxel vf on a grid of side D
// (voxel and element counts stay below 2^31 for batch_max <= 256, so the
// index arithmetic of these kernels is 32-bit)
__device__ __forceinline__ int parent_of(int vf, int D) {
    const int Dc = D / 2, V = D * D * D;
    const int b = vf / V, r = vf % V;
    const int z = r / (D * D), y = (r / D) % D, x = r % D;
    return b * Dc * Dc * Dc + ((z / 2) * Dc + y / 2) * Dc + x / 2;
}
// q-th of the 8 children of coarse voxel vc (side Dc) on the fine grid
__device__ __forceinline__ int child_of(int vc, int Dc, int q) {
    const int D = 2 * Dc, Vc = Dc * Dc * Dc;
    const int b = vc / Vc, r = vc % Vc;
    const int z = r / (Dc * Dc), y = (r / Dc) % Dc, x = r % Dc;
    return b * D * D * D + ((2 * z + (q >> 2)) * D + 2 * y + ((q >> 1) & 1)) * D + 2 * x + (q & 1);
}

// 2x2x2 average pooling (fine side D), C channels
__global__ void k_pool(const bf16* __restrict__ in, int B, int D, int C, bf16* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int Dc = D / 2, C4 = C / 4;
    if (e >= B * Dc * Dc * Dc * C4) return;
    const int c = 4 * (e % C4), vc = e / C4;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int q = 0; q < 8; ++q) {
        const float4 v = ld_bf4(in + child_of(vc, Dc, q) * C + c);
        s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
    }
    st_bf4(out + vc * C + c, make_float4(0.125f * s.x, 0.125f * s.y, 0.125f * s.z, 0.125f * s.w));
}

// concatenation [nearest x2 upsampling of the coarse tensor (C1 channels) |
// skip tensor (C2 channels)] on the fine grid of side D
__global__ void k_up_concat(const bf16* __restrict__ coarse, int C1, const bf16* __restrict__ skip, int C2, int B,
                            int D, bf16* __restrict__ out) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int W4 = (C1 + C2) / 4;
    if (e >= B * D * D * D * W4) return;
    const int c = 4 * (e % W4), vf = e / W4;
    const uint2 w = c < C1 ? *reinterpret_cast<const uint2*>(coarse + parent_of(vf, D) * C1 + c)
                           : *reinterpret_cast<const uint2*>(skip + vf * C2 + (c - C1));
    *reinterpret_cast<uint2*>(out + vf * (C1 + C2) + c) = w;
}

// ReLU backward of the coarse half of an upsampling concatenation:
// dz[vc][c] = (y[vc][c] > 0) * sum over the 8 children of dq[child][c], c < C
__global__ void k_up_bwd_relu(const float* __restrict__ dq, int ldq, int B, int Dc, int C,
                              const bf16* __restrict__ y, bf16* __restrict__ dz) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int C4 = C / 4;
    if (e >= B * Dc * Dc * Dc * C4) return;
    const int c = 4 * (e % C4), vc = e / C4;
    float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int q = 0; q < 8; ++q) {
        const float4 v = *reinterpret_cast<const float4*>(dq + child_of(vc, Dc, q) * ldq + c);
        s.x += v.x; s.y += v.y; s.z += v.z; s.w += v.w;
    }
    const float4 a = ld_bf4(y + vc * C + c);
    st_bf4(dz + vc * C + c, make_float4(a.x > 0.f ? s.x : 0.f, a.y > 0.f ? s.y : 0.f, a.z > 0.f ? s.z : 0.f,
                                        a.w > 0.f ? s.w : 0.f));
}

// ReLU backward of a pooled activation that also feeds a skip connection:
// dz = (y > 0) * (dq[:, off:off+C] + dp[parent] / 8)
__global__ void k_skip_pool_bwd_relu(const float* __restrict__ dq, int ldq, int off, const float* __restrict__ dp,
                                     int B, int D, int C, const bf16* __restrict__ y, bf16* __restrict__ dz) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    const int C4 = C / 4;
    if (e >= B * D * D * D * C4) return;
    const int c = 4 * (e % C4), vf = e / C4;
    const float4 u = *reinterpret_cast<const float4*>(dq + vf * ldq + off + c);
    const float4 p = *reinterpret_cast<const float4*>(dp + parent_of(vf, D) * C + c);
    const float4 a = ld_bf4(y + vf * C + c);
    st_bf4(dz + vf * C + c, make_float4(a.x > 0.f ? u.x + 0.125f * p.x : 0.f, a.y > 0.f ? u.y + 0.125f * p.y : 0.f,
                                        a.z > 0.f ? u.z + 0.125f * p.z : 0.f, a.w > 0.f ? u.w + 0.125f * p.w : 0.f));
}

// dz = dy * (y > 0) as bf16 (ReLU backward; y is the stored activation)
__global__ void k_relu_bwd(const float* __restrict__ dy, const bf16* __restrict__ y, int n, bf16* __restrict__ dz) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n / 4) return;
    const float4 d = *reinterpret_cast<const float4*>(dy + 4 * e);
    const float4 a = ld_bf4(y + 4 * e);
    st_bf4(dz + 4 * e, make_float4(a.x > 0.f ? d.x : 0.f, a.y > 0.f ? d.y : 0.f, a.z > 0.f ? d.z : 0.f,
                                   a.w > 0.f ? d.w : 0.f));
}

// Mean squared error over the used output channels; dY = d loss / d Y (bf16)
__global__ void __launch_bounds__(256)
k_mse(const float* __restrict__ Y, const float* __restrict__ T, long nvox, double inv_count,
      bf16* __restrict__ dY, double* __restrict__ partial) {
    __shared__ double red[256];
    const long v = (long)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (v < nvox) {
        for (int c = 0; c < kOut; ++c) {
            float g = 0.f;
            if (c < kOutUsed) {
                const float d = Y[v * kOut + c] - T[v * kOutUsed + c];
                s += (double)d * d;
                g = (float)(2.0 * inv_count) * d;
            }
            dY[v * kOut + c] = f2bf(g);
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long n, float lr, float b1, float b2, float c1, float c2, float eps) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// FP32 master W[tap][ci][co] -> bf16 forward layout wt[co][tap*CIN+ci] and
// backward-data layout wtb[ci][tap'*COUT+co] with tap' = 26 - tap (mirrored).
__global__ void k_cast_w(const float* __restrict__ W, int CIN, int COUT, bf16* __restrict__ wt, bf16* __restrict__ wtb) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    const long n = 27L * CIN * COUT;
    if (e >= n) return;
    const int co = (int)(e % COUT);
    const int ci = (int)((e / COUT) % CIN);
    const int tap = (int)(e / ((long)COUT * CIN));
    const bf16 h = f2bf(W[e]);
    wt[(long)co * 27 * CIN + tap * CIN + ci] = h;
    wtb[(long)ci * 27 * COUT + (26 - tap) * COUT + co] = h;
}

// Network input channels at the voxel centres.
struct VoxSrc {
    double pos[3];
    double logf;
};
__global__ void k_voxelize(const double* __restrict__ sigma, long ldsig, const int32_t* __restrict__ vtet,
                           const VoxSrc* __restrict__ src, int B, double lo0, double lo1, double lo2,
                           double hv, double L, bf16* __restrict__ X) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)B * kVox) return;
    const int b = (int)(e / kVox), r = (int)(e % kVox);
    const int z = r / (kSide * kSide), y = (r / kSide) % kSide, x = r % kSide;
    const double cx = lo0 + (x + 0.5) * hv, cy = lo1 + (y + 0.5) * hv, cz = lo2 + (z + 0.5) * hv;
    bf16* o = X + e * kIn;
    o[0] = f2bf((float)log10(sigma[(long)b * ldsig + vtet[r]]));
    o[1] = f2bf((float)((cx - src[b].pos[0]) / L));
    o[2] = f2bf((float)((cy - src[b].pos[1]) / L));
    o[3] = f2bf((float)((cz - src[b].pos[2]) / L));
    o[4] = f2bf((float)src[b].logf);
    for (int c = 5; c < kIn; ++c) o[c] = 0;
}

// E_s at the voxel centres from solution DOFs, scaled: T[b][v][6] (training targets)
__global__ void k_vox_field(const double* __restrict__ xyz, const int4* __restrict__ tets,
                            const int32_t* __restrict__ vtet, const int32_t* __restrict__ vdof,
                            const double2* __restrict__ sol, int n_dof, int B, const double* __restrict__ scale,
                            double lo0, double lo1, double lo2, double hv, float* __restrict__ T) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)B * kVox) return;
    const int b = (int)(e / kVox), r = (int)(e % kVox);
    const int z = r / (kSide * kSide), y = (r / kSide) % kSide, x = r % kSide;
    const double p[3] = {lo0 + (x + 0.5) * hv, lo1 + (y + 0.5) * hv, lo2 + (z + 0.5) * hv};
    TetGeom G;
    tet_geometry(xyz, tets[vtet[r]], G);
    double lam[4] = {0.0, 0.0, 0.0, 0.0};
    for (int v = 1; v < 4; ++v)
        for (int k = 0; k < 3; ++k) lam[v] += G.g[v][k] * (p[k] - G.X[0][k]);
    lam[0] = 1.0 - lam[1] - lam[2] - lam[3];
    constexpr int E0[6] = {0, 0, 0, 1, 3, 2};
    constexpr int E1[6] = {1, 2, 3, 2, 1, 3};
    double2 es[3] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0)};
    for (int i = 0; i < 6; ++i) {
        const int d = vdof[6 * r + i];
        if (d < 0) continue;
        const double2 val = sol[(long)b * n_dof + d];
        for (int k = 0; k < 3; ++k) {
            const double nk = G.sl[i] * (lam[E0[i]] * G.g[E1[i]][k] - lam[E1[i]] * G.g[E0[i]][k]);
            es[k].x += nk * val.x;
            es[k].y += nk * val.y;
        }
    }
    const double s = 1.0 / scale[b];
    float* o = T + e * kOutUsed;
    for (int k = 0; k < 3; ++k) {
        o[2 * k] = (float)(es[k].x * s);
        o[2 * k + 1] = (float)(es[k].y * s);
    }
}

// x0[b][d] = scale_b * (E(mid_d) . t_d) with E trilinear in the voxel-centre grid
__global__ void k_grid_to_edges(const float* __restrict__ Y, int B, int n_dof, const double* __restrict__ mid,
                                const double* __restrict__ tan, const double* __restrict__ scale, double lo0,
                                double lo1, double lo2, double hv, double2* __restrict__ x0) {
    const long e = (long)blockIdx.x * 256 + threadIdx.x;
    if (e >= (long)B * n_dof) return;
    const int b = (int)(e / n_dof), d = (int)(e % n_dof);
    const double lo[3] = {lo0, lo1, lo2};
    int i0[3];
    double w[3];
    for (int k = 0; k < 3; ++k) {
        double u = (mid[3 * d + k] - lo[k]) / hv - 0.5;
        u = fmin(fmax(u, 0.0), (double)(kSide - 1));
        int i = (int)floor(u);
        if (i > kSide - 2) i = kSide - 2;
        i0[k] = i;
        w[k] = u - i;
    }
    double f[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 8; ++q) {
        const int dx = q & 1, dy = (q >> 1) & 1, dz = (q >> 2) & 1;
        const double wt = (dx ? w[0] : 1 - w[0]) * (dy ? w[1] : 1 - w[1]) * (dz ? w[2] : 1 - w[2]);
        const long v = (long)b * kVox + ((long)(i0[2] + dz) * kSide + i0[1] + dy) * kSide + i0[0] + dx;
        for (int c = 0; c < 6; ++c) f[c] += wt * Y[v * kOut + c];
    }
    const double s = scale[b];
    const double tx = tan[3 * d], ty = tan[3 * d + 1], tz = tan[3 * d + 2];
    x0[e] = make_double2(s * (f[0] * tx + f[2] * ty + f[4] * tz), s * (f[1] * tx + f[3] * ty + f[5] * tz));
}

__global__ void __launch_bounds__(256) k_vnorm(const double2* __restrict__ b, int n, double* __restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += cabs2(b[i]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = sqrt(red[0]);
}

}  // namespace

// ------------------------------------------------------------------ host

struct NetLayer {
    int cin, cout, side;
    bool relu;
    size_t w_off, b_off;   // offsets into the parameter vector (floats)
    bf16* wt = nullptr;    // forward layout
    bf16* wtb = nullptr;   // backward-data layout
};

}  // namespace petgem

struct petgem_net {
    int batch_max = 0;
    std::vector<petgem::NetLayer> L;
    size_t nparam = 0;
    float *P = nullptr, *Gr = nullptr, *M = nullptr, *Vv = nullptr;
    int step = 0;
    // activations (bf16) and gradients (f32) for batch_max samples
    petgem::bf16 *X0 = nullptr, *A1 = nullptr, *P1 = nullptr, *A2 = nullptr, *P2 = nullptr, *A3 = nullptr,
                 *A4 = nullptr, *Q2 = nullptr, *A5 = nullptr, *Q1 = nullptr, *A6 = nullptr, *dzb = nullptr;
    float* Y = nullptr;
    float *g0 = nullptr, *g1 = nullptr, *g2 = nullptr;   // f32 gradient scratch
    float* wpart = nullptr;                              // backward-weight partials
    petgem::bf16 *tin = nullptr, *tdz = nullptr;         // voxel-quad copies for the weight pass
    double* lpart = nullptr;
    float* T = nullptr;       // targets of the current batch (caller-owned copy not needed)
    double* scal = nullptr;   // per-sample scales on device
    petgem::VoxSrc* vsrc = nullptr;
    double* lpart_h = nullptr;
    double2* bbuf = nullptr;   // right-hand side scratch of petgem_learned_x0
    size_t bcap = 0;
    double* bn = nullptr;      // [batch_max] |b|
};

namespace petgem {

namespace {

inline dim3 g1(long n) { return dim3((unsigned)((n + 255) / 256)); }

// voxel splits of the weight pass: enough blocks to fill the chip. At sides
// 8 and 16 a split is a range of 16-voxel K steps, at least 8 per wave; at
// side 32 it is a range of (sample, z, x segment) columns, a multiple of 4
// so that the 4 waves of a block get the same number.
int bwdw_target(int cin) { return std::max(1, ceil_div(1024, 3 * (cin / 16))); }
long bwdw_col_chunk(int cin, long ncol) {
    const long t = bwdw_target(cin);
    return 4 * std::max(1L, (ncol + 4 * t - 1) / (4 * t));
}
int bwdw_splits(int cin, long nvox, int D) {
    const int target = bwdw_target(cin);
    if (D == 32) {
        const long ncol = nvox / D / 16, chunk = bwdw_col_chunk(cin, ncol);
        return (int)((ncol + chunk - 1) / chunk);
    }
    const long cap = std::max(1L, nvox / 16 / 32);
    return (int)std::min<long>(cap, target);
}
size_t wpart_floats(int cin, int cout, long nvox, int D) {
    return (size_t)bwdw_splits(cin, nvox, D) * (27 * (size_t)cin + 1) * cout;
}

template <int CIN, int COUT, int D, int TY, int NTB>
void conv_t(bool relu, bool outf32, const bf16* in, const bf16* wt, const float* bias, void* out, int nvox,
            hipStream_t s) {
    const dim3 grid((unsigned)(nvox / (TY * D)), COUT / (16 * NTB));
    if (outf32) hipLaunchKernelGGL((k_conv<CIN, COUT, D, TY, NTB, false, true>), grid, dim3(256), 0, s, in, wt, bias, out);
    else if (relu) hipLaunchKernelGGL((k_conv<CIN, COUT, D, TY, NTB, true, false>), grid, dim3(256), 0, s, in, wt, bias, out);
    else hipLaunchKernelGGL((k_conv<CIN, COUT, D, TY, NTB, false, false>), grid, dim3(256), 0, s, in, wt, bias, out);
}

// forward/backward-data convolution dispatch on the (CIN, COUT, side) triples
// of the network; nvox = B side^3
int conv(int cin, int cout, bool relu, bool outf32, const bf16* in, const bf16* wt, const float* bias, void* out,
         int nvox, int D, hipStream_t s) {
#define PG_CV(A, B, SIDE, TY, NTB)                                                     \
    if (cin == A && cout == B && D == SIDE) {                                          \
        conv_t<A, B, SIDE, TY, NTB>(relu, outf32, in, wt, bias, out, nvox, s);         \
        return PETGEM_OK;                                                              \
    }
    PG_CV(16, 16, 32, 8, 1) PG_CV(48, 16, 32, 8, 1) PG_CV(16, 48, 32, 8, 3)
    PG_CV(16, 32, 16, 8, 2) PG_CV(96, 32, 16, 8, 1) PG_CV(32, 96, 16, 8, 3) PG_CV(32, 16, 16, 8, 1)
    PG_CV(32, 64, 8, 8, 1) PG_CV(64, 64, 8, 8, 1) PG_CV(64, 32, 8, 8, 1)
#undef PG_CV
    set_error("unsupported convolution shape");
    return PETGEM_INVALID_ARG;
}

int to_quads(int c, const bf16* in, int nvox, bf16* out, hipStream_t s) {
#define PG_TQ(C)                                                                                    \
    if (c == C) {                                                                                   \
        hipLaunchKernelGGL((k_to_quads<C>), g1(nvox / 4 * (C / 4)), dim3(256), 0, s, in, nvox, out); \
        return PETGEM_OK;                                                                           \
    }
    PG_TQ(16) PG_TQ(32) PG_TQ(48) PG_TQ(64) PG_TQ(96)
#undef PG_TQ
    set_error("unsupported channel count");
    return PETGEM_INVALID_ARG;
}

int conv_bwdw(int cin, int cout, const bf16* inQ, const bf16* dzQ, float* part, int nvox, int D, int nsplit,
              hipStream_t s) {
    const int nb = 3 * (cin / 16) * nsplit;
    const int ncol = nvox / D / 16, chunk = (int)bwdw_col_chunk(cin, ncol);
#define PG_BW(A, B, SIDE)                                                                                     \
    if (cin == A && cout == B && D == SIDE) {                                                                 \
        hipLaunchKernelGGL((k_conv_bwdw<A, B, SIDE>), dim3(nb), dim3(256), 0, s, inQ, dzQ, part, nvox, nsplit); \
        return PETGEM_OK;                                                                                     \
    }
#define PG_BWC(A, B, SIDE)                                                                                         \
    if (cin == A && cout == B && D == SIDE) {                                                                      \
        hipLaunchKernelGGL((k_conv_bwdw_col<A, B, SIDE>), dim3(nb), dim3(256), 0, s, inQ, dzQ, part, ncol, nsplit, \
                           chunk);                                                                                 \
        return PETGEM_OK;                                                                                          \
    }
    PG_BWC(16, 16, 32) PG_BW(16, 32, 16) PG_BW(32, 64, 8) PG_BW(64, 64, 8) PG_BW(96, 32, 16) PG_BWC(48, 16, 32)
#undef PG_BW
#undef PG_BWC
    set_error("unsupported convolution shape");
    return PETGEM_INVALID_ARG;
}

// SplitMix64 + Box-Muller: seeded, platform-independent initial weights
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9e3779b97f4a7c15ull);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u = uniform(), v = uniform();
        return std::sqrt(-2.0 * std::log(u)) * std::cos(2.0 * kPi * v);
    }
};

void release_net(petgem_net* n) {
    for (auto& l : n->L) { dfree(l.wt); dfree(l.wtb); }
    dfree(n->P); dfree(n->Gr); dfree(n->M); dfree(n->Vv);
    dfree(n->X0); dfree(n->A1); dfree(n->P1); dfree(n->A2); dfree(n->P2); dfree(n->A3); dfree(n->A4);
    dfree(n->Q2); dfree(n->A5); dfree(n->Q1); dfree(n->A6); dfree(n->dzb); dfree(n->Y);
    dfree(n->g0); dfree(n->g1); dfree(n->g2); dfree(n->wpart); dfree(n->tin); dfree(n->tdz); dfree(n->lpart); dfree(n->T);
    dfree(n->scal); dfree(n->vsrc); dfree(n->bbuf); dfree(n->bn);
    if (n->lpart_h) (void)hipHostFree(n->lpart_h);
    n->lpart_h = nullptr;
}

int cast_weights(petgem_net* n, hipStream_t s) {
    for (auto& l : n->L)
        hipLaunchKernelGGL(k_cast_w, g1(27L * l.cin * l.cout), dim3(256), 0, s, n->P + l.w_off, l.cin, l.cout, l.wt,
                           l.wtb);
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

// Forward pass on X0 (already filled) for B samples; output Y f32 [B][32^3][16].
int forward(petgem_net* n, int B, hipStream_t s) {
    const int v32 = B * kVox, v16 = B * kVox / 8, v8 = B * kVox / 64;
    auto& L = n->L;
    PG_TRY(conv(16, 16, true, false, n->X0, L[0].wt, n->P + L[0].b_off, n->A1, v32, 32, s));
    hipLaunchKernelGGL(k_pool, g1((long)v16 * 4), dim3(256), 0, s, n->A1, B, 32, 16, n->P1);
    PG_TRY(conv(16, 32, true, false, n->P1, L[1].wt, n->P + L[1].b_off, n->A2, v16, 16, s));
    hipLaunchKernelGGL(k_pool, g1((long)v8 * 8), dim3(256), 0, s, n->A2, B, 16, 32, n->P2);
    PG_TRY(conv(32, 64, true, false, n->P2, L[2].wt, n->P + L[2].b_off, n->A3, v8, 8, s));
    PG_TRY(conv(64, 64, true, false, n->A3, L[3].wt, n->P + L[3].b_off, n->A4, v8, 8, s));
    hipLaunchKernelGGL(k_up_concat, g1((long)v16 * 24), dim3(256), 0, s, n->A4, 64, n->A2, 32, B, 16, n->Q2);
    PG_TRY(conv(96, 32, true, false, n->Q2, L[4].wt, n->P + L[4].b_off, n->A5, v16, 16, s));
    hipLaunchKernelGGL(k_up_concat, g1((long)v32 * 12), dim3(256), 0, s, n->A5, 32, n->A1, 16, B, 32, n->Q1);
    PG_TRY(conv(48, 16, true, false, n->Q1, L[5].wt, n->P + L[5].b_off, n->A6, v32, 32, s));
    PG_TRY(conv(16, 16, false, true, n->A6, L[6].wt, n->P + L[6].b_off, n->Y, v32, 32, s));
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

// weight and bias gradients of layer li from its input `in` and dz (bf16,
// channels-last); the bias gradient lands right after the weights (b_off =
// w_off + 27 cin cout)
int layer_grads(petgem_net* n, int li, const bf16* in, const bf16* dz, int nvox, int D, hipStream_t s) {
    const NetLayer& l = n->L[li];
    PG_TRY(to_quads(l.cin, in, nvox, n->tin, s));
    PG_TRY(to_quads(l.cout, dz, nvox, n->tdz, s));
    const int ns = bwdw_splits(l.cin, nvox, D);
    PG_TRY(conv_bwdw(l.cin, l.cout, n->tin, n->tdz, n->wpart, nvox, D, ns, s));
    const int nw = (27 * l.cin + 1) * l.cout;
    hipLaunchKernelGGL(k_sum_splits, dim3(ceil_div(nw, 64)), dim3(1024), 0, s, n->wpart, ns, nw, n->Gr + l.w_off);
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

// Backward pass from dY (bf16 in n->dzb, layout [B][32^3][16]); fills n->Gr.
int backward(petgem_net* n, int B, hipStream_t s) {
    const int v32 = B * kVox, v16 = B * kVox / 8, v8 = B * kVox / 64;
    auto& L = n->L;
    bf16* dz = n->dzb;
    float *g0 = n->g0, *g1b = n->g1, *g2 = n->g2;
    // c7 (linear): dz = dY
    PG_TRY(layer_grads(n, 6, n->A6, dz, v32, 32, s));
    PG_TRY(conv(16, 16, false, true, dz, L[6].wtb, nullptr, g0, v32, 32, s));                  // dA6
    hipLaunchKernelGGL(k_relu_bwd, g1((long)v32 * 4), dim3(256), 0, s, g0, n->A6, v32 * 16, dz);
    // c6
    PG_TRY(layer_grads(n, 5, n->Q1, dz, v32, 32, s));
    PG_TRY(conv(16, 48, false, true, dz, L[5].wtb, nullptr, g0, v32, 32, s));                  // dQ1 [v32][48]
    // dA5 from the upsampled half of dQ1; g0 keeps dQ1's skip half for dA1
    // until c2's backward
    hipLaunchKernelGGL(k_up_bwd_relu, g1((long)v16 * 8), dim3(256), 0, s, g0, 48, B, 16, 32, n->A5, dz);
    // c5
    PG_TRY(layer_grads(n, 4, n->Q2, dz, v16, 16, s));
    PG_TRY(conv(32, 96, false, true, dz, L[4].wtb, nullptr, g1b, v16, 16, s));                 // dQ2 [v16][96]
    hipLaunchKernelGGL(k_up_bwd_relu, g1((long)v8 * 16), dim3(256), 0, s, g1b, 96, B, 8, 64, n->A4, dz);   // dA4
    // c4
    PG_TRY(layer_grads(n, 3, n->A3, dz, v8, 8, s));
    PG_TRY(conv(64, 64, false, true, dz, L[3].wtb, nullptr, g2, v8, 8, s));                    // dA3
    hipLaunchKernelGGL(k_relu_bwd, g1((long)v8 * 16), dim3(256), 0, s, g2, n->A3, v8 * 64, dz);
    // c3
    PG_TRY(layer_grads(n, 2, n->P2, dz, v8, 8, s));
    float* dP2 = g2;   // [v8][32]
    PG_TRY(conv(64, 32, false, true, dz, L[2].wtb, nullptr, dP2, v8, 8, s));
    // dA2 = skip half of dQ2 (channels 64..95) + pool backward of dP2
    hipLaunchKernelGGL(k_skip_pool_bwd_relu, g1((long)v16 * 8), dim3(256), 0, s, g1b, 96, 64, dP2, B, 16, 32, n->A2,
                       dz);
    // c2
    PG_TRY(layer_grads(n, 1, n->P1, dz, v16, 16, s));
    float* dP1 = g1b;  // [v16][16]
    PG_TRY(conv(32, 16, false, true, dz, L[1].wtb, nullptr, dP1, v16, 16, s));
    // dA1 = skip half of dQ1 (channels 32..47) + pool backward of dP1
    hipLaunchKernelGGL(k_skip_pool_bwd_relu, g1((long)v32 * 4), dim3(256), 0, s, g0, 48, 32, dP1, B, 32, 16, n->A1,
                       dz);
    // c1
    PG_TRY(layer_grads(n, 0, n->X0, dz, v32, 32, s));
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

int loss_and_grads(petgem_net* n, const float* T, int B, hipStream_t s, double* loss) {
    PG_TRY(forward(n, B, s));
    const long nv = (long)B * kVox;
    const int nb = (int)((nv + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(nb), dim3(256), 0, s, n->Y, T, nv, 1.0 / ((double)nv * kOutUsed), n->dzb, n->lpart);
    PG_TRY(backward(n, B, s));
    PG_HIP(hipMemcpyAsync(n->lpart_h, n->lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (int i = 0; i < nb; ++i) sum += n->lpart_h[i];
    if (loss) *loss = sum / ((double)nv * kOutUsed);
    return PETGEM_OK;
}

// Voxel -> element map and voxel DOFs of a system (host location, cached)
int ensure_vox(petgem_system* sys) {
    if (sys->vox_tet) return PETGEM_OK;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int32_t v = 0; v < sys->n_nodes; ++v)
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], sys->xyz_h[3 * (size_t)v + k]);
            hi[k] = std::max(hi[k], sys->xyz_h[3 * (size_t)v + k]);
        }
    const double side = std::max(hi[0] - lo[0], std::max(hi[1] - lo[1], hi[2] - lo[2]));
    for (int k = 0; k < 3; ++k) sys->vox_lo[k] = lo[k];
    sys->vox_h = side / kSide;
    sys->vox_L = 0.5 * side;
    std::vector<double> pts(3 * (size_t)kVox);
    for (int r = 0; r < kVox; ++r) {
        const int z = r / (kSide * kSide), y = (r / kSide) % kSide, x = r % kSide;
        pts[3 * r] = lo[0] + (x + 0.5) * sys->vox_h;
        pts[3 * r + 1] = lo[1] + (y + 0.5) * sys->vox_h;
        pts[3 * r + 2] = lo[2] + (z + 0.5) * sys->vox_h;
    }
    std::vector<int32_t> tet(kVox);
    locate_points(sys->n_tets, sys->xyz_h.data(), sys->tets_h.data(), pts.data(), kVox, 1e-12, tet.data());
    std::vector<int32_t> dof(6 * (size_t)kVox);
    for (int r = 0; r < kVox; ++r) {
        if (tet[r] < 0) {
            set_error("a voxel centre lies outside the mesh (the grid covers the bounding box)");
            return PETGEM_RECEIVER_OUTSIDE;
        }
        for (int i = 0; i < 6; ++i) dof[6 * r + i] = sys->elem_dof_h[6 * (size_t)tet[r] + i];
    }
    // DOF midpoints and unit tangents for the grid -> edge interpolation
    const int n = sys->n_dof;
    std::vector<double> mid(3 * (size_t)n), tan(3 * (size_t)n);
    for (int d = 0; d < n; ++d) {
        const double* a = &sys->xyz_h[3 * (size_t)sys->dof_nodes_h[2 * d]];
        const double* b = &sys->xyz_h[3 * (size_t)sys->dof_nodes_h[2 * d + 1]];
        double t[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double ln = std::sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
        for (int k = 0; k < 3; ++k) {
            mid[3 * d + k] = 0.5 * (a[k] + b[k]);
            tan[3 * d + k] = t[k] / ln;
        }
    }
    PG_TRY(dalloc(&sys->vox_tet, (size_t)kVox));
    PG_TRY(dalloc(&sys->vox_dof, 6 * (size_t)kVox));
    PG_TRY(dalloc(&sys->dof_mid, 3 * (size_t)n));
    PG_TRY(dalloc(&sys->dof_tan, 3 * (size_t)n));
    PG_HIP(hipMemcpy(sys->vox_tet, tet.data(), sizeof(int32_t) * kVox, hipMemcpyHostToDevice));
    PG_HIP(hipMemcpy(sys->vox_dof, dof.data(), sizeof(int32_t) * 6 * kVox, hipMemcpyHostToDevice));
    PG_HIP(hipMemcpy(sys->dof_mid, mid.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    PG_HIP(hipMemcpy(sys->dof_tan, tan.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice));
    return PETGEM_OK;
}

int upload_vsrc(petgem_net* n, const petgem_source* src, int B, hipStream_t s) {
    std::vector<VoxSrc> v(B);
    for (int b = 0; b < B; ++b) {
        for (int k = 0; k < 3; ++k) v[b].pos[k] = src[b].pos[k];
        v[b].logf = std::log10(src[b].freq_hz);
    }
    PG_HIP(hipMemcpyAsync(n->vsrc, v.data(), sizeof(VoxSrc) * B, hipMemcpyHostToDevice, s));
    PG_HIP(hipStreamSynchronize(s));
    return PETGEM_OK;
}

}  // namespace

}  // namespace petgem

using namespace petgem;

extern "C" {

int petgem_net_create(int32_t batch_max, uint64_t seed, petgem_net** out) {
    if (!out || batch_max <= 0 || batch_max > 256) {
        set_error("net: 1 <= batch_max <= 256 and an output handle are required");
        return PETGEM_INVALID_ARG;
    }
    *out = nullptr;
    petgem_net* n = new (std::nothrow) petgem_net();
    if (!n) { set_error("host allocation failed"); return PETGEM_OUT_OF_MEMORY; }
    n->batch_max = batch_max;
    const int spec[7][4] = {{16, 16, 32, 1}, {16, 32, 16, 1}, {32, 64, 8, 1}, {64, 64, 8, 1},
                            {96, 32, 16, 1}, {48, 16, 32, 1}, {16, 16, 32, 0}};
    size_t off = 0;
    for (auto& sp : spec) {
        NetLayer l;
        l.cin = sp[0]; l.cout = sp[1]; l.side = sp[2]; l.relu = sp[3] != 0;
        l.w_off = off;
        off += 27 * (size_t)l.cin * l.cout;
        l.b_off = off;
        off += l.cout;
        n->L.push_back(l);
    }
    n->nparam = off;
    auto fail = [&](int rc) { release_net(n); delete n; return rc; };
    int rc;
    if ((rc = dalloc(&n->P, off)) || (rc = dalloc(&n->Gr, off)) || (rc = dalloc(&n->M, off)) ||
        (rc = dalloc(&n->Vv, off)))
        return fail(rc);
    for (auto& l : n->L)
        if ((rc = dalloc(&l.wt, 27 * (size_t)l.cin * l.cout)) || (rc = dalloc(&l.wtb, 27 * (size_t)l.cin * l.cout)))
            return fail(rc);
    const size_t v32 = (size_t)batch_max * kVox, v16 = v32 / 8, v8 = v32 / 64;
    if ((rc = dalloc(&n->X0, v32 * 16)) || (rc = dalloc(&n->A1, v32 * 16)) || (rc = dalloc(&n->P1, v16 * 16)) ||
        (rc = dalloc(&n->A2, v16 * 32)) || (rc = dalloc(&n->P2, v8 * 32)) || (rc = dalloc(&n->A3, v8 * 64)) ||
        (rc = dalloc(&n->A4, v8 * 64)) || (rc = dalloc(&n->Q2, v16 * 96)) || (rc = dalloc(&n->A5, v16 * 32)) ||
        (rc = dalloc(&n->Q1, v32 * 48)) || (rc = dalloc(&n->A6, v32 * 16)) || (rc = dalloc(&n->dzb, v32 * 48)) ||
        (rc = dalloc(&n->Y, v32 * 16)) || (rc = dalloc(&n->g0, v32 * 48)) || (rc = dalloc(&n->g1, v16 * 96)) ||
        (rc = dalloc(&n->g2, v32 * 16)) || (rc = dalloc(&n->T, v32 * kOutUsed)) ||
        (rc = dalloc(&n->scal, (size_t)batch_max)) || (rc = dalloc(&n->vsrc, (size_t)batch_max)) ||
        (rc = dalloc(&n->bn, (size_t)batch_max)))
        return fail(rc);
    size_t wp = 0;   // the largest split count over every batch size up to batch_max
    for (auto& l : n->L)
        for (int bb = 1; bb <= batch_max; ++bb)
            wp = std::max(wp, wpart_floats(l.cin, l.cout, (long)bb * l.side * l.side * l.side, l.side));
    if ((rc = dalloc(&n->wpart, wp)) || (rc = dalloc(&n->tin, v32 * 48)) || (rc = dalloc(&n->tdz, v32 * 16)) || (rc = dalloc(&n->lpart, (size_t)ceil_div((int64_t)v32, 256))))
        return fail(rc);
    if (hipHostMalloc(reinterpret_cast<void**>(&n->lpart_h), sizeof(double) * ceil_div((int64_t)v32, 256)) != hipSuccess)
        return fail(PETGEM_OUT_OF_MEMORY);
    // He-normal weights (the linear output layer scaled by 0.1, so that the
    // untrained network predicts nearly zero), zero biases, zero Adam moments
    std::vector<float> h(off, 0.f);
    Rng rng{seed};
    for (auto& l : n->L) {
        const double sd = std::sqrt(2.0 / (27.0 * l.cin)) * (l.relu ? 1.0 : 0.1);
        for (size_t i = 0; i < 27 * (size_t)l.cin * l.cout; ++i) h[l.w_off + i] = (float)(sd * rng.normal());
    }
    std::vector<float> z(off, 0.f);
    if (hipMemcpy(n->P, h.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->M, z.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->Vv, z.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(n->Gr, z.data(), sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("net: upload failed");
        return fail(PETGEM_HIP_ERROR);
    }
    if ((rc = cast_weights(n, nullptr)) != PETGEM_OK || hipDeviceSynchronize() != hipSuccess) return fail(rc ? rc : PETGEM_HIP_ERROR);
    *out = n;
    return PETGEM_OK;
}

int64_t petgem_net_num_params(const petgem_net* n) { return n ? (int64_t)n->nparam : -1; }

int petgem_net_get_params(const petgem_net* n, float* host) {
    if (!n || !host) { set_error("net and output are required"); return PETGEM_INVALID_ARG; }
    PG_HIP(hipMemcpy(host, n->P, sizeof(float) * n->nparam, hipMemcpyDeviceToHost));
    return PETGEM_OK;
}

int petgem_net_set_params(petgem_net* n, const float* host) {
    if (!n || !host) { set_error("net and input are required"); return PETGEM_INVALID_ARG; }
    PG_HIP(hipMemcpy(n->P, host, sizeof(float) * n->nparam, hipMemcpyHostToDevice));
    PG_TRY(cast_weights(n, nullptr));
    PG_HIP(hipDeviceSynchronize());
    return PETGEM_OK;
}

int petgem_net_forward(petgem_net* n, const void* x_dev, int32_t B, void* y_dev, void* stream) {
    if (!n || !x_dev || !y_dev || B <= 0 || B > n->batch_max) { set_error("net forward: bad arguments"); return PETGEM_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_HIP(hipMemcpyAsync(n->X0, x_dev, sizeof(bf16) * (size_t)B * kVox * kIn, hipMemcpyDeviceToDevice, s));
    PG_TRY(forward(n, B, s));
    PG_HIP(hipMemcpyAsync(y_dev, n->Y, sizeof(float) * (size_t)B * kVox * kOut, hipMemcpyDeviceToDevice, s));
    return PETGEM_OK;
}

int petgem_net_loss_grad(petgem_net* n, const void* x_dev, const void* t_dev, int32_t B, void* stream,
                         double* loss, float* grad_host) {
    if (!n || !x_dev || !t_dev || B <= 0 || B > n->batch_max) { set_error("net loss: bad arguments"); return PETGEM_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_HIP(hipMemcpyAsync(n->X0, x_dev, sizeof(bf16) * (size_t)B * kVox * kIn, hipMemcpyDeviceToDevice, s));
    PG_TRY(loss_and_grads(n, static_cast<const float*>(t_dev), B, s, loss));
    if (grad_host) {
        PG_HIP(hipMemcpyAsync(grad_host, n->Gr, sizeof(float) * n->nparam, hipMemcpyDeviceToHost, s));
        PG_HIP(hipStreamSynchronize(s));
    }
    return PETGEM_OK;
}

int petgem_net_train_step(petgem_net* n, const void* x_dev, const void* t_dev, int32_t B, float lr, void* stream,
                          double* loss) {
    if (!n || !x_dev || !t_dev || B <= 0 || B > n->batch_max || !(lr > 0.f)) {
        set_error("net train: bad arguments");
        return PETGEM_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_HIP(hipMemcpyAsync(n->X0, x_dev, sizeof(bf16) * (size_t)B * kVox * kIn, hipMemcpyDeviceToDevice, s));
    PG_TRY(loss_and_grads(n, static_cast<const float*>(t_dev), B, s, loss));
    n->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)n->step), c2 = 1.f - std::pow(b2, (float)n->step);
    hipLaunchKernelGGL(k_adam, g1((long)n->nparam), dim3(256), 0, s, n->P, n->Gr, n->M, n->Vv, (long)n->nparam, lr,
                       b1, b2, c1, c2, 1e-8f);
    PG_TRY(cast_weights(n, s));
    return PETGEM_OK;
}

int petgem_voxelize(petgem_system* sys, const double* sigma_dev, const petgem_source* src, int32_t B,
                    void* x_dev, void* stream) {
    if (!sys || !src || B <= 0 || !x_dev) { set_error("voxelize: bad arguments"); return PETGEM_INVALID_ARG; }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_TRY(ensure_vox(sys));
    std::vector<VoxSrc> v(B);
    for (int b = 0; b < B; ++b) {
        for (int k = 0; k < 3; ++k) v[b].pos[k] = src[b].pos[k];
        v[b].logf = std::log10(src[b].freq_hz);
    }
    VoxSrc* vd = nullptr;
    PG_TRY(dalloc(&vd, (size_t)B));
    PG_HIP(hipMemcpyAsync(vd, v.data(), sizeof(VoxSrc) * B, hipMemcpyHostToDevice, s));
    const double* sg = sigma_dev ? sigma_dev : sys->sigma;
    const long ld = sigma_dev ? sys->n_tets : 0;
    hipLaunchKernelGGL(k_voxelize, g1((long)B * kVox), dim3(256), 0, s, sg, ld, sys->vox_tet, vd, B, sys->vox_lo[0],
                       sys->vox_lo[1], sys->vox_lo[2], sys->vox_h, sys->vox_L, static_cast<bf16*>(x_dev));
    PG_HIP(hipGetLastError());
    PG_HIP(hipStreamSynchronize(s));
    dfree(vd);
    return PETGEM_OK;
}

int petgem_vox_targets(const petgem_solution* sol, const double* scale, void* t_dev, void* stream) {
    if (!sol || !scale || !t_dev) { set_error("targets: bad arguments"); return PETGEM_INVALID_ARG; }
    petgem_system* sys = sol->sys;
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_TRY(ensure_vox(sys));
    const int B = sol->n_src;
    double* sd = nullptr;
    PG_TRY(dalloc(&sd, (size_t)B));
    PG_HIP(hipMemcpyAsync(sd, scale, sizeof(double) * B, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_vox_field, g1((long)B * kVox), dim3(256), 0, s, sys->xyz, reinterpret_cast<const int4*>(sys->tets),
                       sys->vox_tet, sys->vox_dof, sol->x, sys->n_dof, B, sd, sys->vox_lo[0], sys->vox_lo[1],
                       sys->vox_lo[2], sys->vox_h, static_cast<float*>(t_dev));
    PG_HIP(hipGetLastError());
    PG_HIP(hipStreamSynchronize(s));
    dfree(sd);
    return PETGEM_OK;
}

int petgem_learned_x0(petgem_system* sys, petgem_net* n, const petgem_source* src, int32_t B, double g,
                      void* x0_dev, double* bnorm_out, void* stream) {
    if (!sys || !n || !src || B <= 0 || B > n->batch_max || !x0_dev || !(g > 0.0)) {
        set_error("learned x0: bad arguments");
        return PETGEM_INVALID_ARG;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    PG_TRY(ensure_vox(sys));
    // |b| of every source (the prediction is scale-free)
    if (n->bcap < (size_t)sys->n_dof) {
        dfree(n->bbuf);
        n->bcap = 0;
        PG_TRY(dalloc(&n->bbuf, (size_t)sys->n_dof));
        n->bcap = (size_t)sys->n_dof;
    }
    double2* b = n->bbuf;
    double* bn = n->bn;
    for (int k = 0; k < B; ++k) {
        PG_TRY(launch_rhs(sys, src[k], b, 1, s));
        hipLaunchKernelGGL(k_vnorm, dim3(1), dim3(256), 0, s, b, sys->n_dof, bn + k);
    }
    std::vector<double> h(B);
    PG_HIP(hipMemcpyAsync(h.data(), bn, sizeof(double) * B, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < B; ++k) {
        if (bnorm_out) bnorm_out[k] = h[k];
        h[k] *= g;
    }
    PG_HIP(hipMemcpyAsync(n->scal, h.data(), sizeof(double) * B, hipMemcpyHostToDevice, s));
    PG_TRY(upload_vsrc(n, src, B, s));
    hipLaunchKernelGGL(k_voxelize, g1((long)B * kVox), dim3(256), 0, s, sys->sigma, 0L, sys->vox_tet, n->vsrc, B,
                       sys->vox_lo[0], sys->vox_lo[1], sys->vox_lo[2], sys->vox_h, sys->vox_L, n->X0);
    PG_TRY(forward(n, B, s));
    hipLaunchKernelGGL(k_grid_to_edges, g1((long)B * sys->n_dof), dim3(256), 0, s, n->Y, B, sys->n_dof, sys->dof_mid,
                       sys->dof_tan, n->scal, sys->vox_lo[0], sys->vox_lo[1], sys->vox_lo[2], sys->vox_h,
                       static_cast<double2*>(x0_dev));
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

int petgem_learned_x0_many(petgem_system* const* systems, petgem_net* n, const petgem_source* src, int32_t n_sys,
                           double g, void* const* x0_dev, double* bnorm_out, void* stream) {
    if (!systems || !n || !src || n_sys <= 0 || n_sys > n->batch_max || !x0_dev || !(g > 0.0)) {
        set_error("learned x0 (many systems): bad arguments");
        return PETGEM_INVALID_ARG;
    }
    for (int k = 0; k < n_sys; ++k)
        if (!systems[k] || !x0_dev[k]) {
            set_error("learned x0 (many systems): system or guess " + std::to_string(k) + " is NULL");
            return PETGEM_INVALID_ARG;
        }
    hipStream_t s = static_cast<hipStream_t>(stream);
    size_t nmax = 0;
    for (int k = 0; k < n_sys; ++k) {
        PG_TRY(ensure_vox(systems[k]));
        nmax = std::max(nmax, (size_t)systems[k]->n_dof);
    }
    if (n->bcap < nmax) {
        dfree(n->bbuf);
        n->bcap = 0;
        PG_TRY(dalloc(&n->bbuf, nmax));
        n->bcap = nmax;
    }
    // |b| of every system's source
    for (int k = 0; k < n_sys; ++k) {
        PG_TRY(launch_rhs(systems[k], src[k], n->bbuf, 1, s));
        hipLaunchKernelGGL(k_vnorm, dim3(1), dim3(256), 0, s, n->bbuf, systems[k]->n_dof, n->bn + k);
    }
    std::vector<double> h(n_sys);
    PG_HIP(hipMemcpyAsync(h.data(), n->bn, sizeof(double) * n_sys, hipMemcpyDeviceToHost, s));
    PG_HIP(hipStreamSynchronize(s));
    for (int k = 0; k < n_sys; ++k) {
        if (bnorm_out) bnorm_out[k] = h[k];
        h[k] *= g;
    }
    PG_HIP(hipMemcpyAsync(n->scal, h.data(), sizeof(double) * n_sys, hipMemcpyHostToDevice, s));
    PG_TRY(upload_vsrc(n, src, n_sys, s));
    // sample k of the batch is system k on its own voxel grid
    for (int k = 0; k < n_sys; ++k) {
        const petgem_system* sys = systems[k];
        hipLaunchKernelGGL(k_voxelize, g1(kVox), dim3(256), 0, s, sys->sigma, 0L, sys->vox_tet, n->vsrc + k, 1,
                           sys->vox_lo[0], sys->vox_lo[1], sys->vox_lo[2], sys->vox_h, sys->vox_L,
                           n->X0 + (size_t)k * kVox * kIn);
    }
    PG_TRY(forward(n, n_sys, s));
    for (int k = 0; k < n_sys; ++k) {
        const petgem_system* sys = systems[k];
        hipLaunchKernelGGL(k_grid_to_edges, g1(sys->n_dof), dim3(256), 0, s, n->Y + (size_t)k * kVox * kOut, 1,
                           sys->n_dof, sys->dof_mid, sys->dof_tan, n->scal + k, sys->vox_lo[0], sys->vox_lo[1],
                           sys->vox_lo[2], sys->vox_h, static_cast<double2*>(x0_dev[k]));
    }
    PG_HIP(hipGetLastError());
    return PETGEM_OK;
}

void petgem_net_free(petgem_net* n) {
    if (!n) return;
    release_net(n);
    delete n;
}

}  // extern "C"
