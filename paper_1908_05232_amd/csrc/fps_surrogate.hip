// Convolutional flood surrogate on gfx950: BF16 MFMA training and inference
// kernels with FP32 accumulation (not part of the paper: a learned shortcut that
// advances the flood state k finite-volume steps per call; the finite-volume
// update of Eq. (2) stays its fallback and judge).
//
// Network: five 3x3 convolutions, channels last, zero padding:
//   16 (h, hu, hv, z, occupancy scaled; 11 zero channels) -> 64 -> 64 -> 64 -> 64 -> 3
// ReLU after the first four layers; the last layer is computed with 16 output
// channels (13 zero) so every layer is a whole number of 16x16x32 MFMA tiles.
//
// Kernels
//   conv_kernel<CIN, COUT, MODE>: implicit GEMM, M = pixels, N = COUT,
//     K = 9 * CIN, for the 16-channel input of the first layer (and the input
//     gradient through the last).  A persistent block computes 16 x 32 pixel
//     tiles; the input tile with its one-pixel halo and the whole weight
//     matrix are staged in LDS; each of the 8 waves owns two image rows (four
//     16-pixel M tiles) and all COUT channels, issuing
//     v_mfma_f32_16x16x32_bf16.  Forward and input-gradient passes use the
//     same kernel (the latter with flipped, transposed weights).
//   conv64_kernel<COUT, MODE>: the same for 64 input channels, with compute
//     waves of 4 rows each that reuse every loaded operand for several MFMAs
//     and loader waves that stage the next tile.
//   wgrad_kernel<CIN, COUT>: dW[co][tap][ci] = sum_p dz[p][co] x[p + tap][ci],
//     M = COUT, N = 9 * CIN, K = pixels; dz and x are staged in LDS as one
//     8-image vector per position and channel (a k-slab is 4 positions x 8
//     images); per-block FP32 partials are summed in a fixed order by
//     reduce_kernel.
//   loss / mask / Adam / weight-prep / pack / apply: elementwise.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <utility>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <mutex>
#include <new>

#include "fps.h"

namespace fps_sur_impl {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int TW = 32;            // columns of the output tile of one convolution block
constexpr int CTH = 16;            // rows of the output tile of one convolution block (x TW columns)
constexpr int kMtPerWave = 4;      // 16-pixel M tiles per wave in the convolution (2 rows x 2)
constexpr int kConvThreads = 512;  // 8 waves, two per SIMD: one computes while the other waits
constexpr int kWgWaves = 4;        // weight gradient: 4 compute waves, one per SIMD (36 MFMA tiles each) ...
constexpr int kWgLoaders = 256;    // ... and 4 loader waves that stage the next tile
constexpr int kWgThreads = kWgWaves * 64 + kWgLoaders;
constexpr int kThreads = 256;
constexpr int kLayers = 5;
constexpr int kCin[kLayers] = {16, 64, 64, 64, 64};
constexpr int kCout[kLayers] = {64, 64, 64, 64, 16};   // last: 3 used
constexpr int kOutUsed = 3;
constexpr int kWgradBlocks = 512;  // persistent blocks of the weight-gradient pass

__host__ __device__ constexpr int kp_of(int cin) { return (9 * cin + 31) / 32 * 32; }

__device__ __forceinline__ bf16 to_bf16(float f) { return (bf16)f; }
__device__ __forceinline__ float to_f32(bf16 b) { return (float)b; }

// ----------------------------------------------------------------------------
// convolution as implicit GEMM (forward and input gradient)
// MODE 0: bias + ReLU -> bf16 [.., COUT];  2: bias -> fp32 [.., 4] (first
// kOutUsed channels, 4th zero);  3: input gradient masked by the ReLU of the
// layer below (mask[p][co] > 0) -> bf16 [.., COUT]
// Persistent blocks, one per CU: the weights are staged in LDS once, then
// the block walks CTH x TW output tiles; while the matrix cores work on one
// tile, the next tile's input (with halo) is already loading into registers
// and is written to LDS after the tile.  Eight waves (two per SIMD), each
// holding 4 M tiles (2 rows of 32 pixels) x COUT/16 N tiles of accumulators.
// ----------------------------------------------------------------------------
template <int CIN, int COUT, int MODE>
__global__ __launch_bounds__(kConvThreads) void conv_kernel(const bf16* __restrict__ X,
                                                        const bf16* __restrict__ Wt,
                                                        const float* __restrict__ bias,
                                                        void* __restrict__ Y, int N, int H, int W,
                                                        const bf16* __restrict__ mask)
{
    constexpr int KP = kp_of(CIN);
    constexpr int PIX = CIN + 8;        // padded pixel stride in LDS (bank spread, 16-byte rows)
    constexpr int WST = KP + 8;         // padded weight row stride in LDS
    constexpr int NT = COUT / 16;
    constexpr int MT = kMtPerWave;
    constexpr int CHUNKS = (CTH + 2) * (TW + 2) * (CIN / 8);
    constexpr int XPT = (CHUNKS + kConvThreads - 1) / kConvThreads;
    constexpr int WCH = COUT * (KP / 8);
    extern __shared__ __align__(16) unsigned char smem[];
    bf16* xin = reinterpret_cast<bf16*>(smem);                        // [(CTH+2)(TW+2)][PIX]
    bf16* wl = xin + (CTH + 2) * (TW + 2) * PIX;                       // [COUT][WST]

    const int tiles_x = W / TW, tiles_y = H / CTH, per_img = tiles_x * tiles_y;
    const int ntiles = N * per_img;
    bf16x8 xb[XPT];
    // input tile (with halo, zeros outside the image) of tile t into registers
    auto fetch = [&](int t) {
        const int n = t / per_img, r = t % per_img;
        const int y0 = (r / tiles_x) * CTH, x0 = (r % tiles_x) * TW;
        const bf16* Xn = X + (size_t)n * H * W * CIN;
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int q = threadIdx.x + u * kConvThreads;
            xb[u] = bf16x8{};
            if (q < CHUNKS) {
                const int px = q / (CIN / 8), c8 = (q % (CIN / 8)) * 8;
                const int gy = y0 + px / (TW + 2) - 1, gx = x0 + px % (TW + 2) - 1;
                if (gy >= 0 && gy < H && gx >= 0 && gx < W)
                    xb[u] = *reinterpret_cast<const bf16x8*>(Xn + ((size_t)gy * W + gx) * CIN + c8);
            }
        }
    };
    auto deposit = [&]() {
#pragma unroll
        for (int u = 0; u < XPT; ++u) {
            const int q = threadIdx.x + u * kConvThreads;
            if (q < CHUNKS) {
                const int px = q / (CIN / 8), c8 = (q % (CIN / 8)) * 8;
                *reinterpret_cast<bf16x8*>(xin + px * PIX + c8) = xb[u];
            }
        }
    };

    int t = blockIdx.x;
    if (t >= ntiles) return;
    fetch(t);
    // the weights [COUT][KP], once per block
    for (int q = threadIdx.x; q < WCH; q += kConvThreads) {
        const int co = q / (KP / 8), k8 = (q % (KP / 8)) * 8;
        *reinterpret_cast<bf16x8*>(wl + co * WST + k8) = *reinterpret_cast<const bf16x8*>(Wt + (size_t)co * KP + k8);
    }
    deposit();
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int row16 = lane & 15, kgrp = lane >> 4;
    float bb[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bb[nt] = bias ? bias[16 * nt + row16] : 0.0f;
    for (; t < ntiles; t += gridDim.x) {
        const int n = t / per_img, r = t % per_img;
        const int y0 = (r / tiles_x) * CTH, x0 = (r % tiles_x) * TW;
        const int tn = t + gridDim.x;
        if (tn < ntiles) fetch(tn);                     // in flight during the matrix work below

        f32x4 acc[MT][NT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        for (int slab = 0; slab < KP / 32; ++slab) {
            const int k0 = slab * 32 + kgrp * 8;
            const int tap = k0 / CIN, c = k0 % CIN;
            const bool valid = tap < 9;
            const int dy = valid ? tap / 3 : 0, dx = valid ? tap % 3 : 0;
            bf16x8 a[MT], b[NT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) {
                // M tile mt: local row 2*wave + mt/2, columns 16*(mt%2) + row16
                const int ly = 2 * wave + (mt >> 1) + dy;
                const int lx = 16 * (mt & 1) + row16 + dx;
                a[mt] = valid ? *reinterpret_cast<const bf16x8*>(xin + (ly * (TW + 2) + lx) * PIX + c)
                              : bf16x8{};
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                b[nt] = *reinterpret_cast<const bf16x8*>(wl + (16 * nt + row16) * WST + k0);
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[mt], b[nt], acc[mt][nt], 0, 0, 0);
        }

        // D tile: lane holds rows (pixels) 4*kgrp + r, column (channel) row16.
        // One M tile at a time: its mask values (MODE 3) loaded together, then the stores.
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const int gy = y0 + 2 * wave + (mt >> 1);
            const size_t p0 = ((size_t)n * H + gy) * W + x0 + 16 * (mt & 1) + 4 * kgrp;
            bf16 mk[NT][4];
            if (MODE == 3) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) mk[nt][rr] = mask[(p0 + rr) * COUT + 16 * nt + row16];
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const int co = 16 * nt + row16;
#pragma unroll
                for (int rr = 0; rr < 4; ++rr) {
                    float v = acc[mt][nt][rr] + bb[nt];
                    const size_t p = p0 + rr;
                    if (MODE == 0) {
                        reinterpret_cast<bf16*>(Y)[p * COUT + co] = to_bf16(fmaxf(v, 0.0f));
                    } else if (MODE == 3) {
                        reinterpret_cast<bf16*>(Y)[p * COUT + co] =
                            to_f32(mk[nt][rr]) > 0.0f ? to_bf16(v) : to_bf16(0.0f);
                    } else {
                        if (co < 4) reinterpret_cast<float*>(Y)[p * 4 + co] = co < kOutUsed ? v : 0.0f;
                    }
                }
            }
        }
        if (tn < ntiles) {
            __syncthreads();          // every wave is done with this tile's input
            deposit();
            __syncthreads();
        }
    }
}

// ----------------------------------------------------------------------------
// convolution with 64 input channels (the four layers after the first, and the
// input gradients through them): the same implicit GEMM and modes as
// conv_kernel, organised so that each operand loaded from LDS feeds more
// matrix work.  A compute wave owns 4 output rows x 32 columns x all COUT
// channels (4 x 2 x COUT/16 accumulator tiles).  The reduction runs over
// (dx, channel half, dy): for a fixed dx and half of the input channels the
// wave loads the 3 x COUT/16 weight operands of the three dy taps once, then
// streams the 6 input rows its output rows need, and each input row's two
// operands feed every (output row, dy) pair that reads that row: 12 A and 12 B
// loads per 96 MFMAs for COUT = 64.  Four loader waves fetch the next tile's
// input into registers during the matrix work and store it to LDS between
// two barriers.
// ----------------------------------------------------------------------------
constexpr int kC64Waves = 4, kC64Loaders = 256, kC64Threads = kC64Waves * 64 + kC64Loaders;
constexpr int kC64Rows = CTH / kC64Waves;     // output rows per compute wave

template <int COUT, int MODE>
__global__ __launch_bounds__(kC64Threads) void conv64_kernel(const bf16* __restrict__ X,
                                                           const bf16* __restrict__ Wt,
                                                           const float* __restrict__ bias,
                                                           void* __restrict__ Y, int N, int H, int W,
                                                           const bf16* __restrict__ mask)
{
    constexpr int CIN = 64, KP = kp_of(CIN);
    constexpr int PIX = CIN + 8;        // padded pixel stride in LDS (bank spread, 16-byte rows)
    constexpr int WST = KP + 8;         // padded weight row stride in LDS
    constexpr int NT = COUT / 16, R = kC64Rows;
    constexpr int CHUNKS = (CTH + 2) * (TW + 2) * (CIN / 8);
    constexpr int XPT = (CHUNKS + kC64Loaders - 1) / kC64Loaders;
    constexpr int WCH = COUT * (KP / 8);
    static_assert(KP == 9 * CIN, "no padding of the reduction");
    extern __shared__ __align__(16) unsigned char smem[];
    bf16* xin = reinterpret_cast<bf16*>(smem);                        // [(CTH+2)(TW+2)][PIX]
    bf16* wl = xin + (CTH + 2) * (TW + 2) * PIX;                       // [COUT][WST]

    const int tiles_x = W / TW, tiles_y = H / CTH, per_img = tiles_x * tiles_y;
    const int ntiles = N * per_img;
    const int wave = threadIdx.x >> 6;
    if ((int)blockIdx.x >= ntiles) return;
    // the weights [COUT][KP], once per block
    for (int q = threadIdx.x; q < WCH; q += kC64Threads) {
        const int co = q / (KP / 8), k8 = (q % (KP / 8)) * 8;
        *reinterpret_cast<bf16x8*>(wl + co * WST + k8) = *reinterpret_cast<const bf16x8*>(Wt + (size_t)co * KP + k8);
    }

    if (wave >= kC64Waves) {
        // ---- loader waves
        const int lt = threadIdx.x - kC64Waves * 64;
        bf16x8 xb[XPT];
        // input tile (with halo, zeros outside the image) of tile t into registers
        auto fetch = [&](int t) {
            const int n = t / per_img, r = t % per_img;
            const int y0 = (r / tiles_x) * CTH, x0 = (r % tiles_x) * TW;
            const bf16* Xn = X + (size_t)n * H * W * CIN;
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int q = lt + u * kC64Loaders;
                const int px = q / (CIN / 8), c8 = (q % (CIN / 8)) * 8;
                const int gy = y0 + px / (TW + 2) - 1, gx = x0 + px % (TW + 2) - 1;
                const bool in = q < CHUNKS && gy >= 0 && gy < H && gx >= 0 && gx < W;
                const bf16x8 l = *reinterpret_cast<const bf16x8*>(
                    Xn + ((size_t)min(max(gy, 0), H - 1) * W + min(max(gx, 0), W - 1)) * CIN + c8);
                xb[u] = in ? l : bf16x8{};
            }
        };
        auto deposit = [&]() {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int q = lt + u * kC64Loaders;
                if (q < CHUNKS) {
                    const int px = q / (CIN / 8), c8 = (q % (CIN / 8)) * 8;
                    *reinterpret_cast<bf16x8*>(xin + px * PIX + c8) = xb[u];
                }
            }
        };
        fetch(blockIdx.x);
        deposit();
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
            __syncthreads();                  // A: tile t (and the weights) in LDS
            const int tn = t + gridDim.x;
            if (tn < ntiles) fetch(tn);
            __syncthreads();                  // B: the compute waves are done with tile t
            if (tn < ntiles) deposit();
        }
        return;
    }

    // ---- compute waves
    const int lane = threadIdx.x & 63;
    const int row16 = lane & 15, kgrp = lane >> 4;
    float bb[NT];
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) bb[nt] = bias ? bias[16 * nt + row16] : 0.0f;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int n = t / per_img, r = t % per_img;
        const int y0 = (r / tiles_x) * CTH, x0 = (r % tiles_x) * TW;
        __syncthreads();                      // A
        f32x4 acc[R][2][NT];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[i][hf][nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 1
        for (int s = 0; s < 6; ++s) {
            const int dx = s >> 1, c = 32 * (s & 1) + 8 * kgrp;
            bf16x8 b[3][NT];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    b[dy][nt] = *reinterpret_cast<const bf16x8*>(wl + (16 * nt + row16) * WST + (dy * 3 + dx) * CIN + c);
            // input row xr of the wave's window is tile row R * wave + xr (one halo row above)
#pragma unroll
            for (int xr = 0; xr < R + 2; ++xr) {
                bf16x8 a[2];
#pragma unroll
                for (int hf = 0; hf < 2; ++hf)
                    a[hf] = *reinterpret_cast<const bf16x8*>(
                        xin + ((R * wave + xr) * (TW + 2) + 16 * hf + row16 + dx) * PIX + c);
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int i = xr - dy;
                    if (i < 0 || i >= R) continue;
#pragma unroll
                    for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                        for (int nt = 0; nt < NT; ++nt)
                            acc[i][hf][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[hf], b[dy][nt], acc[i][hf][nt], 0, 0, 0);
                }
            }
        }
        __syncthreads();                      // B: the loaders may overwrite the input tile

        // D tile: lane holds rows (pixels) 4*kgrp + r, column (channel) row16.
        // One output row at a time: its mask values (MODE 3) loaded together, then the stores.
#pragma unroll
        for (int i = 0; i < R; ++i) {
            const int gy = y0 + R * wave + i;
            const size_t p0 = ((size_t)n * H + gy) * W + x0 + 4 * kgrp;
            bf16 mk[2][NT][4];
            if (MODE == 3) {
#pragma unroll
                for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int rr = 0; rr < 4; ++rr)
                            mk[hf][nt][rr] = mask[(p0 + 16 * hf + rr) * COUT + 16 * nt + row16];
            }
#pragma unroll
            for (int hf = 0; hf < 2; ++hf)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                    const int co = 16 * nt + row16;
#pragma unroll
                    for (int rr = 0; rr < 4; ++rr) {
                        const float v = acc[i][hf][nt][rr] + bb[nt];
                        const size_t p = p0 + 16 * hf + rr;
                        if (MODE == 0) {
                            reinterpret_cast<bf16*>(Y)[p * COUT + co] = to_bf16(fmaxf(v, 0.0f));
                        } else if (MODE == 3) {
                            reinterpret_cast<bf16*>(Y)[p * COUT + co] =
                                to_f32(mk[hf][nt][rr]) > 0.0f ? to_bf16(v) : to_bf16(0.0f);
                        } else {
                            if (co < 4) reinterpret_cast<float*>(Y)[p * 4 + co] = co < kOutUsed ? v : 0.0f;
                        }
                    }
                }
        }
    }
}

// ----------------------------------------------------------------------------
// weight gradient: per-block partials of dW[co][tap][ci] over pixel tiles
//
// The reduction runs over pixels, so each MFMA's k index needs runs of
// consecutive pixels per channel in LDS, and the nine taps shift those runs.
// Here the eight k values a lane supplies are the same pixel of eight images
// (images past the batch are zero): the LDS tiles hold, per pixel position
// and channel, one 16-byte vector of the eight images, so a tap's shift moves
// whole vectors and one copy of the input tile serves all nine taps.  A k-slab
// of 32 is four positions (the four rows of the tile in one column) times
// eight images.
//
// Tile: 4 rows x 8 columns of positions x 8 images (256 pixels).  LDS:
//   dzL[pos][swz(co)][8 images], pos = row * 8 + col           (32 positions)
//   xL[pos][swz(ci)][8 images],  pos = row * 10 + col, halo of one (60 positions)
// with swz(c) = c ^ ((c >> 3) & 7) and a padded position stride, so that the
// 16-byte stores of the staging (a lane per channel group) and the 16-byte
// operand reads (a lane per channel) fall in distinct banks.
// A compute wave owns one 16-channel input tile, every 16-channel output tile
// and all nine taps, and walks the columns of its share of the tile with a
// window of three input columns in registers: per column 3 new B operands and
// COUT / 16 A operands feed 9 * COUT / 16 MFMAs.  Layers with fewer input
// tiles than compute waves split the columns between waves, each writing a
// partial of its own.  Four more waves only load: while the compute waves
// work on a tile they fetch the next one, transpose it in registers and add
// up its bias gradient, and between two barriers they store it to LDS.
// ----------------------------------------------------------------------------
constexpr int WTH = 4, WTW = 8, WNG = 8;      // weight-gradient tile: rows, columns, images
__host__ __device__ constexpr int wg_pad(int c) { return c == 64 ? 8 : 2; }
__host__ __device__ constexpr int wg_co_per(int cout) { return cout / 16; }
__host__ __device__ constexpr int wg_groups(int cin, int cout) { return (cin / 16) * (cout / 16 / wg_co_per(cout)); }
__host__ __device__ constexpr int wg_ksplit(int cin, int cout) { return kWgWaves / wg_groups(cin, cout); }
__host__ __device__ constexpr size_t wg_lds(int cin, int cout)
{
    return (size_t)16 * (WTH * WTW * (cout + wg_pad(cout)) + (WTH + 2) * (WTW + 2) * (cin + wg_pad(cin)));
}

__device__ __forceinline__ int wg_swz(int c) { return c ^ ((c >> 3) & 7); }

template <int CIN, int COUT>
__global__ __launch_bounds__(kWgThreads) void wgrad_kernel(const bf16* __restrict__ X,
                                                         const bf16* __restrict__ DZ,
                                                         float* __restrict__ part, float* __restrict__ bpart,
                                                         int N, int H, int W)
{
    static_assert(CIN == 16 || CIN == 64, "input channels");
    static_assert(COUT == 16 || COUT == 64, "output channels");
    constexpr int PSD = COUT + wg_pad(COUT), PSX = CIN + wg_pad(CIN);   // position strides, 16-byte units
    constexpr int XW = WTW + 2, XPOS = (WTH + 2) * XW;
    constexpr int NCO8 = COUT / 8, NCI8 = CIN / 8;
    constexpr int DZU = WTH * WTW * NCO8, XU = XPOS * NCI8, UNITS = DZU + XU;   // staging units
    constexpr int XPT = (UNITS + kWgLoaders - 1) / kWgLoaders;
    constexpr int CO_PER = wg_co_per(COUT), NCIT = CIN / 16;
    constexpr int G = wg_groups(CIN, COUT), KS = wg_ksplit(CIN, COUT), CPW = WTW / KS;
    static_assert(G * KS == kWgWaves && WTW % KS == 0, "wave split");
    static_assert(DZU <= kWgLoaders, "every dz unit in the first round of a fixed loader thread");
    static_assert(kWgLoaders % NCO8 == 0, "fixed channel group per loader thread");
    extern __shared__ __align__(16) unsigned char smem[];
    bf16x8* dzL = reinterpret_cast<bf16x8*>(smem);
    bf16x8* xL = dzL + WTH * WTW * PSD;

    const int wave = threadIdx.x >> 6;
    const int tiles_x = W / WTW, tiles_y = H / WTH, per_grp = tiles_x * tiles_y;
    const int ntiles = ((N + WNG - 1) / WNG) * per_grp;
    float bsum[8] = {};

    if (wave >= kWgWaves) {
        // ---- loader waves: fetch the next tile, transpose it in registers
        // while the compute waves work, store it to LDS between the barriers
        const int lt = threadIdx.x - kWgWaves * 64;
        typedef bf16x8 Set[XPT][8];
        Set s0;
        // unit u: 8 images x 8 channels of one position; addresses clamped
        // into the arrays, values outside the image or the batch zeroed
        auto fetch = [&](Set& v, int t) {
            const int n0 = (t / per_grp) * WNG, r = t % per_grp;
            const int y0 = (r / tiles_x) * WTH, x0 = (r % tiles_x) * WTW;
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int q = lt + u * kWgLoaders;
                const bool isdz = q < DZU;
                const int qq = isdz ? q : q - DZU;
                const int nc8 = isdz ? NCO8 : NCI8, C = isdz ? COUT : CIN;
                const int pos = qq / nc8, cg = qq % nc8;
                const int gy = isdz ? y0 + pos / WTW : y0 + pos / XW - 1;
                const int gx = isdz ? x0 + pos % WTW : x0 + pos % XW - 1;
                const bool in = q < UNITS && gy >= 0 && gy < H && gx >= 0 && gx < W;
                const bf16* src = (isdz ? DZ : X) +
                                  ((size_t)min(max(gy, 0), H - 1) * W + min(max(gx, 0), W - 1)) * C + 8 * cg;
                const size_t img = (size_t)H * W * C;
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const bf16x8 l = *reinterpret_cast<const bf16x8*>(src + (size_t)min(n0 + j, N - 1) * img);
                    v[u][j] = in && n0 + j < N ? l : bf16x8{};
                }
            }
        };
        // v[u][j][e] (image j, channel e) -> v[u][e][j]; dz units add to the bias sums
        auto transpose = [&](Set& v) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int q = lt + u * kWgLoaders;
                if (u == 0 && q < DZU) {
#pragma unroll
                    for (int j = 0; j < 8; ++j)
#pragma unroll
                        for (int e = 0; e < 8; ++e) bsum[e] += to_f32(v[u][j][e]);
                }
                bf16x8 tv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e)
#pragma unroll
                    for (int j = 0; j < 8; ++j) tv[e][j] = v[u][j][e];
#pragma unroll
                for (int e = 0; e < 8; ++e) v[u][e] = tv[e];
            }
        };
        auto store = [&](Set& v) {
#pragma unroll
            for (int u = 0; u < XPT; ++u) {
                const int q = lt + u * kWgLoaders;
                if (q >= UNITS) continue;
                const bool isdz = q < DZU;
                const int pos = isdz ? q / NCO8 : (q - DZU) / NCI8;
                const int cg = isdz ? q % NCO8 : (q - DZU) % NCI8;
                bf16x8* dst = isdz ? dzL + pos * PSD : xL + pos * PSX;
#pragma unroll
                for (int e = 0; e < 8; ++e) dst[wg_swz(8 * cg + e)] = v[u][e];
            }
        };
        // the next tile's loads are issued at barrier A and land during the
        // compute of this one
        fetch(s0, blockIdx.x);
        transpose(s0);
        store(s0);
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
            __syncthreads();                  // A: tile t is in LDS
            const int t1 = t + gridDim.x;
            if (t1 < ntiles) {
                fetch(s0, t1);
                transpose(s0);
            }
            __syncthreads();                  // B: the compute waves are done with tile t
            if (t1 < ntiles) store(s0);
        }
    } else {
        // ---- compute waves
        const int lane = threadIdx.x & 63;
        const int row16 = lane & 15, kgrp = lane >> 4;
        const int grp = wave % G, ks = wave / G;
        const int ct = grp % NCIT, cp = grp / NCIT;
        f32x4 acc[CO_PER][9];
#pragma unroll
        for (int j = 0; j < CO_PER; ++j)
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[j][k] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        const int ci_sw = wg_swz(16 * ct + row16);
        int co_sw[CO_PER];
#pragma unroll
        for (int j = 0; j < CO_PER; ++j) co_sw[j] = wg_swz(16 * (cp * CO_PER + j) + row16);
        const int c0 = ks * CPW;
        for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
            __syncthreads();                  // A
            // window of input columns: win[dy][k % 3] holds halo column c0 + k, rows kgrp + dy
            bf16x8 win[3][3];
#pragma unroll
            for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                for (int k = 0; k < 2; ++k) win[dy][k] = xL[((kgrp + dy) * XW + c0 + k) * PSX + ci_sw];
#pragma unroll
            for (int cc = 0; cc < CPW; ++cc) {
                const int c = c0 + cc;
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) win[dy][(cc + 2) % 3] = xL[((kgrp + dy) * XW + c + 2) * PSX + ci_sw];
                bf16x8 a[CO_PER];
#pragma unroll
                for (int j = 0; j < CO_PER; ++j) a[j] = dzL[(kgrp * WTW + c) * PSD + co_sw[j]];
#pragma unroll
                for (int j = 0; j < CO_PER; ++j)
#pragma unroll
                    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx)
                            acc[j][dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                a[j], win[dy][(cc + dx) % 3], acc[j][dy * 3 + dx], 0, 0, 0);
            }
            __syncthreads();                  // B
        }
        // partial [block * KS + ks][co][tap][ci]; D tile lane holds rows (co) 4*kgrp + r, column (ci) row16
        float* pb = part + ((size_t)blockIdx.x * KS + ks) * COUT * 9 * CIN;
        const int ci = 16 * ct + row16;
#pragma unroll
        for (int j = 0; j < CO_PER; ++j)
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int co = 16 * (cp * CO_PER + j) + 4 * kgrp + r;
                    pb[((size_t)co * 9 + tap) * CIN + ci] = acc[j][tap][r];
                }
    }
    // bias partial of the block: the loader threads of each channel group in thread order
    __syncthreads();
    float* bs = reinterpret_cast<float*>(smem);
    if (wave >= kWgWaves) {
#pragma unroll
        for (int e = 0; e < 8; ++e) bs[(threadIdx.x - kWgWaves * 64) * 8 + e] = bsum[e];
    }
    __syncthreads();
    if (threadIdx.x < COUT) {
        const int g = threadIdx.x / 8, e = threadIdx.x % 8;
        float s = 0.0f;
        for (int th = g; th < kWgLoaders; th += NCO8) s += bs[th * 8 + e];
        bpart[(size_t)blockIdx.x * COUT + threadIdx.x] = s;
    }
}

// Sum of the per-block partials of every output element in a fixed order:
// 16 threads per element each sum every 16th block, then the 16 sums are
// added in thread order.  Block: 64 elements x 16 groups.  The blocks past
// the weights' (count / 64 rounded up) do the same for the bias partials.
__global__ __launch_bounds__(1024) void reduce_kernel(const float* __restrict__ wpart, int nwparts, int wcount,
                                                      float* __restrict__ wout, const float* __restrict__ bpart,
                                                      int nbparts, int bcount, float* __restrict__ bout)
{
    __shared__ float red[16][64];
    const int wblocks = (wcount + 63) / 64;
    const bool bias = (int)blockIdx.x >= wblocks;
    const float* part = bias ? bpart : wpart;
    const int nblocks = bias ? nbparts : nwparts, count = bias ? bcount : wcount;
    float* out = bias ? bout : wout;
    const int o = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int i = (blockIdx.x - (bias ? wblocks : 0)) * 64 + o;
    float s = 0.0f;
    if (i < count) {
        int b = g;
        for (; b + 48 < nblocks; b += 64) {     // four independent loads in flight
            const float v0 = part[(size_t)b * count + i], v1 = part[(size_t)(b + 16) * count + i];
            const float v2 = part[(size_t)(b + 32) * count + i], v3 = part[(size_t)(b + 48) * count + i];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; b < nblocks; b += 16) s += part[(size_t)b * count + i];
    }
    red[g][o] = s;
    __syncthreads();
    if (g == 0 && i < count) {
        float t = 0.0f;
        for (int k = 0; k < 16; ++k) t += red[k][o];
        out[i] = t;
    }
}

// ----------------------------------------------------------------------------
// elementwise kernels
// ----------------------------------------------------------------------------

// MSE: per-block loss partials and dz of the output layer (bf16, 16 channels)
__global__ void loss_kernel(const float* __restrict__ pred, const float* __restrict__ target, int64_t npix,
                            float scale, bf16* __restrict__ dz, float* __restrict__ part)
{
    __shared__ float red[kThreads];
    float s = 0.0f;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        bf16x8 z0 = {}, z1 = {};
#pragma unroll
        for (int c = 0; c < kOutUsed; ++c) {
            const float d = pred[p * 4 + c] - target[p * 4 + c];
            s += d * d;
            z0[c] = to_bf16(2.0f * d * scale);
        }
        *reinterpret_cast<bf16x8*>(dz + p * 16) = z0;
        *reinterpret_cast<bf16x8*>(dz + p * 16 + 8) = z1;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// sum of the loss partials in a fixed order: thread t adds partials t,
// t + 256, ...; then a tree over the 256 thread sums.  One block of kThreads.
__global__ void sum_kernel(const float* __restrict__ part, int n, float scale, float* __restrict__ out)
{
    __shared__ float red[kThreads];
    float s = 0.0f;
    for (int i = threadIdx.x; i < n; i += kThreads) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// Adam on FP32 master parameters (bias-corrected).
// BF16 copies of the weights a layer's passes read (see prep_weights_kernel)
struct WeightCopies {
    bf16* wf[kLayers];
    bf16* wd[kLayers];       // nullptr for the first layer (no input gradient)
    int off[kLayers + 1];    // parameter offset of each layer
    int cin[kLayers], cout[kLayers];
};

// Adam step of every parameter; the new weights go straight into the BF16
// copies of the forward and input-gradient passes (their zero padding is
// written once, by prep_weights_kernel)
__global__ void adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int n, float lr, float b1, float b2, float eps,
                            float c1, float c2, WeightCopies wc)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    int l = 0;
#pragma unroll
    for (int k = 1; k < kLayers; ++k) l += i >= wc.off[k];
    const int j = i - wc.off[l], cin = wc.cin[l], cout = wc.cout[l];
    if (j < cout * 9 * cin) {
        const int co = j / (9 * cin), tap = (j / cin) % 9, ci = j % cin;
        wc.wf[l][co * kp_of(cin) + tap * cin + ci] = to_bf16(wi);
        if (wc.wd[l]) wc.wd[l][ci * kp_of(cout) + (8 - tap) * cout + co] = to_bf16(wi);
    }
}

// bf16 weights for the forward pass [COUT][KP] (k = tap*CIN + ci) and for the
// input-gradient pass [CIN][KPd] (k = (8 - tap)*COUT + co), from FP32 master [COUT][9][CIN]
__global__ void prep_weights_kernel(const float* __restrict__ w, int cin, int cout, bf16* __restrict__ wf,
                                    bf16* __restrict__ wd)
{
    const int kp = kp_of(cin), kpd = kp_of(cout);
    const int total = cout * kp + (wd ? cin * kpd : 0);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        if (i < cout * kp) {
            const int co = i / kp, k = i % kp;
            wf[i] = to_bf16(k < 9 * cin ? w[((size_t)co * 9 + k / cin) * cin + k % cin] : 0.0f);
        } else {
            const int j = i - cout * kp;
            const int ci = j / kpd, k = j % kpd;
            float val = 0.0f;
            if (k < 9 * cout) {
                const int tapd = k / cout, co = k % cout;
                val = w[((size_t)co * 9 + (8 - tapd)) * cin + ci];
            }
            wd[j] = to_bf16(val);
        }
    }
}

// input scales (h, hu, hv, z, occupancy, inflow depth) and output scales
// (change of h, hu, hv)
__constant__ float kInScale[6] = {1.0f, 1.0f, 1.0f, 1.0f / 3.0f, 0.25f, 1.0f};
__constant__ float kOutScale[3] = {0.05f, 0.05f, 0.05f};

// Network input of one state: channels h, hu, hv, z, occupancy and the depth
// the inflow adds over the block (on the cells of the inflow segment only).
__global__ void pack_kernel(int64_t npix, int nx, int ny, const float* __restrict__ h,
                            const float* __restrict__ hu, const float* __restrict__ hv,
                            const float* __restrict__ z, const int32_t* __restrict__ occ, int inflow_side,
                            int c0, int c1, float inflow_depth, bf16* __restrict__ x)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(p % nx), j = (int)(p / nx);
        bool in = false;
        if (inflow_side == FPS_SIDE_S) in = j == 0 && i >= c0 && i < c1;
        else if (inflow_side == FPS_SIDE_N) in = j == ny - 1 && i >= c0 && i < c1;
        else if (inflow_side == FPS_SIDE_W) in = i == 0 && j >= c0 && j < c1;
        else if (inflow_side == FPS_SIDE_E) in = i == nx - 1 && j >= c0 && j < c1;
        bf16x8 a = {}, b = {};
        a[0] = to_bf16(h[p] * kInScale[0]);
        a[1] = to_bf16(hu[p] * kInScale[1]);
        a[2] = to_bf16(hv[p] * kInScale[2]);
        a[3] = to_bf16(z[p] * kInScale[3]);
        a[4] = to_bf16(occ ? (float)occ[p] * kInScale[4] : 0.0f);
        a[5] = to_bf16(in ? inflow_depth * kInScale[5] : 0.0f);
        *reinterpret_cast<bf16x8*>(x + p * 16) = a;
        *reinterpret_cast<bf16x8*>(x + p * 16 + 8) = b;
    }
}

__global__ void target_kernel(int64_t npix, const float* __restrict__ h0, const float* __restrict__ hu0,
                              const float* __restrict__ hv0, const float* __restrict__ h1,
                              const float* __restrict__ hu1, const float* __restrict__ hv1,
                              float* __restrict__ t)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        t[p * 4 + 0] = (h1[p] - h0[p]) / kOutScale[0];
        t[p * 4 + 1] = (hu1[p] - hu0[p]) / kOutScale[1];
        t[p * 4 + 2] = (hv1[p] - hv0[p]) / kOutScale[2];
        t[p * 4 + 3] = 0.0f;
    }
}

// U += scale * y; depth kept >= 0; a cell that was dry stays dry unless the
// network puts at least h_snap of water on it; no discharge where dry
__global__ void apply_kernel(int64_t npix, const float* __restrict__ y, float* __restrict__ h,
                             float* __restrict__ hu, float* __restrict__ hv, float h_dry, float h_snap)
{
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < npix; p += (int64_t)gridDim.x * blockDim.x) {
        const float h0 = h[p];
        float hn = fmaxf(h0 + kOutScale[0] * y[p * 4 + 0], 0.0f);
        if (!(h0 > h_dry) && hn < h_snap) hn = 0.0f;
        float qx = hu[p] + kOutScale[1] * y[p * 4 + 1];
        float qy = hv[p] + kOutScale[2] * y[p * 4 + 2];
        if (!(hn > h_dry)) {
            qx = 0.0f;
            qy = 0.0f;
        }
        h[p] = hn;
        hu[p] = qx;
        hv[p] = qy;
    }
}

__device__ __forceinline__ int hazard_class(float h, float qx, float qy, float eps, const float* thr)
{
    if (!(h > eps)) return 0;
    float hr = (fmaxf(fabsf(qx / h), fabsf(qy / h)) + 0.5f) * h;
    return hr < thr[0] ? 1 : hr < thr[1] ? 2 : hr < thr[2] ? 3 : 4;
}

// containing cell: IEEE division and floor in FP32, clamped to the grid
__device__ __forceinline__ int cell_index(float x, float d, int n)
{
    return (int)fminf(fmaxf(floorf(x / d), 0.0f), (float)(n - 1));
}

// Judge: over the sampled agents (every stride-th) that have not exited,
// count those where the two flood states differ in depth by more than tol or
// in hazard class (Table 1 thresholds), and the largest depth difference.
// out[0] = count (int), out[1] = max |dh| (float bits).
// The people the judge looks at: every stride-th agent that has not exited,
// and, when a selection state (hs, qxs, qys) is given, every agent whose
// cell there is within h_margin of the dry threshold or has a hazard rate
// within margin of a Table 1 threshold (people whose class a small depth
// error could change).
struct JudgePick {
    int stride;
    const float* hs;
    const float* qxs;
    const float* qys;
    float margin, h_margin, eps, t1, t2, t3;
};
__device__ __forceinline__ bool judged(const JudgePick& q, int64_t a, size_t c)
{
    if (a % q.stride == 0) return true;
    if (!q.hs) return false;
    const float h = q.hs[c];
    if (!(h > q.eps + q.h_margin)) return true;
    const float hr = (fmaxf(fabsf(q.qxs[c] / h), fabsf(q.qys[c] / h)) + 0.5f) * h;
    return fabsf(hr - q.t1) < q.margin || fabsf(hr - q.t2) < q.margin || fabsf(hr - q.t3) < q.margin;
}

__global__ void judge_kernel(int na, JudgePick q, const float* __restrict__ x, const float* __restrict__ y,
                             const uint8_t* __restrict__ state, int nx, int ny, float dx, float dy,
                             const float* __restrict__ ha, const float* __restrict__ qxa,
                             const float* __restrict__ qya, const float* __restrict__ hb,
                             const float* __restrict__ qxb, const float* __restrict__ qyb, float tol,
                             int32_t* __restrict__ out)
{
    // every agent when a selection state is given, else only the sample
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t a = q.hs ? t : t * q.stride;
    if (a >= na || state[a] == FPS_ST_EXITED || state[a] == FPS_ST_OUTSIDE) return;
    const size_t c = (size_t)cell_index(y[a], dy, ny) * nx + cell_index(x[a], dx, nx);
    if (!judged(q, a, c)) return;
    const float thr[3] = {q.t1, q.t2, q.t3};
    const float d = fabsf(ha[c] - hb[c]);
    const bool bad = d > tol || hazard_class(ha[c], qxa[c], qya[c], q.eps, thr) !=
                                    hazard_class(hb[c], qxb[c], qyb[c], q.eps, thr);
    if (bad) atomicAdd(&out[0], 1);
    atomicMax(&out[1], __float_as_int(d));    // non-negative floats order as ints
    atomicAdd(&out[2], 1);
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
        p[k] = 0;
}

// Judge region: mark every block x block cell block within halo cells of a
// judged agent's cell (the same people as the judge).
__global__ void judge_mask_kernel(int na, JudgePick q, const float* __restrict__ x, const float* __restrict__ y,
                                  const uint8_t* __restrict__ state, int nx, int ny, float dx, float dy, int halo,
                                  int block, uint8_t* __restrict__ mask)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t a = q.hs ? t : t * q.stride;
    if (a >= na || state[a] == FPS_ST_EXITED || state[a] == FPS_ST_OUTSIDE) return;
    const int i = cell_index(x[a], dx, nx), j = cell_index(y[a], dy, ny);
    if (!judged(q, a, (size_t)j * nx + i)) return;
    const int mbx = (nx + block - 1) / block;
    const int bx0 = max(i - halo, 0) / block, bx1 = min(i + halo, nx - 1) / block;
    const int by0 = max(j - halo, 0) / block, by1 = min(j + halo, ny - 1) / block;
    for (int by = by0; by <= by1; ++by)
        for (int bx = bx0; bx <= bx1; ++bx) mask[(size_t)by * mbx + bx] = 1;
}

// per-cell counts of evacuees still evacuating (the rule of the coupled step)
__global__ void occupancy_kernel(int na, const float* __restrict__ x, const float* __restrict__ y,
                                 const uint8_t* __restrict__ role, const uint8_t* __restrict__ state, int nx,
                                 int ny, float dx, float dy, int32_t* __restrict__ counts)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na || role[a] != FPS_ROLE_EVACUEE || state[a] != FPS_ST_EVAC) return;
    atomicAdd(&counts[(size_t)cell_index(y[a], dy, ny) * nx + cell_index(x[a], dx, nx)], 1);
}

__global__ void copy3_kernel(int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                             const float* __restrict__ c, float* __restrict__ A, float* __restrict__ B,
                             float* __restrict__ Cc)
{
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        A[k] = a[k];
        B[k] = b[k];
        Cc[k] = c[k];
    }
}

}  // namespace fps_sur_impl

// ============================================================================
// host side
// ============================================================================
using namespace fps_sur_impl;

struct fps_sur {
    int max_batch = 0, H = 0, W = 0;
    int cus = 256;                   // compute units of the device (persistent convolution blocks)
    int conv_cap = 0, wgrad_cap = 0; // caps on the blocks of the two kernels (0 = none)
    hipStream_t stream = nullptr;
    char err[512] = "";
    float *params = nullptr, *m = nullptr, *v = nullptr, *grads = nullptr;
    bf16* wf[kLayers] = {};
    bf16* wd[kLayers] = {};
    bf16* act[kLayers - 1] = {};     // outputs of layers 1..4, [B][H][W][64]
    float* y = nullptr;              // [B][H][W][4]
    bf16* g = nullptr;               // input gradient of a layer, [B][H][W][64]
    bf16* dz = nullptr;              // masked gradient, [B][H][W][64]
    bf16* dz5 = nullptr;             // output-layer gradient, [B][H][W][16]
    float* wpart = nullptr;          // weight-gradient partials
    float* bpart = nullptr;          // bias-gradient partials
    float* lpart = nullptr;          // loss partials
    int adam_step = 0;
    bool have_grads = false;
};

namespace {

char g_sur_err[512] = "";

int sfail(fps_sur* s, int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(s ? s->err : g_sur_err, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define SCHK(s, expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return sfail(s, FPS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

constexpr int kLossBlocks = 1024;

size_t a256(size_t v) { return (v + 255) & ~size_t(255); }

int64_t w_count(int l) { return (int64_t)kCout[l] * 9 * kCin[l]; }
int64_t layer_params(int l) { return w_count(l) + kCout[l]; }
int64_t param_offset(int l)
{
    int64_t o = 0;
    for (int k = 0; k < l; ++k) o += layer_params(k);
    return o;
}
int64_t total_params() { return param_offset(kLayers); }

struct SurLayout {
    size_t params, m, v, grads, wf[kLayers], wd[kLayers], act[kLayers - 1], y, g, dz, dz5, wpart, bpart,
        lpart, total;
};

SurLayout sur_layout(int B, int H, int W)
{
    SurLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = a256(o + bytes);
        return at;
    };
    const size_t np = (size_t)total_params();
    const size_t pix = (size_t)B * H * W;
    L.params = take(4 * np);
    L.m = take(4 * np);
    L.v = take(4 * np);
    L.grads = take(4 * np);
    for (int l = 0; l < kLayers; ++l) {
        L.wf[l] = take(2 * (size_t)kCout[l] * kp_of(kCin[l]));
        L.wd[l] = take(2 * (size_t)kCin[l] * kp_of(kCout[l]));
    }
    for (int l = 0; l < kLayers - 1; ++l) L.act[l] = take(2 * pix * 64);
    L.y = take(4 * pix * 4);
    L.g = take(2 * pix * 64);
    L.dz = take(2 * pix * 64);
    L.dz5 = take(2 * pix * 16);
    L.wpart = take(4 * (size_t)kWgradBlocks * 64 * 9 * 64);
    L.bpart = take(4 * (size_t)kWgradBlocks * 64);
    L.lpart = take(4 * (size_t)kLossBlocks);
    L.total = o;
    return L;
}

template <int CIN, int COUT, int MODE>
int conv(fps_sur* s, int n, const bf16* x, const bf16* w, const float* b, void* y, const bf16* mask = nullptr)
{
    constexpr int KP = kp_of(CIN);
    const size_t lds = (size_t)(CTH + 2) * (TW + 2) * (CIN + 8) * 2 + (size_t)COUT * (KP + 8) * 2;
    void (*k)(const bf16*, const bf16*, const float*, void*, int, int, int, const bf16*);
    int threads;
    if constexpr (CIN == 64) {
        k = conv64_kernel<COUT, MODE>;
        threads = kC64Threads;
    } else {
        k = conv_kernel<CIN, COUT, MODE>;
        threads = kConvThreads;
    }
    SCHK(s, hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int tiles = n * (s->H / CTH) * (s->W / TW);
    // persistent: one block per compute unit (or fewer, when capped)
    const int blocks = std::min(tiles, s->conv_cap > 0 ? std::min(s->conv_cap, s->cus) : s->cus);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s->stream, x, w, b, y, n, s->H, s->W, mask);
    SCHK(s, hipGetLastError());
    return FPS_OK;
}

// weight and bias gradients of one layer: per-block partials, then the fixed-order sums
template <int CIN, int COUT>
int wgrad(fps_sur* s, int n, const bf16* x, const bf16* dz, int layer)
{
    const size_t lds = wg_lds(CIN, COUT);
    auto k = wgrad_kernel<CIN, COUT>;
    SCHK(s, hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    const int tiles = (n + WNG - 1) / WNG * (s->H / WTH) * (s->W / WTW);
    // persistent: one block per compute unit (or fewer, when capped)
    const int cap = std::min(s->cus, kWgradBlocks);
    const int blocks = std::min(tiles, s->wgrad_cap > 0 ? std::min(s->wgrad_cap, cap) : cap);
    const int nparts = blocks * wg_ksplit(CIN, COUT);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(kWgThreads), lds, s->stream, x, dz, s->wpart, s->bpart, n, s->H,
                       s->W);
    SCHK(s, hipGetLastError());
    const int count = COUT * 9 * CIN;
    float* dw = s->grads + param_offset(layer);
    hipLaunchKernelGGL(reduce_kernel, dim3((count + 63) / 64 + (COUT + 63) / 64), dim3(1024), 0, s->stream,
                       s->wpart, nparts, count, dw, s->bpart, blocks, COUT, dw + w_count(layer));
    SCHK(s, hipGetLastError());
    return FPS_OK;
}

int prep_weights(fps_sur* s)
{
    for (int l = 0; l < kLayers; ++l) {
        hipLaunchKernelGGL(prep_weights_kernel, dim3(64), dim3(256), 0, s->stream, s->params + param_offset(l),
                           kCin[l], kCout[l], s->wf[l], l > 0 ? s->wd[l] : (bf16*)nullptr);
        SCHK(s, hipGetLastError());
    }
    return FPS_OK;
}

const float* bias_of(const fps_sur* s, int l) { return s->params + param_offset(l) + w_count(l); }

int forward(fps_sur* s, int n, const bf16* x, float* y)
{
    int rc = conv<16, 64, 0>(s, n, x, s->wf[0], bias_of(s, 0), s->act[0]);
    for (int l = 1; l < 4 && rc == FPS_OK; ++l)
        rc = conv<64, 64, 0>(s, n, s->act[l - 1], s->wf[l], bias_of(s, l), s->act[l]);
    if (rc == FPS_OK) rc = conv<64, 16, 2>(s, n, s->act[3], s->wf[4], bias_of(s, 4), y);
    return rc;
}

int check_args(fps_sur* s, int n)
{
    if (n < 1 || n > s->max_batch) return sfail(s, FPS_E_CAPACITY, "batch %d outside [1, %d]", n, s->max_batch);
    return FPS_OK;
}

// Scratch of the allocation-free forward pass (fps_sur_forward_noalloc): the
// BF16 weight matrices of the five layers, then two activation buffers used in
// turn by layers 1-4, each of kNoallocPixels x 64 BF16 channels.  One copy per
// GPU, held until the process ends; every call on a GPU uses the same copy.
constexpr int64_t kNoallocPixels = 131072;          // n * H * W per call, at most (two 256^2 patches)
constexpr size_t noalloc_weight_bytes()
{
    size_t o = 0;
    for (int l = 0; l < kLayers; ++l) o += (2 * (size_t)kCout[l] * kp_of(kCin[l]) + 255) / 256 * 256;
    return o;
}
constexpr size_t kNoallocActBytes = 2 * (size_t)kNoallocPixels * 64;
constexpr size_t kNoallocBytes = noalloc_weight_bytes() + 2 * kNoallocActBytes;
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

// Device address of this GPU's copy of the scratch array and its compute-unit
// count, looked up once per device (with that device current) and kept.  In
// host code the array's name is not a device address: only this pointer is
// passed to kernels.
constexpr int kMaxDevices = 64;
struct NoallocDevice {
    unsigned char* ptr = nullptr;
    int cus = 0;
};
std::mutex g_noalloc_mu;
NoallocDevice g_noalloc[kMaxDevices];

int noalloc_device(NoallocDevice* out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return sfail(nullptr, FPS_E_DEVICE, "fps_sur_forward_noalloc: no usable current device (%d)", dev);
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoallocDevice& d = g_noalloc[dev];
    if (!d.ptr) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sfail(nullptr, FPS_E_DEVICE, "fps_sur_forward_noalloc: hipGetSymbolAddress: %s",
                         hipGetErrorString(e));
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        d.cus = cus;
        d.ptr = static_cast<unsigned char*>(p);
    }
    *out = d;
    return FPS_OK;
}

}  // namespace

extern "C" {

int32_t fps_sur_param_count(void) { return (int32_t)total_params(); }

int fps_sur_set_blocks(fps_sur* s, int32_t conv_blocks, int32_t wgrad_blocks)
{
    if (!s) return sfail(nullptr, FPS_E_INVALID, "fps_sur_set_blocks: sur is NULL");
    if (conv_blocks < 0 || wgrad_blocks < 0) return sfail(s, FPS_E_INVALID, "fps_sur_set_blocks: negative cap");
    s->conv_cap = conv_blocks;
    s->wgrad_cap = wgrad_blocks;
    return FPS_OK;
}

size_t fps_sur_workspace_bytes(int32_t max_batch, int32_t H, int32_t W)
{
    if (max_batch < 1 || H < CTH || W < TW || H % CTH || W % TW) return 0;
    return sur_layout(max_batch, H, W).total;
}

int fps_sur_create(int32_t max_batch, int32_t H, int32_t W, void* ws, size_t ws_bytes, void* stream,
                   fps_sur** out)
{
    if (!out) return sfail(nullptr, FPS_E_INVALID, "fps_sur_create: out is NULL");
    *out = nullptr;
    if (max_batch < 1 || H < CTH || W < TW || H % CTH || W % TW)
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_create: need batch >= 1 and H, W multiples of %d, %d", CTH,
                     TW);
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_create: workspace NULL or not 256-byte aligned");
    SurLayout L = sur_layout(max_batch, H, W);
    if (ws_bytes < L.total)
        return sfail(nullptr, FPS_E_CAPACITY, "fps_sur_create: workspace %zu < %zu bytes", ws_bytes, L.total);
    fps_sur* s = new (std::nothrow) fps_sur();
    if (!s) return sfail(nullptr, FPS_E_DEVICE, "fps_sur_create: out of host memory");
    s->max_batch = max_batch;
    s->H = H;
    s->W = W;
    s->stream = static_cast<hipStream_t>(stream);
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            s->cus = cus;
    }
    char* b = static_cast<char*>(ws);
    s->params = reinterpret_cast<float*>(b + L.params);
    s->m = reinterpret_cast<float*>(b + L.m);
    s->v = reinterpret_cast<float*>(b + L.v);
    s->grads = reinterpret_cast<float*>(b + L.grads);
    for (int l = 0; l < kLayers; ++l) {
        s->wf[l] = reinterpret_cast<bf16*>(b + L.wf[l]);
        s->wd[l] = reinterpret_cast<bf16*>(b + L.wd[l]);
    }
    for (int l = 0; l < kLayers - 1; ++l) s->act[l] = reinterpret_cast<bf16*>(b + L.act[l]);
    s->y = reinterpret_cast<float*>(b + L.y);
    s->g = reinterpret_cast<bf16*>(b + L.g);
    s->dz = reinterpret_cast<bf16*>(b + L.dz);
    s->dz5 = reinterpret_cast<bf16*>(b + L.dz5);
    s->wpart = reinterpret_cast<float*>(b + L.wpart);
    s->bpart = reinterpret_cast<float*>(b + L.bpart);
    s->lpart = reinterpret_cast<float*>(b + L.lpart);
    *out = s;
    return FPS_OK;
}

void fps_sur_destroy(fps_sur* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

int fps_sur_set_params(fps_sur* s, const float* params)
{
    if (!s || !params) return sfail(s, FPS_E_INVALID, "fps_sur_set_params: NULL argument");
    const size_t bytes = 4 * (size_t)total_params();
    SCHK(s, hipMemcpyAsync(s->params, params, bytes, hipMemcpyDeviceToDevice, s->stream));
    SCHK(s, hipMemsetAsync(s->m, 0, bytes, s->stream));
    SCHK(s, hipMemsetAsync(s->v, 0, bytes, s->stream));
    s->adam_step = 0;
    s->have_grads = false;
    return prep_weights(s);
}

int fps_sur_get_params(fps_sur* s, float* params)
{
    if (!s || !params) return sfail(s, FPS_E_INVALID, "fps_sur_get_params: NULL argument");
    SCHK(s, hipMemcpyAsync(params, s->params, 4 * (size_t)total_params(), hipMemcpyDeviceToDevice, s->stream));
    return FPS_OK;
}

int fps_sur_forward(fps_sur* s, int32_t n, const void* x, float* y)
{
    if (!s || !x || !y) return sfail(s, FPS_E_INVALID, "fps_sur_forward: NULL argument");
    int rc = check_args(s, n);
    if (rc != FPS_OK) return rc;
    return forward(s, n, static_cast<const bf16*>(x), y);
}

int fps_sur_forward_noalloc(const float* params, int32_t n, int32_t H, int32_t W, const void* x, float* y,
                            void* stream)
{
    if (!params || !x || !y) return sfail(nullptr, FPS_E_INVALID, "fps_sur_forward_noalloc: NULL argument");
    if (n < 1 || H < CTH || W < TW || H % CTH || W % TW)
        return sfail(nullptr, FPS_E_INVALID,
                     "fps_sur_forward_noalloc: need n >= 1 and H, W positive multiples of %d, %d", CTH, TW);
    if ((int64_t)n * H * W > kNoallocPixels)
        return sfail(nullptr, FPS_E_CAPACITY, "fps_sur_forward_noalloc: %d x %d x %d pixels exceed the %lld of the "
                     "static scratch", n, H, W, (long long)kNoallocPixels);
    NoallocDevice d;
    int rc = noalloc_device(&d);
    if (rc != FPS_OK) return rc;
    // a handle on the stack over the scratch: the same kernels as fps_sur_forward
    fps_sur t;
    t.max_batch = n;
    t.H = H;
    t.W = W;
    t.cus = d.cus;
    t.stream = static_cast<hipStream_t>(stream);
    t.params = const_cast<float*>(params);       // read only: biases and the weights converted below
    size_t o = 0;
    for (int l = 0; l < kLayers; ++l) {
        t.wf[l] = reinterpret_cast<bf16*>(d.ptr + o);
        o += (2 * (size_t)kCout[l] * kp_of(kCin[l]) + 255) / 256 * 256;
    }
    bf16* a = reinterpret_cast<bf16*>(d.ptr + o);
    bf16* b = reinterpret_cast<bf16*>(d.ptr + o + kNoallocActBytes);
    t.act[0] = a;                                 // layer l reads act[l - 1] and writes act[l]
    t.act[1] = b;
    t.act[2] = a;
    t.act[3] = b;
    for (int l = 0; l < kLayers; ++l)
        hipLaunchKernelGGL(prep_weights_kernel, dim3(64), dim3(256), 0, t.stream, params + param_offset(l), kCin[l],
                           kCout[l], t.wf[l], (bf16*)nullptr);
    if (hipGetLastError() != hipSuccess) return sfail(nullptr, FPS_E_DEVICE, "fps_sur_forward_noalloc: launch failed");
    rc = forward(&t, n, static_cast<const bf16*>(x), y);
    if (rc != FPS_OK) snprintf(g_sur_err, sizeof(g_sur_err), "fps_sur_forward_noalloc: %s", t.err);
    return rc;
}

int fps_sur_gradients(fps_sur* s, int32_t n, const void* xv, const float* target, float* grads_out,
                      float* loss)
{
    if (!s || !xv || !target || !loss) return sfail(s, FPS_E_INVALID, "fps_sur_gradients: NULL argument");
    int rc = check_args(s, n);
    if (rc != FPS_OK) return rc;
    const bf16* x = static_cast<const bf16*>(xv);
    rc = forward(s, n, x, s->y);
    if (rc != FPS_OK) return rc;
    const int64_t npix = (int64_t)n * s->H * s->W;
    const float scale = 1.0f / (float)(npix * kOutUsed);
    hipLaunchKernelGGL(loss_kernel, dim3(kLossBlocks), dim3(kThreads), 0, s->stream, s->y, target, npix, scale,
                       s->dz5, s->lpart);
    hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(kThreads), 0, s->stream, s->lpart, kLossBlocks, scale, loss);
    SCHK(s, hipGetLastError());
    // layer 5 (no ReLU): dz5 -> dW5; its input gradient masked by the ReLU of
    // layer 4 is dz of layer 4.  Then down the layers, dz ping-ponging
    // between two buffers.
    rc = wgrad<64, 16>(s, n, s->act[3], s->dz5, 4);
    bf16* dz_cur = s->dz;
    bf16* dz_next = s->g;
    if (rc == FPS_OK) rc = conv<16, 64, 3>(s, n, s->dz5, s->wd[4], nullptr, dz_cur, s->act[3]);
    for (int l = 3; l >= 0 && rc == FPS_OK; --l) {
        if (l > 0) {
            rc = wgrad<64, 64>(s, n, s->act[l - 1], dz_cur, l);
            if (rc == FPS_OK) rc = conv<64, 64, 3>(s, n, dz_cur, s->wd[l], nullptr, dz_next, s->act[l - 1]);
            std::swap(dz_cur, dz_next);
        } else {
            rc = wgrad<16, 64>(s, n, x, dz_cur, 0);
        }
    }
    if (rc != FPS_OK) return rc;
    s->have_grads = true;
    if (grads_out)
        SCHK(s, hipMemcpyAsync(grads_out, s->grads, 4 * (size_t)total_params(), hipMemcpyDeviceToDevice, s->stream));
    return FPS_OK;
}

int fps_sur_adam(fps_sur* s, float lr)
{
    if (!s) return sfail(nullptr, FPS_E_INVALID, "fps_sur_adam: NULL argument");
    if (!s->have_grads) return sfail(s, FPS_E_STATE, "fps_sur_adam: no gradients computed");
    if (!(lr >= 0.0f) || !std::isfinite(lr)) return sfail(s, FPS_E_INVALID, "fps_sur_adam: bad learning rate");
    s->adam_step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - std::pow(b1, (float)s->adam_step), c2 = 1.0f - std::pow(b2, (float)s->adam_step);
    const int n = (int)total_params();
    WeightCopies wc{};
    for (int l = 0; l < kLayers; ++l) {
        wc.wf[l] = s->wf[l];
        wc.wd[l] = l > 0 ? s->wd[l] : nullptr;
        wc.off[l] = (int)param_offset(l);
        wc.cin[l] = kCin[l];
        wc.cout[l] = kCout[l];
    }
    wc.off[kLayers] = n;
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, s->stream, s->params, s->m, s->v,
                       s->grads, n, lr, b1, b2, 1e-8f, c1, c2, wc);
    SCHK(s, hipGetLastError());
    return FPS_OK;
}

int fps_sur_train_step(fps_sur* s, int32_t n, const void* x, const float* target, float lr, float* loss)
{
    int rc = fps_sur_gradients(s, n, x, target, nullptr, loss);
    if (rc != FPS_OK) return rc;
    return fps_sur_adam(s, lr);
}

int fps_sur_pack(int32_t nx, int32_t ny, const float* h, const float* hu, const float* hv, const float* z,
                 const int32_t* occupancy, int32_t inflow_side, int32_t inflow_c0, int32_t inflow_c1,
                 double inflow_depth, void* x, void* stream)
{
    if (nx < 1 || ny < 1 || !h || !hu || !hv || !z || !x || inflow_side < -1 || inflow_side > FPS_SIDE_N ||
        !std::isfinite(inflow_depth))
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_pack: bad argument");
    const int64_t npix = (int64_t)nx * ny;
    hipLaunchKernelGGL(pack_kernel, dim3((unsigned)std::min<int64_t>((npix + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), npix, nx, ny, h, hu, hv, z, occupancy, inflow_side,
                       inflow_c0, inflow_c1, (float)inflow_depth, static_cast<bf16*>(x));
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

int fps_sur_make_target(int64_t npix, const float* h0, const float* hu0, const float* hv0, const float* h1,
                        const float* hu1, const float* hv1, float* target, void* stream)
{
    if (npix < 1 || !h0 || !hu0 || !hv0 || !h1 || !hu1 || !hv1 || !target)
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_make_target: bad argument");
    hipLaunchKernelGGL(target_kernel, dim3(2048), dim3(256), 0, static_cast<hipStream_t>(stream), npix, h0, hu0,
                       hv0, h1, hu1, hv1, target);
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

int fps_sur_apply(int64_t npix, const float* y, float* h, float* hu, float* hv, float h_dry, float h_snap,
                  void* stream)
{
    if (npix < 1 || !y || !h || !hu || !hv || !(h_snap >= 0.0f))
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_apply: bad argument");
    hipLaunchKernelGGL(apply_kernel, dim3((unsigned)std::min<int64_t>((npix + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), npix, y, h, hu, hv, h_dry, h_snap);
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

int fps_sur_judge(int32_t na, int32_t stride, const float* x, const float* y, const uint8_t* state, int32_t nx,
                  int32_t ny, double dx, double dy, const float* ha, const float* qxa, const float* qya,
                  const float* hb, const float* qxb, const float* qyb, double tol, double h_dry,
                  const double* hr_thresholds, const float* hs, const float* qxs, const float* qys, double hr_margin,
                  double h_margin, int32_t* out3, void* stream)
{
    if (na < 0 || stride < 1 || nx < 1 || ny < 1 || !(dx > 0) || !(dy > 0) || !out3 || !hr_thresholds ||
        (na > 0 && (!x || !y || !state || !ha || !qxa || !qya || !hb || !qxb || !qyb)) ||
        (hs && (!qxs || !qys)) || !(hr_margin >= 0) || !(h_margin >= 0))
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_judge: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(fill_u8_kernel, dim3(1), dim3(64), 0, st, reinterpret_cast<uint8_t*>(out3), (int64_t)12);
    const JudgePick q{stride, hs, qxs, qys, (float)hr_margin, (float)h_margin, (float)h_dry,
                      (float)hr_thresholds[0], (float)hr_thresholds[1], (float)hr_thresholds[2]};
    const int64_t nt = hs ? (int64_t)na : ((int64_t)na + stride - 1) / stride;
    if (nt > 0) {
        hipLaunchKernelGGL(judge_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, na, q, x, y, state,
                           nx, ny, (float)dx, (float)dy, ha, qxa, qya, hb, qxb, qyb, (float)tol, out3);
    }
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

int fps_sur_judge_mask(int32_t na, int32_t stride, const float* x, const float* y, const uint8_t* state,
                       int32_t nx, int32_t ny, double dx, double dy, const float* hs, const float* qxs,
                       const float* qys, double h_dry, const double* hr_thresholds, double hr_margin, double h_margin,
                       int32_t halo, int32_t block, uint8_t* mask, void* stream)
{
    if (na < 0 || stride < 1 || nx < 1 || ny < 1 || !(dx > 0) || !(dy > 0) || halo < 0 || block < 1 || !mask ||
        (na > 0 && (!x || !y || !state)) || (hs && (!qxs || !qys || !hr_thresholds)) || !(hr_margin >= 0) ||
        !(h_margin >= 0))
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_judge_mask: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nm = (int64_t)((nx + block - 1) / block) * ((ny + block - 1) / block);
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)std::min<int64_t>((nm + 255) / 256, 1024)), dim3(256), 0, st,
                       mask, nm);
    const JudgePick q{stride, hs, qxs, qys, (float)hr_margin, (float)h_margin, (float)h_dry,
                      hs ? (float)hr_thresholds[0] : 0.0f, hs ? (float)hr_thresholds[1] : 0.0f,
                      hs ? (float)hr_thresholds[2] : 0.0f};
    const int64_t nt = hs ? (int64_t)na : ((int64_t)na + stride - 1) / stride;
    if (nt > 0)
        hipLaunchKernelGGL(judge_mask_kernel, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, st, na, q, x, y,
                           state, nx, ny, (float)dx, (float)dy, halo, block, mask);
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

int fps_sur_occupancy(int32_t na, const float* x, const float* y, const uint8_t* role, const uint8_t* state,
                      int32_t nx, int32_t ny, double dx, double dy, int32_t* counts, void* stream)
{
    if (na < 0 || nx < 1 || ny < 1 || !(dx > 0) || !(dy > 0) || !counts ||
        (na > 0 && (!x || !y || !role || !state)))
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_occupancy: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nc = (int64_t)nx * ny;
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)std::min<int64_t>((4 * nc + 255) / 256, 4096)), dim3(256), 0,
                       st, reinterpret_cast<uint8_t*>(counts), 4 * nc);
    if (na > 0)
        hipLaunchKernelGGL(occupancy_kernel, dim3((na + 255) / 256), dim3(256), 0, st, na, x, y, role, state, nx, ny,
                           (float)dx, (float)dy, counts);
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

int fps_sur_copy_state(int64_t npix, const float* h, const float* hu, const float* hv, float* h_out,
                       float* hu_out, float* hv_out, void* stream)
{
    if (npix < 1 || !h || !hu || !hv || !h_out || !hu_out || !hv_out)
        return sfail(nullptr, FPS_E_INVALID, "fps_sur_copy_state: bad argument");
    hipLaunchKernelGGL(copy3_kernel, dim3((unsigned)std::min<int64_t>((npix + 255) / 256, 4096)), dim3(256), 0,
                       static_cast<hipStream_t>(stream), npix, h, hu, hv, h_out, hu_out, hv_out);
    SCHK(nullptr, hipGetLastError());
    return FPS_OK;
}

const char* fps_sur_last_error(const fps_sur* s) { return s ? s->err : g_sur_err; }

}  // extern "C"
