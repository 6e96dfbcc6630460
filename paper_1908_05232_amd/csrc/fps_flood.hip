// Flood update of one time step on gfx950: the explicit first-order
// Godunov-type finite-volume scheme of Eq. (2) (sec. 2.2) for the shallow-water
// equations of Eq. (1), with wetting/drying and terrain treatment at every
// face, Manning friction, the inflow hydrograph of sec. 3.1, and the CFL time
// step of sec. 3 reduced on the device for the next step.
//
// Readings of the paper used here (the scheme is deferred to Wang et al. 2011):
//   HLLC face flux (Toro) with dry-bed wave speeds (or, selected per launch,
//   HLL for all three components); non-negative hydrostatic
//   reconstruction z_f = max(zL, zR), h* = h - (z_f - z), h* <= h_dry counts
//   as dry; bed slope as the one-sided pressure correction 1/2 g h*^2; walls by
//   mirrored ghost cells passing no mass; transmissive sides by copied ghosts;
//   splitting point-implicit Manning friction with a no-reversal limiter and
//   roughness n0 (1 + min(Np, cap)) from the evacuee counts (sec. 2.4).
//
// Design: one wave marches up a strip of 64 columns (62 outputs plus a halo
// column each side).  At every row each lane loads one cell (coalesced SoA
// rows), computes the y face above it in registers (the face below is carried
// from the previous row), and the x face to its east from its neighbour lane's
// state (cross-lane shuffle); the west face arrives from the neighbour lane.
// Every face is evaluated once; no LDS staging is needed.  Each wave writes
// partials (FP64 mass / volumes, FP32 max wave speed); a finalize kernel (one
// block per scenario) at the end of the step reduces them in a fixed order,
// advances time and sets the next time step (no cross-block fences inside the
// update).  One launch covers the flood tiles of every scenario of an
// ensemble; each wave finds its scenario and reads its parameters.
#include "fps_device.h"

namespace fps {
namespace {

struct Cell {
    float h, qx, qy, z, u, v;
};

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt_fast(float x) { return __builtin_amdgcn_sqrtf(x); }

// Whole-wave DPP shifts (a VALU move, no LDS traffic): lane i receives lane
// i + 1 (wave_shl:1) or lane i - 1 (wave_shr:1); the lane without a source
// receives 0 by the bound control (never used: lanes 0 and 63 are halo
// lanes), so no old value has to be set first.
__device__ __forceinline__ float lane_from_above(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x130, 0xF, 0xF, true));
}
__device__ __forceinline__ float lane_from_below(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 0x138, 0xF, 0xF, true));
}

// Cell (i, j) with i in [-1, nx], j in [-1, ny]; a ghost mirrors the adjacent
// interior cell (normal discharge negated at a wall).  Indices beyond the
// ghost layer clamp into the grid (their values are never used).  The raw
// load and the derived velocities are split so loads can be issued rows ahead.
struct Src {
    const FPS_GLOBAL float* __restrict__ h;
    const FPS_GLOBAL float* __restrict__ qx;
    const FPS_GLOBAL float* __restrict__ qy;
    const FPS_GLOBAL float* __restrict__ z;
};

// Element idx of a grid array: a 32-bit byte offset from a wave-uniform base
// (grids hold fewer than 2^30 cells), so the access is one global load or
// store with the base in scalar registers and no 64-bit address arithmetic.
template <class T>
__device__ __forceinline__ T ld(const FPS_GLOBAL T* base, uint32_t idx)
{
    return *(const FPS_GLOBAL T*)((const FPS_GLOBAL char*)base + idx * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void st_at(FPS_GLOBAL T* base, uint32_t idx, T v)
{
    *(FPS_GLOBAL T*)((FPS_GLOBAL char*)base + idx * (uint32_t)sizeof(T)) = v;
}

__device__ __forceinline__ Cell load_raw(const Src& src, const FvParams& p, int ii, int j)
{
    const int jj = min(max(j, 0), p.ny - 1);
    const uint32_t k = (uint32_t)jj * (uint32_t)p.nx + (uint32_t)ii;
    Cell c;
    c.h = ld(src.h, k);
    c.qx = ld(src.qx, k);
    c.qy = ld(src.qy, k);
    c.z = ld(src.z, k);
    return c;
}

__device__ __forceinline__ void derive(const FvParams& p, Cell& c, bool mirror_x, int j)
{
    if (mirror_x) c.qx = -c.qx;
    if ((j < 0 && p.bc[2] == FPS_BC_WALL) || (j >= p.ny && p.bc[3] == FPS_BC_WALL)) c.qy = -c.qy;
    float r = c.h > p.eps ? rcp(c.h) : 0.0f;
    c.u = c.qx * r;
    c.v = c.qy * r;
}

// Hydrostatic pressure 1/2 g h^2 of a reconstructed depth.  Never contracted
// into a neighbouring add: the flux and the bed-slope correction must use the
// identical rounded value for still water to stay exactly at rest.
__device__ __forceinline__ float pressure(float half_g, float h)
{
#pragma clang fp contract(off)
    return half_g * h * h;
}

// One face: reconstruction, then the HLLC flux.  (un, ut) are the normal and
// tangential velocities of each side; F0 mass, F1 normal momentum, F2
// tangential momentum; pL / pR the pressures 1/2 g h*^2 of the reconstructed
// depth each side sees (the bed-slope correction of the two cells).
// Written without divergent branches: every case is evaluated and selected.
// kHll: the tangential momentum by the HLL average of the two outer waves, in
// the same left-anchored form as mass and normal momentum, instead of from the
// side of the contact wave.
template <bool kHll>
__device__ __forceinline__ void face_flux(const FvParams& p, float hL, float unL, float utL,
                                          float zL, float hR, float unR, float utR, float zR,
                                          bool wall, float& F0, float& F1, float& F2,
                                          float& pL, float& pR)
{
    // max(zL, zR) by compare and select: fmaxf would first quieten the two
    // raw loaded values (bed elevations are finite, and the result is one of
    // them either way)
    float zf = zL > zR ? zL : zR;
    float hl = hL - (zf - zL);
    float hr = hR - (zf - zR);
    hl = hl > p.eps ? hl : 0.0f;
    hr = hr > p.eps ? hr : 0.0f;
    pL = pressure(p.half_g, hl);
    pR = pressure(p.half_g, hr);
    const bool wetL = hl > 0.0f, wetR = hr > 0.0f;
    float cL = sqrt_fast(p.g * hl), cR = sqrt_fast(p.g * hr);
    float us = 0.5f * (unL + unR) + cL - cR;
    float cs = 0.5f * (cL + cR) + 0.25f * (unL - unR);
    float sL = fminf(unL - cL, us - cs);
    float sR = fmaxf(unR + cR, us + cs);
    // dry-bed wave speeds
    sL = wetL ? (wetR ? sL : unL - cL) : unR - 2.0f * cR;
    sR = wetL ? (wetR ? sR : unL + 2.0f * cL) : unR + cR;
    float qL = hl * unL, qR = hr * unR;
    float FL0 = qL, FL1 = qL * unL + pL, FL2 = qL * utL;
    float FR0 = qR, FR1 = qR * unR + pR, FR2 = qR * utR;
    // HLL written from the left flux with the wave speeds clamped to either
    // side of zero: the one formula is the left flux exactly when sL >= 0
    // (the clamped sL is 0), the right flux up to rounding when sR <= 0, and
    // the star-region flux between, with no selection of the case; identical
    // states give F exactly.  Only a face dry on both sides has a zero
    // denominator, and its flux is set to zero below.
    const float sLc = fminf(sL, 0.0f), sRc = fmaxf(sR, 0.0f);
    float inv = rcp(sRc - sLc);
    float H0 = FL0 + sLc * ((FL0 - FR0) + sRc * (hr - hl)) * inv;
    float H1 = FL1 + sLc * ((FL1 - FR1) + sRc * (qR - qL)) * inv;
    float H2;
    if (kHll) {
        H2 = FL2 + sLc * ((FL2 - FR2) + sRc * (hr * utR - hl * utL)) * inv;
    } else {
        // tangential momentum from the side of the contact wave: s_M = num /
        // den with den < 0 here, so s_M >= 0 iff num <= 0 (the left state for
        // sL >= 0, the right one for sR <= 0)
        float num = sL * hr * (unR - sR) - sR * hl * (unL - sL);
        H2 = H0 * (num <= 0.0f ? utL : utR);
    }
    const bool none = !(wetL || wetR);
    F0 = (none || wall) ? 0.0f : H0;
    F1 = none ? 0.0f : H1;
    F2 = (none || wall) ? 0.0f : H2;
}

// Wave reductions by DPP lane moves (VALU only, no LDS round trips): pairs,
// quads (quad permutes), eight and sixteen lanes (half-row and row mirrors)
// leave every lane of a row with the row's total; the row broadcasts of lanes
// 15 and 31 then add the rows, lane 63 ending with the wave's total, which is
// returned to every lane.  Rows a broadcast does not write receive 0; the
// first four moves have a source for every lane, so no old value is set for
// them.  A fixed order, so the result is reproducible.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_i32(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xF, kRowMask == 0xF);
}
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_i32<kCtrl, kRowMask>((int)(unsigned)u);
    const unsigned hi = (unsigned)dpp_i32<kCtrl, kRowMask>((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
constexpr int kQuadSwap1 = 0xB1, kQuadSwap2 = 0x4E;          // quad_perm [1,0,3,2], [2,3,0,1]
constexpr int kRowHalfMirror = 0x141, kRowMirror = 0x140, kRowBcast15 = 0x142, kRowBcast31 = 0x143;

__device__ __forceinline__ double readlane_f64(double v, int l)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<kQuadSwap1, 0xF>(v);
    v += dpp_f64<kQuadSwap2, 0xF>(v);
    v += dpp_f64<kRowHalfMirror, 0xF>(v);
    v += dpp_f64<kRowMirror, 0xF>(v);
    v += dpp_f64<kRowBcast15, 0xA>(v);
    v += dpp_f64<kRowBcast31, 0xC>(v);
    return readlane_f64(v, kWave - 1);
}
// Maximum of non-negative floats (the wave speeds): their bit patterns order
// as the values do, so an unsigned maximum of the bits serves (one
// instruction; a NaN, above every finite pattern, comes through to the time
// step check).  The rows a broadcast skips receive 0 = +0.0.
__device__ __forceinline__ float wave_max(float v)
{
    unsigned u = __builtin_bit_cast(unsigned, v);
    u = max(u, (unsigned)dpp_i32<kQuadSwap1, 0xF>((int)u));
    u = max(u, (unsigned)dpp_i32<kQuadSwap2, 0xF>((int)u));
    u = max(u, (unsigned)dpp_i32<kRowHalfMirror, 0xF>((int)u));
    u = max(u, (unsigned)dpp_i32<kRowMirror, 0xF>((int)u));
    u = max(u, (unsigned)dpp_i32<kRowBcast15, 0xA>((int)u));
    u = max(u, (unsigned)dpp_i32<kRowBcast31, 0xC>((int)u));
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane((int)u, kWave - 1));
}

// Blocks are handed to the 8 XCDs round-robin by block id; this mapping gives
// each XCD a contiguous run of tiles (a band of rows), so the halo columns and
// rows shared by neighbouring tiles are reused in that XCD's L2.
__device__ __forceinline__ int xcd_tile_block(int b, int nblocks)
{
    const int per = nblocks >> 3;          // nblocks is a multiple of 8
    return (b & 7) * per + (b >> 3);
}

template <bool kOne, bool kHll>
__global__ __launch_bounds__(kFvBlock) void fv_step_kernel(Batch B)
{
    const int lane = threadIdx.x & (kWave - 1);
    // the wave's flattened tile, its scenario and local tile (wave-uniform)
    const int g = __builtin_amdgcn_readfirstlane(
        xcd_tile_block(blockIdx.x, B.fv_blocks) * (kFvBlock / kWave) + (int)(threadIdx.x >> 6));
    int sc, tile;
    if (kOne) {
        sc = 0;
        tile = g;
    } else if (B.s_only >= 0) {
        sc = B.s_only;
        tile = g;
    } else {
        if (g >= B.total_tiles) return;
        sc = find_scenario(B.tile_off, B.S, g);
        tile = g - B.tile_off[sc];
    }
    // parameters by value: wave-uniform registers, not reloaded after the
    // stores of the march (which the compiler cannot tell apart from them)
    const FvParams p = scn_at<kOne>(B, sc).fv;
    if (tile >= p.ntiles) return;
    DevState* st = p.st;
    if (!st->active || flood_skipped(st)) return;
    // the state words are read through a generic pointer: make them wave-uniform
    // so that the buffer selects below are scalar
    const int cur = __builtin_amdgcn_readfirstlane(st->cur);
    // selects, not indexing, so that the parameter copy stays in registers
    const Src src{gmem<const float>(cur ? p.h[1] : p.h[0]), gmem<const float>(cur ? p.qx[1] : p.qx[0]),
                  gmem<const float>(cur ? p.qy[1] : p.qy[0]), gmem(p.z)};
    FPS_GLOBAL float* __restrict__ ho = gmem(cur ? p.h[0] : p.h[1]);
    FPS_GLOBAL float* __restrict__ qxo = gmem(cur ? p.qx[0] : p.qx[1]);
    FPS_GLOBAL float* __restrict__ qyo = gmem(cur ? p.qy[0] : p.qy[1]);
    const FPS_GLOBAL int32_t* __restrict__ npp = gmem(p.np);
    double m_acc = 0.0, vout_acc = 0.0, vclip_acc = 0.0;
    float smax = 0.0f;
    const float dt = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, st->dt)));
    const float inc = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, st->inc)));
    const float lx = dt * p.inv_dx, ly = dt * p.inv_dy;

    {
        const int sx = tile % p.nsx, sy = tile / p.nsx;
        if (p.jmask) {
            // judge region: skip waves whose output cells meet no set block
            const int bx0 = sx * kStrip / p.jb, bx1 = min(sx * kStrip + kStrip - 1, p.nx - 1) / p.jb;
            const int by0 = sy * p.H / p.jb, by1 = (min(sy * p.H + p.H, p.ny) - 1) / p.jb;
            int any = 0;
            for (int by = by0; by <= by1 && !any; ++by)
                for (int bx = bx0; bx <= bx1; ++bx) any |= p.jmask[by * p.jbx + bx];
            if (!any) {
                if (lane == 0) {
                    FPS_GLOBAL double* dst = gmem(&p.partials[4 * tile]);
                    dst[0] = 0.0;
                    dst[1] = 0.0;
                    dst[2] = 0.0;
                    dst[3] = 0.0;
                }
                return;
            }
        }
        const int i = sx * kStrip - 1 + lane;
        const int ii = min(max(i, 0), p.nx - 1);
        const int j0 = sy * p.H, j1 = min(j0 + p.H, p.ny);
        const bool out_lane = lane >= 1 && lane <= kStrip && i < p.nx;
        const bool mirror_x = (i < 0 && p.bc[0] == FPS_BC_WALL) || (i >= p.nx && p.bc[1] == FPS_BC_WALL);
        const bool xwall = (i == -1 && p.bc[0] == FPS_BC_WALL) ||
                           (i + 1 == p.nx && p.bc[1] == FPS_BC_WALL);
        bool inflow_col = false;
        if (p.inflow_side == FPS_SIDE_S || p.inflow_side == FPS_SIDE_N)
            inflow_col = i >= p.c0 && i < p.c1;

        // Row j0-1 now, rows j0 .. j0+2 in flight (rows past j1 are never needed).  The first pass of the loop
        // (j = j0-1) only forms the face below row j0, so every y face goes
        // through the same code (same rounding) whatever the tile height.
        Cell c = load_raw(src, p, ii, j0 - 1);
        Cell pf0 = load_raw(src, p, ii, j0);
        Cell pf1 = {}, pf2 = {};
        if (j0 + 1 <= j1) pf1 = load_raw(src, p, ii, j0 + 1);
        if (j0 + 2 <= j1) pf2 = load_raw(src, p, ii, j0 + 2);
        derive(p, c, mirror_x, j0 - 1);
        float Fs0 = 0.0f, Fs1 = 0.0f, Fs2 = 0.0f, pS = 0.0f;
        for (int j = j0 - 1; j < j1; ++j) {
            Cell nb = pf0;
            pf0 = pf1;
            pf1 = pf2;
            if (j + 4 <= j1) pf2 = load_raw(src, p, ii, j + 4);   // rows above the tile's last need stay unread
            derive(p, nb, mirror_x, j + 1);
            // north face (y normal: pass v as normal, u as tangential)
            float Fn0, Fn1, Fn2, pN, pS_next;
            face_flux<kHll>(p, c.h, c.v, c.u, c.z, nb.h, nb.v, nb.u, nb.z,
                      (j + 1 == 0 && p.bc[2] == FPS_BC_WALL) || (j + 1 == p.ny && p.bc[3] == FPS_BC_WALL),
                      Fn0, Fn1, Fn2, pN, pS_next);
            if (j < j0) {
                Fs0 = Fn0;
                Fs1 = Fn1;
                Fs2 = Fn2;
                pS = pS_next;
                c = nb;
                continue;
            }
            const uint32_t k = (uint32_t)j * (uint32_t)p.nx + (uint32_t)i;
            int npc = 0;
            if (out_lane) npc = ld(npp, k);
            // east face with the neighbour lane's cell
            float eh = lane_from_above(c.h), eu = lane_from_above(c.u);
            float ev = lane_from_above(c.v), ez = lane_from_above(c.z);
            float Fe0, Fe1, Fe2, pE, pW_east;
            face_flux<kHll>(p, c.h, c.u, c.v, c.z, eh, eu, ev, ez, xwall, Fe0, Fe1, Fe2, pE, pW_east);
            // west face = east face of the lane below
            float Fw0 = lane_from_below(Fe0), Fw1 = lane_from_below(Fe1);
            float Fw2 = lane_from_below(Fe2), pW = lane_from_below(pW_east);
            if (out_lane) {
                float hn = c.h - (lx * (Fe0 - Fw0) + ly * (Fn0 - Fs0));
                float qxn = c.qx - (lx * ((Fe1 - pE) - (Fw1 - pW)) + ly * (Fn2 - Fs2));
                float qyn = c.qy - (ly * ((Fn1 - pN) - (Fs1 - pS)) + lx * (Fe2 - Fw2));
                // inflow line source (sec. 3.1)
                bool inflow = false;
                if (p.inflow_side == FPS_SIDE_S) inflow = inflow_col && j == 0;
                else if (p.inflow_side == FPS_SIDE_N) inflow = inflow_col && j == p.ny - 1;
                else if (p.inflow_side == FPS_SIDE_W) inflow = i == 0 && j >= p.c0 && j < p.c1;
                else if (p.inflow_side == FPS_SIDE_E) inflow = i == p.nx - 1 && j >= p.c0 && j < p.c1;
                if (inflow) hn += inc;
                // non-negative depth, no discharge on dry cells
                if (hn < 0.0f) {
                    vclip_acc += (double)(-hn);
                    hn = 0.0f;
                }
                if (!(hn > p.eps)) {
                    qxn = 0.0f;
                    qyn = 0.0f;
                }
                if (hn > p.eps) {
                    float r = rcp(hn);
                    float u = qxn * r, v = qyn * r;
                    float V2 = u * u + v * v;
                    if (V2 > 0.0f) {
                        // Manning friction, splitting point-implicit
                        float n = p.n_base + (float)min(npc, p.np_cap) * p.n_base;
                        float speed = sqrt_fast(V2);
                        float hm13 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(hn) * (1.0f / 3.0f));
                        float Cf = p.g * n * n * hm13;
                        float Sx = -Cf * u * speed, Sy = -Cf * v * speed;
                        float a = dt * Cf * r * rcp(speed);
                        float Dx = 1.0f + a * (2.0f * u * u + v * v);
                        float Dy = 1.0f + a * (2.0f * v * v + u * u);
                        float dqx = dt * Sx * rcp(Dx), dqy = dt * Sy * rcp(Dy);
                        if (fabsf(dqx) > fabsf(qxn)) dqx = -qxn;
                        if (fabsf(dqy) > fabsf(qyn)) dqy = -qyn;
                        qxn += dqx;
                        qyn += dqy;
                        u = qxn * r;
                        v = qyn * r;
                    }
                    float cel = sqrt_fast(p.g * hn);
                    smax = fmaxf(smax, fmaxf((fabsf(u) + cel) * p.inv_dx, (fabsf(v) + cel) * p.inv_dy));
                }
                m_acc += (double)hn;
                // outflow through transmissive sides
                if (i == 0 || i == p.nx - 1 || j == 0 || j == p.ny - 1) {    // rare: skipped by most waves
                    if (i == 0 && p.bc[0] == FPS_BC_TRANSMISSIVE) vout_acc -= (double)Fw0 * dt * p.dy;
                    if (i == p.nx - 1 && p.bc[1] == FPS_BC_TRANSMISSIVE) vout_acc += (double)Fe0 * dt * p.dy;
                    if (j == 0 && p.bc[2] == FPS_BC_TRANSMISSIVE) vout_acc -= (double)Fs0 * dt * p.dx;
                    if (j == p.ny - 1 && p.bc[3] == FPS_BC_TRANSMISSIVE) vout_acc += (double)Fn0 * dt * p.dx;
                }
                st_at(ho, k, hn);
                st_at(qxo, k, qxn);
                st_at(qyo, k, qyn);
            }
            Fs0 = Fn0;
            Fs1 = Fn1;
            Fs2 = Fn2;
            pS = pS_next;
            c = nb;
        }
    }
    // wave partials, fixed reduction order; reduced by the finalize kernel.
    // Outflow and clipped volumes are zero in almost every wave (outflow only
    // on transmissive sides, clipping only where a depth went negative): their
    // sums are skipped when no lane holds a non-zero value.
    m_acc = wave_sum(m_acc);
    if (__ballot(vout_acc != 0.0)) vout_acc = wave_sum(vout_acc);
    else vout_acc = 0.0;
    if (__ballot(vclip_acc != 0.0)) vclip_acc = wave_sum(vclip_acc);
    else vclip_acc = 0.0;
    smax = wave_max(smax);
    if (lane == 0) {
        FPS_GLOBAL double* dst = gmem(&p.partials[4 * tile]);
        dst[0] = m_acc;
        dst[1] = vout_acc;
        dst[2] = vclip_acc;
        dst[3] = (double)smax;
        // one flag per group of blocks; every wet wave of the group stores the
        // same 1 with a plain store (no read-modify-write, nothing to wait for:
        // the wave ends as soon as its stores are issued)
        if (smax > 0.0f) st_at(gmem(p.wet), (uint32_t)(kWetStride * (blockIdx.x & (kWetSlots - 1))), 1);
    }
}

// ---------------------------------------------------------------------------
// Second-order variant (the scheme the paper reduced to first order, sec.
// 2.2): MUSCL reconstruction of (h, eta = h + z, u, v) per direction with
// the minmod limiter (zero slope where the cell or a neighbour in that
// direction is dry, and in ghost cells), the hydrostatic reconstruction and
// the HLLC / HLL flux of the first-order scheme at each face on the
// reconstructed states, the second-order bed-slope form of Audusse et al.
// (2004) (each face adds g/2 (h_f^2 - h*_f^2) to its side's normal momentum,
// each cell the centred -g/2 (h_w + h_e)(z_e - z_w)), and Heun's two-stage
// Runge-Kutta step: U1 = U + dt L(U), U' = (U + U1 + dt L(U1)) / 2, with the
// depth cleanup after each stage and the inflow and friction once after both.
//
// The march of the first-order update widened to the stencil of radius 2: a
// wave holds 64 adjacent columns and owns the middle kStrip2 (two halo lanes
// a side), marching down its rows with a window of three rows in registers.
// Each row is reconstructed once per direction: in x from the neighbour
// lanes' cells (DPP moves), in y from the window.  Each face is evaluated
// once: a lane forms its west face (the east state of the lane below against
// its own west state) and takes its east face from the lane above; the face
// below row r is formed when row r is reconstructed and, carried, is the
// face above row r - 1, which is then complete and updated (one row behind).
// ---------------------------------------------------------------------------
constexpr int kStrip2 = kWave - 4;      // output columns of one wave in the second-order march

struct V4 {
    float h, eta, u, v;     // depth, surface elevation, velocities (0 where h <= h_dry)
};

__device__ __forceinline__ float minmod(float a, float b)
{
    return a * b > 0.0f ? (fabsf(a) <= fabsf(b) ? a : b) : 0.0f;
}

// the velocities and surface of a raw cell (a ghost mirrors the adjacent
// interior cell: the normal velocity negated at a wall)
__device__ __forceinline__ V4 v4_of(const FvParams& p, const Cell& c, bool mirror_x, int j)
{
    V4 v;
    v.h = c.h;
    v.eta = c.h + c.z;
    const float r = c.h > p.eps ? rcp(c.h) : 0.0f;
    v.u = c.qx * r;
    v.v = c.qy * r;
    if (mirror_x) v.u = -v.u;
    if ((j < 0 && p.bc[2] == FPS_BC_WALL) || (j >= p.ny && p.bc[3] == FPS_BC_WALL)) v.v = -v.v;
    return v;
}

// cell b reconstructed at its two faces in one direction, from its
// neighbours a (before) and c (after): lo at the face towards a, hi at the
// face towards c; no slope for a ghost or next to a dry cell
__device__ __forceinline__ void recon(const FvParams& p, const V4& a, const V4& b, const V4& c, bool ghost,
                                      V4& lo, V4& hi)
{
    lo = b;
    hi = b;
    if (ghost || !(a.h > p.eps) || !(b.h > p.eps) || !(c.h > p.eps)) return;
    const float mh = minmod(c.h - b.h, b.h - a.h), me = minmod(c.eta - b.eta, b.eta - a.eta);
    const float mu = minmod(c.u - b.u, b.u - a.u), mv = minmod(c.v - b.v, b.v - a.v);
    hi.h += 0.5f * mh;
    hi.eta += 0.5f * me;
    hi.u += 0.5f * mu;
    hi.v += 0.5f * mv;
    lo.h += -0.5f * mh;
    lo.eta += -0.5f * me;
    lo.u += -0.5f * mu;
    lo.v += -0.5f * mv;
}

// one face between reconstructed states L and R in the face's normal
// direction (un, ut: normal and tangential velocity): flux and, per side, the
// hydrostatic depth
template <bool kHll>
__device__ __forceinline__ void face2(const FvParams& p, float hL, float etaL, float unL, float utL, float hR,
                                      float etaR, float unR, float utR, bool wall, float& F0, float& F1,
                                      float& F2, float& hsL, float& hsR)
{
    const float zL = etaL - hL, zR = etaR - hR;
    const bool wL = hL > p.eps, wR = hR > p.eps;
    float pL, pR;
    face_flux<kHll>(p, hL, wL ? unL : 0.0f, wL ? utL : 0.0f, zL, hR, wR ? unR : 0.0f, wR ? utR : 0.0f, zR, wall,
                    F0, F1, F2, pL, pR);
    // the hydrostatic depths themselves (the pressures are their squares)
    const float zf = zL > zR ? zL : zR;
    const float hl = hL - (zf - zL), hr = hR - (zf - zR);
    hsL = hl > p.eps ? hl : 0.0f;
    hsR = hr > p.eps ? hr : 0.0f;
}

// One Runge-Kutta stage of the second-order variant over one tile (kStage 1:
// U1 = U + dt L(U) into the stage buffer; kStage 2: U' = (U + U1 + dt L(U1))
// / 2 into the other ping-pong buffer, then inflow, friction, volumes and the
// wave speed).  The outflow and clipped volumes of stage 1 are left in the
// tile's partial slots for stage 2 to add to (each stage counts half).
template <bool kOne, bool kHll, int kStage>
__global__ __launch_bounds__(kFvBlock) void fv2_stage_kernel(Batch B)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int g = __builtin_amdgcn_readfirstlane(
        xcd_tile_block(blockIdx.x, B.fv_blocks) * (kFvBlock / kWave) + (int)(threadIdx.x >> 6));
    int sc, tile;
    if (kOne) {
        sc = 0;
        tile = g;
    } else if (B.s_only >= 0) {
        sc = B.s_only;
        tile = g;
    } else {
        if (g >= B.total_tiles) return;
        sc = find_scenario(B.tile_off, B.S, g);
        tile = g - B.tile_off[sc];
    }
    const FvParams p = scn_at<kOne>(B, sc).fv;
    if (tile >= p.ntiles) return;
    DevState* st = p.st;
    if (!st->active || flood_skipped(st)) return;
    const int cur = __builtin_amdgcn_readfirstlane(st->cur);
    const Src s0{gmem<const float>(cur ? p.h[1] : p.h[0]), gmem<const float>(cur ? p.qx[1] : p.qx[0]),
                 gmem<const float>(cur ? p.qy[1] : p.qy[0]), gmem(p.z)};
    const Src s1{gmem<const float>(p.h1), gmem<const float>(p.qx1), gmem<const float>(p.qy1), gmem(p.z)};
    const Src& src = kStage == 1 ? s0 : s1;        // the state the residual is taken of
    const float dt = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, st->dt)));
    const float inc = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, st->inc)));
    const float lx = dt * p.inv_dx, ly = dt * p.inv_dy;
    const int sx = tile % p.nsx, sy = tile / p.nsx;
    const int i = sx * kStrip2 - 2 + lane;
    const int ii = min(max(i, 0), p.nx - 1);
    const int j0 = sy * p.H, j1 = min(j0 + p.H, p.ny);
    const bool out_lane = lane >= 2 && lane < 2 + kStrip2 && i < p.nx;
    const bool gx = i < 0 || i >= p.nx;       // ghost column (no x slope)
    const bool mirror_x = (i < 0 && p.bc[0] == FPS_BC_WALL) || (i >= p.nx && p.bc[1] == FPS_BC_WALL);
    // the west face of this lane's column is a wall face
    const bool xwall = (i == 0 && p.bc[0] == FPS_BC_WALL) || (i == p.nx && p.bc[1] == FPS_BC_WALL);
    double m_acc = 0.0, vout_acc = 0.0, vclip_acc = 0.0;
    float smax = 0.0f;
    FPS_GLOBAL double* part = gmem(&p.partials[4 * tile]);

    // window: rows r - 1, r, r + 1 (raw and derived), two rows in flight
    Cell cm = load_raw(src, p, ii, j0 - 2), c0 = load_raw(src, p, ii, j0 - 1), cp = load_raw(src, p, ii, j0);
    Cell pf0 = load_raw(src, p, ii, j0 + 1), pf1 = load_raw(src, p, ii, j0 + 2);
    V4 vm = v4_of(p, cm, mirror_x, j0 - 2), v0 = v4_of(p, c0, mirror_x, j0 - 1), vp = v4_of(p, cp, mirror_x, j0);
    // carried from row r - 1: its north state, and its residual but the north face
    V4 nprev = {};
    Cell crow = {};                                // raw values of row r - 1 (the stage's base)
    float Fs0 = 0.0f, Fs1 = 0.0f, Fs2 = 0.0f, hsS = 0.0f, hS = 0.0f, zS = 0.0f, hN = 0.0f, zN = 0.0f;
    float ex0 = 0.0f, ex1 = 0.0f, ex2 = 0.0f, cx = 0.0f;
    double rate_x = 0.0;                           // outflow rate through the row's x boundary faces
    for (int r = j0 - 1; r <= j1; ++r) {
        // y reconstruction of row r from the window (rows r - 1, r, r + 1)
        V4 sr, nr;
        recon(p, vm, v0, vp, r < 0 || r >= p.ny, sr, nr);
        if (r >= j0) {
            // the face below row r: north state of row r - 1 against the south state of row r
            float F0, F1, F2, hsl, hsr;
            face2<kHll>(p, nprev.h, nprev.eta, nprev.v, nprev.u, sr.h, sr.eta, sr.v, sr.u,
                        (r == 0 && p.bc[2] == FPS_BC_WALL) || (r == p.ny && p.bc[3] == FPS_BC_WALL), F0, F1,
                        F2, hsl, hsr);
            if (r > j0) {
                // row r - 1 is complete: its north face is this one
                const int jr = r - 1;
                const float cy = p.half_g * (hN * hN - hsl * hsl) - p.half_g * (hS * hS - hsS * hsS) +
                                 p.half_g * (hS + hN) * (zN - zS);
                const float dh = -(lx * ex0 + ly * (F0 - Fs0));
                const float dqx = -(lx * (ex1 + cx) + ly * (F2 - Fs2));
                const float dqy = -(ly * ((F1 - Fs1) + cy) + lx * ex2);
                if (out_lane) {
                    const uint32_t k = (uint32_t)jr * (uint32_t)p.nx + (uint32_t)i;
                    double rate = rate_x;
                    if (jr == 0 && p.bc[2] == FPS_BC_TRANSMISSIVE) rate -= (double)Fs0 * p.dx;
                    if (jr == p.ny - 1 && p.bc[3] == FPS_BC_TRANSMISSIVE) rate += (double)F0 * p.dx;
                    vout_acc += 0.5 * rate * (double)dt;
                    float h = crow.h + dh, qx = crow.qx + dqx, qy = crow.qy + dqy;
                    if (h < 0.0f) {
                        vclip_acc += 0.5 * (double)(-h);
                        h = 0.0f;
                    }
                    if (!(h > p.eps)) {
                        qx = 0.0f;
                        qy = 0.0f;
                    }
                    if (kStage == 1) {
                        st_at(gmem(p.h1), k, h);
                        st_at(gmem(p.qx1), k, qx);
                        st_at(gmem(p.qy1), k, qy);
                    } else {
                        float hn = 0.5f * (ld(s0.h, k) + h), qxn = 0.5f * (ld(s0.qx, k) + qx),
                              qyn = 0.5f * (ld(s0.qy, k) + qy);
                        bool inflow = false;
                        if (p.inflow_side == FPS_SIDE_S) inflow = jr == 0 && i >= p.c0 && i < p.c1;
                        else if (p.inflow_side == FPS_SIDE_N) inflow = jr == p.ny - 1 && i >= p.c0 && i < p.c1;
                        else if (p.inflow_side == FPS_SIDE_W) inflow = i == 0 && jr >= p.c0 && jr < p.c1;
                        else if (p.inflow_side == FPS_SIDE_E) inflow = i == p.nx - 1 && jr >= p.c0 && jr < p.c1;
                        if (inflow) hn += inc;
                        if (!(hn > p.eps)) {
                            qxn = 0.0f;
                            qyn = 0.0f;
                        }
                        if (hn > p.eps) {
                            const float rr = rcp(hn);
                            float u = qxn * rr, v = qyn * rr;
                            const float V2 = u * u + v * v;
                            if (V2 > 0.0f) {
                                // Manning friction, splitting point-implicit (as in the first-order update)
                                const int npc = ld(gmem<const int32_t>(p.np), k);
                                const float n = p.n_base + (float)min(npc, p.np_cap) * p.n_base;
                                const float speed = sqrt_fast(V2);
                                const float hm13 = __builtin_amdgcn_exp2f(-__builtin_amdgcn_logf(hn) * (1.0f / 3.0f));
                                const float Cf = p.g * n * n * hm13;
                                const float Sx = -Cf * u * speed, Sy = -Cf * v * speed;
                                const float a = dt * Cf * rr * rcp(speed);
                                const float Dx = 1.0f + a * (2.0f * u * u + v * v);
                                const float Dy = 1.0f + a * (2.0f * v * v + u * u);
                                float dfx = dt * Sx * rcp(Dx), dfy = dt * Sy * rcp(Dy);
                                if (fabsf(dfx) > fabsf(qxn)) dfx = -qxn;
                                if (fabsf(dfy) > fabsf(qyn)) dfy = -qyn;
                                qxn += dfx;
                                qyn += dfy;
                                u = qxn * rr;
                                v = qyn * rr;
                            }
                            const float cel = sqrt_fast(p.g * hn);
                            smax = fmaxf(smax, fmaxf((fabsf(u) + cel) * p.inv_dx, (fabsf(v) + cel) * p.inv_dy));
                        }
                        m_acc += (double)hn;
                        st_at(gmem(cur ? p.h[0] : p.h[1]), k, hn);
                        st_at(gmem(cur ? p.qx[0] : p.qx[1]), k, qxn);
                        st_at(gmem(cur ? p.qy[0] : p.qy[1]), k, qyn);
                    }
                }
            }
            Fs0 = F0;
            Fs1 = F1;
            Fs2 = F2;
            hsS = hsr;
        }
        if (r >= j0 && r < j1) {
            // x reconstruction of row r from the neighbour lanes, its west face,
            // and its east face from the lane above
            const V4 w{lane_from_below(v0.h), lane_from_below(v0.eta), lane_from_below(v0.u), lane_from_below(v0.v)};
            const V4 e{lane_from_above(v0.h), lane_from_above(v0.eta), lane_from_above(v0.u), lane_from_above(v0.v)};
            V4 wr, er;
            recon(p, w, v0, e, gx, wr, er);
            const V4 el{lane_from_below(er.h), lane_from_below(er.eta), lane_from_below(er.u), lane_from_below(er.v)};
            float Fw0, Fw1, Fw2, hsw_l, hsw_r;
            face2<kHll>(p, el.h, el.eta, el.u, el.v, wr.h, wr.eta, wr.u, wr.v, xwall, Fw0, Fw1, Fw2, hsw_l, hsw_r);
            const float Fe0 = lane_from_above(Fw0), Fe1 = lane_from_above(Fw1), Fe2 = lane_from_above(Fw2);
            const float hsE = lane_from_above(hsw_l);
            const float zW = wr.eta - wr.h, zE = er.eta - er.h;
            cx = p.half_g * (er.h * er.h - hsE * hsE) - p.half_g * (wr.h * wr.h - hsw_r * hsw_r) +
                 p.half_g * (wr.h + er.h) * (zE - zW);
            ex0 = Fe0 - Fw0;
            ex1 = Fe1 - Fw1;
            ex2 = Fe2 - Fw2;
            rate_x = 0.0;
            if (i == 0 && p.bc[0] == FPS_BC_TRANSMISSIVE) rate_x -= (double)Fw0 * p.dy;
            if (i == p.nx - 1 && p.bc[1] == FPS_BC_TRANSMISSIVE) rate_x += (double)Fe0 * p.dy;
            hS = sr.h;
            zS = sr.eta - sr.h;
            hN = nr.h;
            zN = nr.eta - nr.h;
            crow = c0;
        }
        nprev = nr;
        // advance the window
        cm = c0;
        c0 = cp;
        cp = pf0;
        pf0 = pf1;
        if (r + 4 <= j1 + 1) pf1 = load_raw(src, p, ii, r + 4);     // rows past the last one needed stay unread
        vm = v0;
        v0 = vp;
        vp = v4_of(p, cp, mirror_x, r + 2);
    }
    // the two stages' volumes in the tile's partials (stage 1 leaves its
    // outflow and clipped volumes there for stage 2)
    vout_acc = wave_sum(vout_acc);
    vclip_acc = wave_sum(vclip_acc);
    if (kStage == 1) {
        if (lane == 0) {
            part[1] = vout_acc;
            part[2] = vclip_acc;
        }
        return;
    }
    m_acc = wave_sum(m_acc);
    smax = wave_max(smax);
    if (lane == 0) {
        const double vo1 = part[1], vc1 = part[2];
        part[0] = m_acc;
        part[1] = vo1 + vout_acc;
        part[2] = vc1 + vclip_acc;
        part[3] = (double)smax;
        if (smax > 0.0f) st_at(gmem(p.wet), (uint32_t)(kWetStride * (blockIdx.x & (kWetSlots - 1))), 1);
    }
}

// Scan of the current state only: mass, wetness and the time step that the
// next update will use (no time advance).  One scenario; one partial per block.
__global__ __launch_bounds__(kFvBlock) void fv_scan_kernel(Batch B, int sc)
{
    const FvParams& p = B.scn[sc].fv;
    const int cur = p.st->cur;
    const float* __restrict__ hh = p.h[cur];
    const float* __restrict__ qxx = p.qx[cur];
    const float* __restrict__ qyy = p.qy[cur];
    double m_acc = 0.0;
    float smax = 0.0f;
    const int64_t nc = (int64_t)p.nx * p.ny;
    for (int64_t k = (int64_t)blockIdx.x * kFvBlock + threadIdx.x; k < nc;
         k += (int64_t)gridDim.x * kFvBlock) {
        float h = hh[k];
        m_acc += (double)h;
        if (h > p.eps) {
            float r = rcp(h);
            float u = qxx[k] * r, v = qyy[k] * r;
            float cel = sqrt_fast(p.g * h);
            smax = fmaxf(smax, fmaxf((fabsf(u) + cel) * p.inv_dx, (fabsf(v) + cel) * p.inv_dy));
        }
    }
    __shared__ double wred[kFvBlock / kWave][2];
    m_acc = wave_sum(m_acc);
    smax = wave_max(smax);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        wred[threadIdx.x >> 6][0] = m_acc;
        wred[threadIdx.x >> 6][1] = (double)smax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s3 = 0;
        for (int w = 0; w < kFvBlock / kWave; ++w) {
            s0 += wred[w][0];
            s3 = fmax(s3, wred[w][1]);
        }
        double* dst = &p.partials[4 * blockIdx.x];
        dst[0] = s0;
        dst[1] = 0.0;
        dst[2] = 0.0;
        dst[3] = s3;
    }
}

// Exact integral over [a, b] of the piecewise-linear hydrograph (sec. 3.1),
// on one wave whose lane k holds knot k (tk, qk) for k < nh: lane k takes the
// part of [a, b] in [t_k, t_k+1] by the trapezoid rule (exact on a linear
// piece), lane 0 the constant part before the first knot, lane nh - 1 the
// constant part after the last; the pieces are added in time order.  Every
// lane returns the total.
__device__ double wave_hydro_integral(int nh, double tk, double qk, double a, double b)
{
    const int lane = threadIdx.x & (kWave - 1);
    // the next knot from the lane above (a whole-wave DPP shift; lane 63,
    // which gets 0, has no next knot: nh <= 64)
    const double tn = dpp_f64<0x130, 0xF>(tk), qn = dpp_f64<0x130, 0xF>(qk);
    if (nh <= 0 || !(b > a)) return 0.0;
    double piece = 0.0, before = 0.0, after = 0.0;
    if (lane + 1 < nh) {
        const double lo = fmax(a, tk), hi = fmin(b, tn);
        if (hi > lo) {
            const double ql = qk + ((lo - tk) / (tn - tk)) * (qn - qk);
            const double qh = qk + ((hi - tk) / (tn - tk)) * (qn - qk);
            piece = 0.5 * (ql + qh) * (hi - lo);
        }
    }
    if (lane == 0 && a < tk) before = qk * (fmin(b, tk) - a);
    if (lane == nh - 1 && b > tk) after = qk * (b - fmax(a, tk));
    double total = readlane_f64(before, 0);
    for (unsigned long long m = __ballot(piece != 0.0); m; m &= m - 1)
        total += readlane_f64(piece, __builtin_ctzll(m));
    return total + readlane_f64(after, nh - 1);
}

// End of a step: blocks (scenario, 0) update the state, blocks (scenario, 1)
// rebuild the neighbour bins of scenarios binned in LDS; the two run side by
// side (they share no data).  The state update reduces the flood partials in
// a fixed order, advances time, sets the next CFL time step (sec. 3) and
// inflow depth, applies the sandbag drops of the step to the barrier line
// (sec. 2.4) and, for scenarios binned in global memory, scans the histogram
// of the new agent bins (and, for small agent counts, places the agents in bin
// order), or, for scenarios with many bins, the chunk counts of the
// multi-block scan.  Mode 1 only recomputes the time step and mass of the current state.
template <bool kOne>
__global__ __launch_bounds__(kScanThreads) void finalize_kernel(Batch B, int mode, int s_first)
{
    const int sc = s_first + blockIdx.x;
    const Scn& S = scn_at<kOne>(B, sc);
    if (blockIdx.y == 1) {
        if (S.lds_bins && S.na > 0) lds_bins_build(S.bins);
        return;
    }
    // the parameters used, in registers: loaded in the first round, not
    // reloaded after the stores below
    const FvParams& p = S.fv;
    DevState* gst = p.st;
    const double* partials = p.partials;
    int32_t* wet = p.wet;
    const int ntiles = p.ntiles, n_inflow = p.n_inflow, inflow_side = p.inflow_side;
    const double dxdy = p.dxdy;
    const float cfl = p.cfl, dt_max = p.dt_max, dn = inflow_side <= 1 ? p.dx : p.dy;
    const bool jmask = p.jmask != nullptr;
    const int na = S.na, inline_place = S.inline_place, lds_bins = S.lds_bins, nline = S.bar.nline;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    // The scenario's state words go through LDS: one cooperative load, the
    // serial end-of-step logic on the copy, one cooperative store.  Nothing
    // else touches them while this block runs.  The hydrograph knots stay out
    // of the copy (they do not change): they are loaded into registers, one
    // knot per lane, and the first wave uses them.
    __shared__ DevState sst;
    constexpr int kWords = (int)(sizeof(DevState) / sizeof(uint32_t));
    constexpr int kHyd0 = (int)(offsetof(DevState, hyd_t) / sizeof(uint32_t));
    constexpr int kHyd1 = (int)(offsetof(DevState, step) / sizeof(uint32_t));
    constexpr int kCopy = kHyd0 + kWords - kHyd1;
    static_assert(sizeof(DevState) % sizeof(uint32_t) == 0, "DevState is copied as words");
    static_assert(offsetof(DevState, hyd_q) == offsetof(DevState, hyd_t) + sizeof(double) * kMaxHydro &&
                  offsetof(DevState, step) == offsetof(DevState, hyd_q) + sizeof(double) * kMaxHydro,
                  "the hydrograph knots are one run of words");
    static_assert(kCopy <= kScanThreads && kMaxHydro <= kWave, "one word per thread, one knot per lane");
    // Every load of the block goes out before the first wait: the state words
    // and the hydrograph knots into registers (written to LDS afterwards), and
    // eight flood partials per thread.  The loads are unconditional, at
    // clamped indices, and the values past the end are dropped when summed: a
    // load under a condition makes the compiler wait for it before the
    // lanes that skip it may touch its register.
    const int cw = threadIdx.x < kHyd0 ? (int)threadIdx.x : (int)threadIdx.x - kHyd0 + kHyd1;
    const uint32_t word = reinterpret_cast<const uint32_t*>(gst)[threadIdx.x < kCopy ? cw : 0];
    const double hk_t = gst->hyd_t[lane], hk_q = gst->hyd_q[lane];
    // the flood partials summed in tile order
    double m = 0.0, vo = 0.0, vc = 0.0, sm = 0.0;
    {
        constexpr int kPU = 8;
        const double2* P2 = reinterpret_cast<const double2*>(partials);
        double2 a[kPU], c[kPU];
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            const int b = threadIdx.x + u * kScanThreads, bc = b < ntiles ? b : 0;
            a[u] = P2[2 * bc];
            c[u] = P2[2 * bc + 1];
        }
        if (threadIdx.x < kCopy) reinterpret_cast<uint32_t*>(&sst)[cw] = word;
#pragma unroll
        for (int u = 0; u < kPU; ++u) {
            if (threadIdx.x + u * kScanThreads < ntiles) {
                m += a[u].x;
                vo += a[u].y;
                vc += c[u].x;
                sm = fmax(sm, c[u].y);
            }
        }
        for (int b = threadIdx.x + kPU * kScanThreads; b < ntiles; b += kScanThreads) {
            m += partials[4 * b + 0];
            vo += partials[4 * b + 1];
            vc += partials[4 * b + 2];
            sm = fmax(sm, partials[4 * b + 3]);
        }
    }
    __syncthreads();
    DevState* st = &sst;
    if (mode == 0 && !st->active) return;     // the whole block: one LDS word
    const bool skipped = mode == 0 && flood_skipped(st);
    if (skipped) {
        m = 0.0;
        vo = 0.0;
        vc = 0.0;
        sm = 0.0;
    }
    // the pedestrians of this step have read the wetness flags: clear them
    if (threadIdx.x < kWetSlots) wet[kWetStride * threadIdx.x] = 0;
    __shared__ double red[kScanThreads / kWave][4];
    m = wave_sum(m);
    vo = wave_sum(vo);
    vc = wave_sum(vc);
    sm = (double)wave_max((float)sm);     // the partials hold FP32 wave speeds
    if (lane == 0) {
        red[wid][0] = m;
        red[wid][1] = vo;
        red[wid][2] = vc;
        red[wid][3] = sm;
    }
    __syncthreads();
    if (wid == 0) {
        // the serial end of the step, on every lane of the first wave (same
        // values); lane 0 stores
        // lanes 0-3 combine one quantity each over the waves, in wave order
        double acc = 0.0;
        if (lane < 4) {
            acc = red[0][lane];
            for (int w = 1; w < kScanThreads / kWave; ++w)
                acc = lane == 3 ? fmax(acc, red[w][lane]) : acc + red[w][lane];
        }
        const double M = readlane_f64(acc, 0), VO = readlane_f64(acc, 1), VC = readlane_f64(acc, 2),
                     SM = readlane_f64(acc, 3);
        double t = st->t, v_out = st->v_out, v_clip = st->v_clip, v_in = st->v_in, mass = st->mass;
        int64_t step = st->step;
        float dt = st->dt, dt_prev = st->dt_prev;
        int cur = st->cur, flood_steps = st->flood_steps, settled = st->settled, any_wet = st->any_wet;
        int status = st->status;
        if (mode == 0) {
            t += (double)dt;
            step += 1;
            dt_prev = dt;
            if (!skipped) {
                v_out += VO;
                v_clip += VC * dxdy;
                v_in += (double)st->inc * (double)n_inflow * dxdy;
                cur ^= 1;
                flood_steps += 1;
                settled = 1;
            }
        }
        if (!skipped) {
            const float smax = (float)SM;
            mass = M * dxdy;
            any_wet = smax > 0.0f;
            dt = any_wet && !jmask ? fminf(cfl / smax, dt_max) : dt_max;
        }
        float inc = 0.0f;
        if (inflow_side >= 0)
            inc = (float)(wave_hydro_integral(st->nh, hk_t, hk_q, t, t + (double)dt) / (double)dn);
        if (!isfinite(mass) || !(dt > 0.0f) || !isfinite(dt) || !(SM == SM)) status = FPS_E_NUMERIC;
        if (lane == 0) {
            st->t = t;
            st->step = step;
            st->dt_prev = dt_prev;
            st->v_out = v_out;
            st->v_clip = v_clip;
            st->v_in = v_in;
            st->cur = cur;
            st->flood_steps = flood_steps;
            st->settled = settled;
            st->mass = mass;
            st->any_wet = any_wet;
            st->dt = dt;
            st->inc = inc;
            st->status = status;
            // sandbag write-back: drops of this step applied to the barrier line in order
            if (mode == 0 && na > 0) {
                const int D = st->drops;
                st->drops = 0;
                st->drops_total += D;
                if (!st->done && nline > 0) {
                    const BarrierParams& Bb = S.bar;     // read only while a barrier is built
                    int bags = st->bags + D;
                    int cell = st->active_cell, layers = st->layers_done, fin = 0;
                    while (!fin && bags >= Bb.bags_per) {
                        bags -= Bb.bags_per;
                        const float th = layers == Bb.n_layers - 1 ? Bb.t_last : Bb.t_bag;
                        Bb.z[Bb.line[cell]] += th;
                        cell += 1;
                        if (cell == Bb.nline) {
                            cell = 0;
                            layers += 1;
                            if (layers >= Bb.n_layers) fin = 1;
                        }
                    }
                    st->bags = bags;
                    st->active_cell = cell;
                    st->layers_done = layers;
                    st->done = fin;
                }
            }
            if (mode == 0) st->active = !(st->t_end > 0.0) || t < st->t_end;
        }
    }
    __syncthreads();
    if (threadIdx.x < kCopy)
        reinterpret_cast<uint32_t*>(gst)[cw] = reinterpret_cast<const uint32_t*>(&sst)[cw];
    if (mode == 0 && na > 0 && !lds_bins) {
        const BinParams bp = S.bins;
        if (bp.nchunk > 0) {
            block_scan_chunks(bp);      // the chunk scans follow in a launch of their own
        } else {
            block_scan_bins(bp);
            if (inline_place) inline_bins_place(bp);
        }
    }
}

// After the last step of a call: scenarios whose state sits in the scratch
// buffer copy it back to the caller's buffers (grid: blocks x scenarios).
__global__ void sync_back_kernel(Batch B)
{
    const FvParams& p = B.scn[blockIdx.y].fv;
    if (p.st->cur == 0) return;
    const int64_t nc = (int64_t)p.nx * p.ny;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nc;
         k += (int64_t)gridDim.x * blockDim.x) {
        p.h[0][k] = p.h[1][k];
        p.qx[0][k] = p.qx[1][k];
        p.qy[0][k] = p.qy[1][k];
    }
}
__global__ void reset_cur_kernel(Batch B)
{
    for (int s = threadIdx.x; s < B.S; s += blockDim.x) B.scn[s].fv.st->cur = 0;
}

// Streaming probe: n_in arrays read and n_out arrays written, 16 bytes a
// lane, grid-stride; out_k = sum of the inputs + k, so every input byte is
// used.  A bandwidth ceiling for kernels that stream SoA fields.
template <int NIN, int NOUT>
__global__ __launch_bounds__(256) void stream_probe_kernel(float* __restrict__ buf, int64_t n4, int64_t stride4)
{
    const float4* in = reinterpret_cast<const float4*>(buf);
    float4* out = reinterpret_cast<float4*>(buf) + NIN * stride4;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        float4 a[NIN];
#pragma unroll
        for (int k = 0; k < NIN; ++k) a[k] = in[k * stride4 + i];
        float4 t = a[0];
#pragma unroll
        for (int k = 1; k < NIN; ++k) t = make_float4(t.x + a[k].x, t.y + a[k].y, t.z + a[k].z, t.w + a[k].w);
#pragma unroll
        for (int k = 0; k < NOUT; ++k)
            out[k * stride4 + i] = make_float4(t.x + (float)k, t.y + (float)k, t.z + (float)k, t.w + (float)k);
    }
}

}  // namespace

hipError_t launch_stream_probe(float* buf, int64_t n, int64_t stride, int n_in, int n_out, int blocks, hipStream_t s)
{
    const int64_t n4 = n / 4, s4 = stride / 4;
    const dim3 grid(blocks), block(256);
    if (n_in == 1 && n_out == 1) hipLaunchKernelGGL((stream_probe_kernel<1, 1>), grid, block, 0, s, buf, n4, s4);
    else if (n_in == 5 && n_out == 3) hipLaunchKernelGGL((stream_probe_kernel<5, 3>), grid, block, 0, s, buf, n4, s4);
    else if (n_in == 4 && n_out == 3) hipLaunchKernelGGL((stream_probe_kernel<4, 3>), grid, block, 0, s, buf, n4, s4);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

int fv_rows_per_wave(int nx, int ny)
{
    // long marches on large grids (halo rows amortised), short ones on small
    // grids so that there are enough waves to spread over the 1024 SIMDs
    const int64_t nsx = (nx + kStrip - 1) / kStrip;
    int H = 64;
    while (H > 4 && nsx * ((ny + H - 1) / H) < 4096) H >>= 1;
    return H;
}

int fv_tiles2(int nx, int ny, int H)
{
    const int64_t nsx = (nx + kStrip2 - 1) / kStrip2;
    return (int)(nsx * ((ny + H - 1) / H));
}

int fv_strip(bool order2) { return order2 ? kStrip2 : kStrip; }

int fv_tiles(int nx, int ny, int H)
{
    const int64_t nsx = (nx + kStrip - 1) / kStrip;
    return (int)(nsx * ((ny + H - 1) / H));
}

int fv_blocks_for_tiles(int64_t tiles)
{
    const int64_t blocks = (tiles + kFvBlock / kWave - 1) / (kFvBlock / kWave);
    return (int)((blocks + 7) / 8 * 8);    // a multiple of the 8 XCDs
}

hipError_t launch_fv(const Batch& b, hipStream_t s)
{
    if (b.fv_blocks > 0 && b.order2) {
        const dim3 grid(b.fv_blocks), block(kFvBlock);
        if (b.S == 1) {
            if (b.hll) {
                hipLaunchKernelGGL((fv2_stage_kernel<true, true, 1>), grid, block, 0, s, b);
                hipLaunchKernelGGL((fv2_stage_kernel<true, true, 2>), grid, block, 0, s, b);
            } else {
                hipLaunchKernelGGL((fv2_stage_kernel<true, false, 1>), grid, block, 0, s, b);
                hipLaunchKernelGGL((fv2_stage_kernel<true, false, 2>), grid, block, 0, s, b);
            }
        } else {
            if (b.hll) {
                hipLaunchKernelGGL((fv2_stage_kernel<false, true, 1>), grid, block, 0, s, b);
                hipLaunchKernelGGL((fv2_stage_kernel<false, true, 2>), grid, block, 0, s, b);
            } else {
                hipLaunchKernelGGL((fv2_stage_kernel<false, false, 1>), grid, block, 0, s, b);
                hipLaunchKernelGGL((fv2_stage_kernel<false, false, 2>), grid, block, 0, s, b);
            }
        }
        return hipGetLastError();
    }
    if (b.fv_blocks > 0) {
        const dim3 grid(b.fv_blocks), block(kFvBlock);
        if (b.S == 1) {
            if (b.hll) hipLaunchKernelGGL((fv_step_kernel<true, true>), grid, block, 0, s, b);
            else hipLaunchKernelGGL((fv_step_kernel<true, false>), grid, block, 0, s, b);
        } else {
            if (b.hll) hipLaunchKernelGGL((fv_step_kernel<false, true>), grid, block, 0, s, b);
            else hipLaunchKernelGGL((fv_step_kernel<false, false>), grid, block, 0, s, b);
        }
    }
    return hipGetLastError();
}

hipError_t launch_fv_scan(const Batch& b, int scenario, int ntiles, hipStream_t s)
{
    hipLaunchKernelGGL(fv_scan_kernel, dim3(ntiles), dim3(kFvBlock), 0, s, b, scenario);
    return hipGetLastError();
}

hipError_t prepare_finalize(int lds_bytes)
{
    static int granted = 0;     // the attribute is per kernel: raise it once to the largest size
    if (lds_bytes <= granted) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)finalize_kernel<true>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e == hipSuccess)
        e = hipFuncSetAttribute((const void*)finalize_kernel<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds_bytes);
    if (e == hipSuccess) granted = lds_bytes;
    return e;
}

hipError_t launch_finalize(const Batch& b, int mode, int s_first, int count, hipStream_t s)
{
    // the binning blocks only where some scenario is binned in LDS
    const bool bins = mode == 0 && b.fin_lds_bytes > 0;
    const dim3 grid(count, bins ? 2 : 1);
    const int lds = bins ? b.fin_lds_bytes : 0;
    if (b.S == 1) hipLaunchKernelGGL(finalize_kernel<true>, grid, dim3(kScanThreads), lds, s, b, mode, s_first);
    else hipLaunchKernelGGL(finalize_kernel<false>, grid, dim3(kScanThreads), lds, s, b, mode, s_first);
    return hipGetLastError();
}

hipError_t launch_sync_back(const Batch& b, int64_t max_cells, hipStream_t s)
{
    int gx = (int)std::min<int64_t>((max_cells + 255) / 256, 2048);
    hipLaunchKernelGGL(sync_back_kernel, dim3(std::max(gx, 1), b.S), dim3(256), 0, s, b);
    hipLaunchKernelGGL(reset_cur_kernel, dim3(1), dim3(256), 0, s, b);
    return hipGetLastError();
}

}  // namespace fps
