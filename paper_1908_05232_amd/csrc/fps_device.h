// Device helpers shared by the step kernels of libfps (header-only so every
// translation unit inlines them; no relocatable device code is needed).
#pragma once

#include "fps_internal.h"

// Pointers read from memory are generic (flat) to the compiler; a cast to
// the global address space makes their loads and stores global_* ones, which
// wait on the vector-memory counter only.
#define FPS_GLOBAL __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ FPS_GLOBAL T* gmem(T* p)
{
    return (FPS_GLOBAL T*)p;
}

namespace fps {

// Scenario owning flattened index g: the largest s with off[s] <= g (off has
// S + 1 entries, non-decreasing).  Called with wave-uniform arguments.
__device__ __forceinline__ int find_scenario(const int* off, int S, int g)
{
    int lo = 0, hi = S - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The scenario record of a step kernel.  A launch that holds one scenario
// reads it from its kernel arguments (one round of dependent loads fewer than
// the device table the ensemble launches read).
template <bool kOne>
__device__ __forceinline__ const Scn& scn_at(const Batch& B, int sc)
{
    if constexpr (kOne) return B.one;
    else return B.scn[sc];
}

// Inclusive prefix sum over the 64 lanes of a wave by DPP lane moves (VALU
// only): shifts by 1, 2, 4 and 8 within each row of 16 lanes (lanes without a
// source add 0), then the row broadcasts of lanes 15 and 31 carry the row
// totals into the rows above.  Integer, so the result is exact.
__device__ __forceinline__ int wave_inclusive_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, true);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, true);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, true);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, true);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);  // row_bcast:15 into rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);  // row_bcast:31 into rows 2, 3
    return v;
}

// A step whose flood update is skipped: either it is the identity (nothing
// is wet, no inflow enters during the step, and the state already came out of
// a flood update, so dry cells carry no discharge; the 1 s dry step of sec. 3
// then only advances the pedestrians), or the flood is held by the caller
// (fps_set_flood_frozen: the pedestrians walk on a flood state set from
// outside).  Every kernel of the step evaluates this on the same device state
// before the finalize changes it.
__device__ __forceinline__ bool flood_skipped(const DevState* st)
{
    return st->frozen || (st->settled && !st->any_wet && st->inc == 0.0f);
}

__device__ __forceinline__ double hydro_q(const DevState* st, double t)
{
    int n = st->nh;
    if (n <= 0) return 0.0;
    if (t <= st->hyd_t[0]) return st->hyd_q[0];
    if (t >= st->hyd_t[n - 1]) return st->hyd_q[n - 1];
    for (int k = 0; k + 1 < n; ++k) {
        if (t >= st->hyd_t[k] && t <= st->hyd_t[k + 1]) {
            double w = (t - st->hyd_t[k]) / (st->hyd_t[k + 1] - st->hyd_t[k]);
            return st->hyd_q[k] + w * (st->hyd_q[k + 1] - st->hyd_q[k]);
        }
    }
    return st->hyd_q[n - 1];
}

// exact integral of the piecewise-linear hydrograph over [a, b] (sec. 3.1)
__device__ inline double hydro_integral(const DevState* st, double a, double b)
{
    if (st->nh <= 0 || !(b > a)) return 0.0;
    double total = 0.0, lo = a;
    for (int k = 0; k < st->nh; ++k) {
        double tk = st->hyd_t[k];
        if (tk > lo && tk < b) {
            total += 0.5 * (hydro_q(st, lo) + hydro_q(st, tk)) * (tk - lo);
            lo = tk;
        }
    }
    return total + 0.5 * (hydro_q(st, lo) + hydro_q(st, b)) * (b - lo);
}

// Exclusive scan of the bin histogram by one block of kScanThreads: tiles of
// 16 * kScanThreads counts, sixteen consecutive counts per lane (four 16-byte
// loads), a wave scan and a scan of the wave totals per tile.  The counts of
// up to four tiles are loaded in one round before any of them is scanned (a
// round per tile made the scan of a large grid a chain of dependent loads);
// the histogram is cleared behind the loads for the next step.
__device__ inline void block_scan_bins(const BinParams& b)
{
    constexpr int IPT = 16, TILES = 4, TILE = IPT * kScanThreads;
    __shared__ int wtot[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    int carry = 0;     // bins before the current tile (uniform)
    for (int base = 0; base < b.nbins; base += TILES * TILE) {
        int v[TILES][IPT];
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            const int k0 = base + t * TILE + IPT * threadIdx.x;
            if (k0 + IPT <= b.nbins) {
#pragma unroll
                for (int q = 0; q < IPT / 4; ++q) {
                    const int4 w = *reinterpret_cast<const int4*>(b.bin_count + k0 + 4 * q);
                    v[t][4 * q] = w.x; v[t][4 * q + 1] = w.y; v[t][4 * q + 2] = w.z; v[t][4 * q + 3] = w.w;
                }
            } else {
#pragma unroll
                for (int e = 0; e < IPT; ++e) v[t][e] = k0 + e < b.nbins ? b.bin_count[k0 + e] : 0;
            }
        }
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            const int k0 = base + t * TILE + IPT * threadIdx.x;
            if (k0 + IPT <= b.nbins) {
#pragma unroll
                for (int q = 0; q < IPT / 4; ++q)
                    *reinterpret_cast<int4*>(b.bin_count + k0 + 4 * q) = make_int4(0, 0, 0, 0);
            } else {
                for (int e = 0; e < IPT; ++e)
                    if (k0 + e < b.nbins) b.bin_count[k0 + e] = 0;
            }
        }
#pragma unroll
        for (int t = 0; t < TILES; ++t) {
            if (base + t * TILE >= b.nbins) break;      // uniform
            const int k0 = base + t * TILE + IPT * threadIdx.x;
            int tsum = 0;
#pragma unroll
            for (int e = 0; e < IPT; ++e) tsum += v[t][e];
            const int incl = wave_inclusive_scan(tsum);
            if (lane == kWave - 1) wtot[wid] = incl;
            __syncthreads();
            int wbase = 0, total = 0;
            for (int w = 0; w < kScanThreads / kWave; ++w) {
                const int x = wtot[w];
                wbase += w < wid ? x : 0;
                total += x;
            }
            int run = carry + wbase + incl - tsum;
            if (k0 + IPT <= b.nbins) {
#pragma unroll
                for (int q = 0; q < IPT / 4; ++q) {
                    int4 w;
                    w.x = run; run += v[t][4 * q];
                    w.y = run; run += v[t][4 * q + 1];
                    w.z = run; run += v[t][4 * q + 2];
                    w.w = run; run += v[t][4 * q + 3];
                    *reinterpret_cast<int4*>(b.bin_start + k0 + 4 * q) = w;
                }
            } else {
                for (int e = 0; e < IPT; ++e) {
                    if (k0 + e < b.nbins) b.bin_start[k0 + e] = run;
                    run += v[t][e];
                }
            }
            carry += total;
            __syncthreads();      // wtot is rewritten by the next tile
        }
    }
    if (threadIdx.x == 0) b.bin_start[b.nbins] = carry;
    __syncthreads();
}

// The middle step of the multi-block bin scan, by the scenario's end-of-step
// block: the chunk counts (written by the chunk-count launch) become their
// exclusive offsets in place, one value per thread per round, and the total
// closes the bin starts.
__device__ inline void block_scan_chunks(const BinParams& b)
{
    __shared__ int wtot[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    int carry = 0;
    for (int base = 0; base < b.nchunk; base += kScanThreads) {
        const int i = base + (int)threadIdx.x;
        const int v = i < b.nchunk ? b.csum[i] : 0;
        const int incl = wave_inclusive_scan(v);
        if (lane == kWave - 1) wtot[wid] = incl;
        __syncthreads();
        int wbase = 0, total = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            const int x = wtot[w];
            wbase += w < wid ? x : 0;
            total += x;
        }
        if (i < b.nchunk) b.csum[i] = carry + wbase + incl - v;
        carry += total;
        __syncthreads();      // wtot is rewritten by the next round
    }
    if (threadIdx.x == 0) b.bin_start[b.nbins] = carry;
    __syncthreads();
}

// Placement of the agents into their bins by rank, then the stable order: an
// agent's final slot counts the smaller ids of its own bin.  Whole-grid
// version, in two kernels (one thread per agent).  An agent alone in its bin
// (most of them in a sparse crowd) takes the bin's first slot in the
// placement pass; the others are marked (slot -1) for the order pass, which
// passes over everyone else after reading their slot and key (both read in
// agent order, no bin bounds).
__device__ inline void place_agent(const BinParams& b, int a)
{
    const int k = b.key[a], r = b.rank[a];
    const float x = b.x[a], y = b.y[a];
    if (k < 0) return;
    const int s0 = b.bin_start[k], s1 = b.bin_start[k + 1];
    if (s1 - s0 > 1) {
        b.perm_u[s0 + r] = a;
        b.slot[a] = -1;
    } else {
        b.slot[a] = s0;
        b.xy[s0] = make_float2(x, y);
    }
}
__device__ inline void sort_agent(const BinParams& b, int a)
{
    const int k = b.key[a], sl = b.slot[a];
    if (k < 0 || sl >= 0) return;
    const int s0 = b.bin_start[k], s1 = b.bin_start[k + 1];
    int below = 0;
    for (int s = s0; s < s1; ++s) below += b.perm_u[s] < a;
    const int f = s0 + below;
    b.slot[a] = f;
    b.xy[f] = make_float2(b.x[a], b.y[a]);
}

// Placement and stable order of at most kInlinePlace agents by one block,
// after its scan of the global histogram (grids with more bins than the LDS
// binning takes).  Every global load goes out in two rounds (the agents' keys,
// ranks and positions; then the bounds of their bins), the unordered
// placement lives in LDS, and an agent's final slot counts the smaller ids of
// its bin there.  Same results as place_agent followed by sort_agent.
__device__ inline void inline_bins_place(const BinParams& b)
{
    constexpr int APT = kInlinePlace / kScanThreads;
    __shared__ int lp[kInlinePlace];
    int key[APT], rank[APT], s0[APT], s1[APT];
    float ax[APT], ay[APT];
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const int a = threadIdx.x + q * kScanThreads, ac = a < b.na ? a : 0;
        const int k = b.key[ac];
        rank[q] = b.rank[ac];
        ax[q] = b.x[ac];
        ay[q] = b.y[ac];
        key[q] = a < b.na ? k : -1;
    }
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const int kc = key[q] >= 0 ? key[q] : 0;
        s0[q] = b.bin_start[kc];
        s1[q] = b.bin_start[kc + 1];
    }
#pragma unroll
    for (int q = 0; q < APT; ++q)
        if (key[q] >= 0) lp[s0[q] + rank[q]] = threadIdx.x + q * kScanThreads;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        if (key[q] < 0) continue;
        const int a = threadIdx.x + q * kScanThreads;
        int below = 0;
        for (int s = s0[q]; s < s1[q]; ++s) below += lp[s] < a;
        const int f = s0[q] + below;
        b.slot[a] = f;
        b.xy[f] = make_float2(ax[q], ay[q]);
    }
}

// One-block binning in LDS for small grids (nbins <= 16 * kScanThreads, at
// most kInlinePlace agents; dynamic shared memory of nbins + 1 + na words),
// run by a block of its own beside the end-of-step state update.  It starts
// from the agents' bin keys alone: a histogram by LDS atomics, the exclusive
// scan (sixteen bins per thread, the wave by shuffles, the waves in LDS), the
// placement by LDS atomics and the stable order by id; only the results are
// stored.  Being a function of the keys, it gives the same bins however often
// it runs on them (a scenario that did not step keeps its bins).  Same results
// as the global binning.
__device__ inline void lds_bins_build(const BinParams& b)
{
    constexpr int APT = kInlinePlace / kScanThreads;
    extern __shared__ int4 fin_lds4[];
    int* lb = reinterpret_cast<int*>(fin_lds4);    // [nbins + 1]: counts, then starts, then ends
    int* lp = lb + b.nbins + 1;                    // [na]: agents by bin, unordered
    __shared__ int wtot[kScanThreads / kWave];
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    const int k0 = 16 * threadIdx.x;
    const bool full = k0 + 16 <= b.nbins;
    int key[APT];
    float ax[APT], ay[APT];
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const int a = threadIdx.x + q * kScanThreads;
        key[q] = -1;
        if (a < b.na) {
            key[q] = b.key[a];
            ax[q] = b.x[a];
            ay[q] = b.y[a];
        }
    }
    if (full) {
#pragma unroll
        for (int q = 0; q < 4; ++q) reinterpret_cast<int4*>(lb + k0)[q] = make_int4(0, 0, 0, 0);
    } else {
        for (int e = k0; e < b.nbins; ++e) lb[e] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < APT; ++q)
        if (key[q] >= 0) atomicAdd(&lb[key[q]], 1);
    __syncthreads();
    int hist[16];
    if (full) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 w = reinterpret_cast<const int4*>(lb + k0)[q];
            hist[4 * q] = w.x; hist[4 * q + 1] = w.y; hist[4 * q + 2] = w.z; hist[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) hist[e] = k0 + e < b.nbins ? lb[k0 + e] : 0;
    }
    int tsum = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) tsum += hist[e];
    const int incl = wave_inclusive_scan(tsum);
    if (lane == kWave - 1) wtot[wid] = incl;
    __syncthreads();
    int run = incl - tsum, total = 0;
    for (int w = 0; w < kScanThreads / kWave; ++w) {
        run += w < wid ? wtot[w] : 0;
        total += wtot[w];
    }
    if (full) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int4 w;
            w.x = run; run += hist[4 * q];
            w.y = run; run += hist[4 * q + 1];
            w.z = run; run += hist[4 * q + 2];
            w.w = run; run += hist[4 * q + 3];
            reinterpret_cast<int4*>(b.bin_start + k0)[q] = w;
            reinterpret_cast<int4*>(lb + k0)[q] = w;
        }
    } else {
        for (int e = 0; e < 16 && k0 + e < b.nbins; ++e) {
            b.bin_start[k0 + e] = run;
            lb[k0 + e] = run;
            run += hist[e];
        }
    }
    if (threadIdx.x == 0) {
        b.bin_start[b.nbins] = total;
        lb[b.nbins] = total;
    }
    __syncthreads();
    // unordered placement: each agent takes the next free slot of its bin;
    // afterwards lb[k] is the end of bin k (= start of bin k + 1)
#pragma unroll
    for (int q = 0; q < APT; ++q)
        if (key[q] >= 0) lp[atomicAdd(&lb[key[q]], 1)] = threadIdx.x + q * kScanThreads;
    __syncthreads();
    // stable order: an agent's slot counts the smaller ids of its bin
#pragma unroll
    for (int q = 0; q < APT; ++q) {
        const int k = key[q];
        if (k < 0) continue;
        const int a = threadIdx.x + q * kScanThreads;
        const int s0 = k > 0 ? lb[k - 1] : 0, s1 = lb[k];
        int below = 0;
        for (int s = s0; s < s1; ++s) below += lp[s] < a;
        const int f = s0 + below;
        b.slot[a] = f;
        b.xy[f] = make_float2(ax[q], ay[q]);
    }
}

}  // namespace fps
