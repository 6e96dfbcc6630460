// Device helpers shared by the step kernels of libfps (header-only so every
// translation unit inlines them; no relocatable device code is needed).
#pragma once

#include "fps_internal.h"

namespace fps {

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
// 4 * kScanThreads counts, four consecutive counts per lane (16-byte loads), a
// wave scan by shuffles and a scan of the wave totals; the histogram is
// cleared behind the scan for the next step.
__device__ inline void block_scan_bins(const BinParams& b)
{
    __shared__ int wtot[kScanThreads / kWave];
    __shared__ int carry_s;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int base = 0; base < b.nbins; base += 4 * kScanThreads) {
        const int k0 = base + 4 * threadIdx.x;
        int v[4] = {0, 0, 0, 0};
        if (k0 + 3 < b.nbins) {
            int4 q = *reinterpret_cast<const int4*>(b.bin_count + k0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
            *reinterpret_cast<int4*>(b.bin_count + k0) = make_int4(0, 0, 0, 0);
        } else {
            for (int e = 0; e < 4; ++e)
                if (k0 + e < b.nbins) {
                    v[e] = b.bin_count[k0 + e];
                    b.bin_count[k0 + e] = 0;
                }
        }
        const int tsum = v[0] + v[1] + v[2] + v[3];
        int incl = tsum;
        for (int o = 1; o < kWave; o <<= 1) {
            int u = __shfl_up(incl, o, kWave);
            if (lane >= o) incl += u;
        }
        if (lane == kWave - 1) wtot[wid] = incl;
        __syncthreads();
        int wbase = 0, total = 0;
        for (int w = 0; w < kScanThreads / kWave; ++w) {
            int t = wtot[w];
            wbase += w < wid ? t : 0;
            total += t;
        }
        int run = carry_s + wbase + incl - tsum;
        for (int e = 0; e < 4; ++e) {
            if (k0 + e < b.nbins) b.bin_start[k0 + e] = run;
            run += v[e];
        }
        __syncthreads();
        if (threadIdx.x == 0) carry_s += total;
        __syncthreads();
    }
    if (threadIdx.x == 0) b.bin_start[b.nbins] = carry_s;
    __syncthreads();
}

}  // namespace fps
