// Internal declarations of libfps: device-resident step state, kernel
// parameter blocks and launchers.  Not part of the public ABI (include/fps.h).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "fps.h"

namespace fps {

constexpr int kWave = 64;
constexpr int kStrip = kWave - 2;      // output columns of one wave in the flood march
constexpr int kFvBlock = 256;          // 4 waves
constexpr int kPedBlock = 64;
constexpr int kScanThreads = 1024;
constexpr int kMaskBits = 128;       // obstacle bitmask per cell (uint4)
constexpr int kMaxHydro = 64;

// Scalars that live in device memory so that n steps run without the host.
struct DevState {
    double t;              // time at the start of the next step
    double mass;           // sum h dx dy after the last step
    double v_in, v_out, v_clip;
    double hyd_t[kMaxHydro], hyd_q[kMaxHydro];
    int64_t step;
    unsigned long long ped_steps;  // agent-steps of non-exited agents
    float dt;              // step length of the next step
    float dt_prev;         // step length of the last step
    float inc;             // inflow depth of the next step
    int32_t nh;
    int32_t any_wet;
    int32_t status;
    uint32_t fv_ctr, ped_ctr;
    // sandbag barrier (sec. 2.4)
    int32_t active, layers_done, bags, done, drops, drops_total;
    int32_t pad[2];
};

struct FvParams {
    const float* __restrict__ h;
    const float* __restrict__ qx;
    const float* __restrict__ qy;
    float* __restrict__ ho;
    float* __restrict__ qxo;
    float* __restrict__ qyo;
    const float* __restrict__ z;
    const int32_t* __restrict__ np;
    DevState* st;
    double* partials;      // [nblocks][4]: mass sum, outflow volume, clipped depth sum, max speed
    // (the flood kernels only write them; the finalize kernel reduces them)
    int nx, ny, H, nsx, ntiles, nblocks;
    int bc[4];
    int inflow_side, c0, c1, n_inflow;
    int np_cap;
    int mode;              // 0 = step, 1 = scan the current state only (first time step)
    float dx, dy, inv_dx, inv_dy, g, half_g, eps, cfl, dt_max, n_base;
    double dxdy;
};

struct PedParams {
    float* __restrict__ x;
    float* __restrict__ y;
    float* __restrict__ vx;
    float* __restrict__ vy;
    const float* __restrict__ vbase;
    const uint8_t* __restrict__ role;
    uint8_t* __restrict__ state;
    uint8_t* __restrict__ cls;
    int32_t* __restrict__ dest;
    float* __restrict__ timer;
    int na;
    const float* __restrict__ h;   // flood state after this step's update
    const float* __restrict__ qx;
    const float* __restrict__ qy;
    float* z;
    int32_t* np;
    const float* __restrict__ dist;
    const uint8_t* __restrict__ walk;
    int n_dest, n_exit;
    const int32_t* __restrict__ bin_start;   // bins of the positions at the start of the step
    const float2* __restrict__ xy;           // positions in bin order
    const int32_t* __restrict__ slot;        // each agent's place in that order
    const uint4* __restrict__ wmask;         // per cell: obstacle cells within r_cut (bit per offset)
    int32_t* bin_count;                      // histogram of the new positions
    int32_t* rank;
    int32_t* key;
    DevState* st;
    int nx, ny, bsx, bsy, nbx, nby, Rx, Ry, nblocks;
    int use_wmask;                           // masks valid: (2Rx+1)(2Ry+1) <= 128
    float dx, dy, eps, tau, a_over_m, inv_b, two_r, radius, r_cut, r_arrive;
    float v_class[5], hr_t[3], pick_s, drop_s;
    int storage_dest, barrier_dest;
    const double* fv_partials;               // flood partials of this step (wetness)
    int fv_blocks;
};

// Sandbag barrier of sec. 2.4: the fill order and layer rules.
struct BarrierParams {
    float* z;
    const int32_t* line;
    int nline, n_layers, bags_per;
    float t_bag, t_last;
};

struct BinParams {
    const float* x;
    const float* y;
    const uint8_t* state;
    const uint8_t* role;
    int32_t* bin_count;
    int32_t* bin_start;
    int32_t* rank;
    int32_t* key;
    int32_t* perm_u;
    int32_t* perm;
    float2* xy;
    int32_t* slot;
    int32_t* np;
    int na, nbins, nx, ny, bsx, bsy, nbx;
    float dx, dy;
};

// End of a step, one block: reduction of the flood partials (time, next time
// step, inflow, volumes), sandbag write-back, and the scan of the new bins.
struct FinParams {
    FvParams fv;
    BarrierParams bar;
    BinParams bins;
    int do_barrier, do_scan;
};

// launchers (stream-ordered, no synchronisation)
hipError_t launch_finalize(const FinParams& f, hipStream_t s);
hipError_t launch_fv(const FvParams& p, hipStream_t s);
int fv_blocks(int nx, int ny, int H);
int fv_rows_per_wave(int nx, int ny);
hipError_t launch_ped(const PedParams& p, hipStream_t s);
hipError_t launch_bin_keys(const BinParams& b, hipStream_t s);   // keys + ranks from positions
hipError_t launch_bin_scan(const BinParams& b, hipStream_t s);
hipError_t launch_bin_place(const BinParams& b, hipStream_t s);
hipError_t launch_bin_sort(const BinParams& b, hipStream_t s);
hipError_t launch_count(const BinParams& b, hipStream_t s);      // per-cell evacuee counts
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_hazard(const float* h, const float* qx, const float* qy, float* hr, int64_t n,
                         float eps, hipStream_t s);
hipError_t launch_agent_stats(const uint8_t* state, const uint8_t* cls, int na, int32_t* out11,
                              hipStream_t s);
// bad2[0]: agents outside the domain; bad2[1]: invalid role / state / destination
hipError_t launch_wall_mask(const uint8_t* walk, uint4* mask, int nx, int ny, int Rx, int Ry,
                            hipStream_t s);
hipError_t launch_check_agents(const float* x, const float* y, const uint8_t* role,
                               const uint8_t* state, const int32_t* dest, int na, float lx,
                               float ly, int n_dest, int32_t* bad2, hipStream_t s);

}  // namespace fps
