// Internal declarations of libfps: device-resident step state, per-scenario
// parameter blocks and launchers.  Not part of the public ABI (include/fps.h).
//
// Every kernel is scenario-indexed: the parameters of each scenario of an
// ensemble live in a device array of Scn records, flood tiles and agents of
// all scenarios are flattened into one launch, and each scenario keeps its own
// time, time step, ping-pong parity and active flag in its DevState.  A
// standalone simulation is an ensemble of one.  Launch arguments are the same
// every step, so a step can be captured once in a HIP graph and replayed.
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
constexpr int kSlots = 16;             // partial sums of an agent's forces (the most lanes per agent)
constexpr int kScanThreads = 1024;
constexpr int kMaxHydro = 64;
constexpr int kMaskBits = 128;         // obstacle bitmask per cell (uint4)
constexpr int kInlinePlace = 8192;     // agent counts binned inside the one-block finalize
constexpr int kLdsBinWords = 30 * 1024;  // LDS words for bin starts + placement in the finalize
constexpr int kLdsScanBins = 16 * kScanThreads;   // bins the LDS binning scans in one pass
constexpr int kWetSlots = 64;          // wetness flags of a flood update, one per group of blocks
constexpr int kWetStride = 32;         // ints between flags (one 128-byte line each)
constexpr int kMaxDoor = 16;           // entrance doors of the pre-flood flow
constexpr int kCodeDest = 16;          // destinations whose direction codes are kept (more: read the distances)
constexpr int kChunkBins = 4096;       // bins per block of the multi-block bin scan (256 threads x 16)
constexpr int kMbScanBins = 32768;     // scenarios with more bins scan them with many blocks

// Scalars that live in device memory so that n steps run without the host.
struct DevState {
    double t;              // time at the start of the next step
    double t_end;          // the scenario stops advancing at t >= t_end (<= 0: never)
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
    int32_t cur;           // which of the two flood buffers holds the state
    int32_t active;        // 0 once t >= t_end
    int32_t flood_steps;   // steps whose flood update ran (the rest were dry and skipped)
    // sandbag barrier (sec. 2.4)
    int32_t layers_done, active_cell, bags, done, drops, drops_total;
    int32_t settled;       // the state came out of a flood update (dry cells carry no discharge)
    int32_t frozen;        // the flood update is held: steps of dt_max move only the pedestrians
    // pre-flood door flow (sec. 3.2)
    int32_t doors_closed;  // some cell has been wet: no more entries
    int32_t n_outside;     // agents in state OUTSIDE (free slots)
    int64_t door_in, door_out;   // entries and leaves so far
};

struct FvParams {
    float* h[2];           // ping-pong flood state; [0] is the caller's buffer
    float* qx[2];
    float* qy[2];
    const float* z;
    const int32_t* np;
    DevState* st;
    float* h1;             // the first Runge-Kutta stage of the second-order variant
    float* qx1;
    float* qy1;
    double* partials;      // [ntiles][4]: mass sum, outflow volume, clipped depth, max speed
    int32_t* wet;          // [kWetSlots * kWetStride]: set by waves with a wet cell, cleared by the finalize
    int nx, ny, H, nsx, ntiles;
    int bc[4];
    int inflow_side, c0, c1, n_inflow;
    int np_cap;
    float dx, dy, inv_dx, inv_dy, g, half_g, eps, cfl, dt_max, n_base;
    double dxdy;
    // judge region: only waves whose cells meet a set block of jmask
    // ([ceil(ny/jb)][jbx] blocks of jb x jb cells) update; the time step is
    // then dt_max, not the CFL step
    const uint8_t* jmask;
    int jb, jbx, jby;
};

struct PedParams {
    float* x;
    float* y;
    float* vx;
    float* vy;
    const float* vbase;
    const uint8_t* role;
    uint8_t* state;
    uint8_t* cls;
    int32_t* dest;
    float* timer;
    int na;
    int32_t* np;
    const float* dist;
    const uint8_t* walk;
    int n_dest, n_exit;
    const int32_t* bin_start;   // bins of the positions at the start of the step
    const float2* xy;           // positions in bin order
    const int32_t* slot;        // each agent's place in that order
    const uint4* wmask;         // per cell: obstacle cells within r_cut (bit per offset)
    const uint8_t* codes;       // [n_dest][ny][nx]: heading (bits 0-3) and arrival (bit 4) per destination and cell
    int use_codes;              // codes valid (n_dest <= kCodeDest); else the step reads the distances
    int32_t* bin_count;         // histogram of the new positions
    int32_t* rank;
    int32_t* key;
    int nx, ny, bsx, bsy, nbx, nby, Rx, Ry;
    int use_wmask;              // masks valid: (2Rx+1)(2Ry+1) <= 128
    float dx, dy, eps, tau, a_over_m, inv_b, two_r, radius, r_cut, r_arrive;
    float v_class[5], hr_t[3], pick_s, drop_s;
    int storage_dest, barrier_dest;
    int need_rank;              // histogram + each agent's rank in its bin (the global binning needs them)
    // pre-flood door flow: door cells [0, kMaxDoor) then their destinations [kMaxDoor, 2 kMaxDoor)
    const int32_t* doors;
    int n_door, door_rate;
    uint64_t door_seed;
    // stability rule: bodies (NULL: body_h0 / body_m0 for everyone) and constants
    const float* body_h;
    const float* body_m;
    int stab;
    float stab_kd, stab_mu, stab_rw, stab_rb, stab_g, body_h0, body_m0;   // kd = rho_w c_drag / 2
    // wading rule: the speed cap sqrt(wade_k W' / (kd b h))
    int wade;
    float wade_k;
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
    float2* xy;
    int32_t* slot;
    int32_t* np;
    int32_t* csum;     // multi-block scan: per chunk of kChunkBins bins its count, then its offset; [nchunk]: active flag
    int na, nbins, nx, ny, bsx, bsy, nbx;
    int nchunk;        // chunks of the multi-block scan (0: the bins are scanned by one block)
    float dx, dy;
};

// One scenario: everything its kernels need.
struct Scn {
    FvParams fv;
    PedParams ped;
    BinParams bins;
    BarrierParams bar;
    int na;
    int inline_place;      // agents placed in their bins inside the finalize block
    int lds_bins;          // ... with the bin starts and the placement in LDS (small grids)
};

// Flattened launch description of an ensemble (device arrays).
struct Batch {
    const Scn* scn;
    const int* tile_off;   // [S+1] prefix of flood tiles (waves) per scenario
    const int* agent_off;  // [S+1] prefix of agents per scenario
    const int* chunk_off;  // [S+1] prefix of multi-block bin-scan chunks per scenario
    int S;
    int total_tiles, total_agents, total_chunks;
    int fv_blocks;         // launched flood blocks: a multiple of 8 covering total_tiles
    int fin_lds_bytes;     // dynamic LDS of the finalize launch (LDS binning)
    int s_only;            // >= 0: restrict the flood launch to one scenario (tuning)
    Scn one;               // S == 1: the scenario itself, read from the kernel arguments
    int hll;               // face flux: HLL (1) or HLLC (0), the same for every scenario
    int order2;            // the second-order (MUSCL, two-stage) variant for every scenario
};

// launchers (stream-ordered, no synchronisation)
int fv_blocks_for_tiles(int64_t tiles);
int fv_tiles(int nx, int ny, int H);
int fv_tiles2(int nx, int ny, int H);    // tiles of the second-order march (narrower strips)
int fv_strip(bool order2);               // output columns of one wave of the march
int fv_rows_per_wave(int nx, int ny);
hipError_t launch_fv(const Batch& b, hipStream_t s);
hipError_t launch_fv_scan(const Batch& b, int scenario, int ntiles, hipStream_t s);
hipError_t launch_finalize(const Batch& b, int mode, int s_first, int count, hipStream_t s);
hipError_t prepare_finalize(int lds_bytes);   // host, outside any capture: allow that much dynamic LDS
hipError_t launch_sync_back(const Batch& b, int64_t max_cells, hipStream_t s);
hipError_t launch_ped(const Batch& b, hipStream_t s);
// n_in = 1, 4 or 5 arrays in and n_out = 1 or 3 out (see fps_stream_probe)
hipError_t launch_stream_probe(float* buf, int64_t n, int64_t stride, int n_in, int n_out, int blocks,
                               hipStream_t s);
int ped_lanes(int64_t total_agents);     // lanes per agent of the pedestrian step
hipError_t launch_doors(const Batch& b, hipStream_t s);    // entries of the pre-flood flow, one block per scenario
hipError_t launch_count_state(const uint8_t* state, int na, int value, int32_t* out, hipStream_t s);
hipError_t launch_bin_place_all(const Batch& b, hipStream_t s);
hipError_t launch_perm_from_slots(const int32_t* key, const int32_t* slot, int na, int32_t* perm, hipStream_t s);
hipError_t launch_bin_chunk_sum(const Batch& b, hipStream_t s);    // multi-block scan: chunk counts
hipError_t launch_bin_chunk_scan(const Batch& b, hipStream_t s);   // multi-block scan: bin starts
hipError_t launch_bin_sort_all(const Batch& b, hipStream_t s);
hipError_t launch_bin_keys(const BinParams& b, hipStream_t s);   // keys + ranks from positions
hipError_t launch_bin_scan(const BinParams& b, hipStream_t s);
hipError_t launch_bin_place(const BinParams& b, hipStream_t s);
hipError_t launch_bin_sort(const BinParams& b, hipStream_t s);
hipError_t launch_count(const BinParams& b, hipStream_t s);      // per-cell evacuee counts
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t launch_hazard(const float* h, const float* qx, const float* qy, float* hr, int64_t n,
                         float eps, hipStream_t s);
hipError_t launch_agent_stats(const uint8_t* state, const uint8_t* cls, int na, int32_t* out14,
                              hipStream_t s);
hipError_t launch_wall_mask(const uint8_t* walk, uint4* mask, int nx, int ny, int Rx, int Ry,
                            hipStream_t s);
hipError_t launch_nav_codes(const float* dist, const uint8_t* walk, int n_dest, int nx, int ny, float r_arrive,
                            int Rx, int Ry, uint8_t* codes, hipStream_t s);
// bad2[0]: agents outside the domain; bad2[1]: invalid role / state / destination
hipError_t launch_check_agents(const float* x, const float* y, const uint8_t* role,
                               const uint8_t* state, const int32_t* dest, int na, float lx,
                               float ly, int n_dest, int32_t* bad2, hipStream_t s);

}  // namespace fps
