// C-ABI of libfps (declared in include/fps.h): handles, workspace carving,
// argument validation, parameter upload and the stream-ordered step loop.
//
// An Engine runs S scenarios with one set of launches per step (see the
// kernels' Batch).  fps_create makes an engine of one scenario and returns its
// member handle; fps_ens_create makes an engine of S members.  The step's
// launches take the same arguments every step (parities, time steps and
// activity live on the device), so chunks of steps are captured once in a HIP
// graph and replayed on an internal stream ordered after the caller's stream.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "fps_internal.h"

using namespace fps;

struct Engine;

struct fps_sim {
    Engine* eng;
    int idx;
    fps_grid_desc G;
    fps_ped_params P;
    int32_t max_agents;
    char err[512];
    // workspace carve
    DevState* st;
    double* partials;
    int32_t* wet;
    float *h2, *qx2, *qy2;
    float *h1, *qx1, *qy1;     // first stage of the second-order variant
    int32_t* np;
    int32_t *bin_count, *bin_start, *rank, *key, *perm_u;
    float2* xy;
    int32_t* slot;
    uint4* wmask;
    uint8_t* codes;            // heading / arrival codes of up to kCodeDest destinations
    int32_t* line;
    int32_t* stats;
    int32_t* doors;            // door cells, then their destinations (kMaxDoor each)
    int32_t* csum;             // chunk counts / offsets of the multi-block bin scan
    int32_t line_cap;
    int H;
    int nbins, bsx, bsy, nbx, nby, Rx, Ry;
    int n_inflow;
    bool use_wmask;
    bool use_codes;
    double t_end;
    double hyd_t[kMaxHydro], hyd_q[kMaxHydro];   // host copy of the hydrograph
    int hyd_n;
    const uint8_t* jmask;  // judge region (NULL: whole grid, CFL time step)
    int jb;
    // bound caller memory
    float *h, *qx, *qy, *z;
    bool fields_bound;
    int32_t na;
    float *x, *y, *vx, *vy, *vbase, *timer;
    uint8_t *role, *state, *cls;
    int32_t* dest;
    const float* dist;
    const uint8_t* walk;
    int32_t n_dest, n_exit;
    bool nav_bound;
    int32_t nline, storage_dest, barrier_dest, n_layers, bags_per;
    float t_bag, t_last;
    const float *body_h, *body_m;   // bodies of the stability rule (NULL: the default body)
    int32_t n_door, door_rate;
    uint64_t door_seed;
    bool numeric_fault;
};

struct Engine {
    int S = 0;
    bool standalone = false;
    hipStream_t stream = nullptr;   // the caller's stream
    hipStream_t cap = nullptr;      // internal stream for graph capture and replay
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<fps_sim*> m;
    Scn* scn_d = nullptr;
    int* tile_off_d = nullptr;
    int* agent_off_d = nullptr;
    int* chunk_off_d = nullptr;
    std::vector<Scn> scn_h;
    std::vector<int> tile_off_h, agent_off_h, chunk_off_h;
    int total_tiles = 0, total_agents = 0, total_chunks = 0, fv_blocks = 0;
    int64_t max_cells = 0;
    int fin_lds_bytes = 0;
    bool any_big = false;
    bool any_doors = false;          // some scenario runs the pre-flood door flow
    bool dirty = true;
    int graph_chunk = 16;
    int hll = 0;                     // face flux of every scenario: HLL instead of HLLC
    int order2 = 0;                  // second-order (MUSCL, two-stage) variant for every scenario
    hipGraphExec_t exec = nullptr;
    int exec_steps = 0;
    char err[512] = "";
};

struct fps_ens : Engine {};

namespace {

char g_err[512] = "";

int failv(char* buf, int code, const char* fmt, va_list ap)
{
    vsnprintf(buf, 512, fmt, ap);
    return code;
}

int fail(fps_sim* s, int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    int r = failv(s ? s->err : g_err, code, fmt, ap);
    va_end(ap);
    return r;
}

int efail(Engine* e, int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    int r = failv(e ? e->err : g_err, code, fmt, ap);
    va_end(ap);
    return r;
}

#define HIPCHK(sim, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(sim, FPS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define HIPCHK_E(eng, expr)                                                                 \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return efail(eng, FPS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool valid_desc(const fps_grid_desc* d, char* why)
{
    if (!d) return (snprintf(why, 256, "desc is NULL"), false);
    if (d->nx < 1 || d->ny < 1) return (snprintf(why, 256, "nx, ny must be >= 1"), false);
    if ((int64_t)d->nx * d->ny > (int64_t)1 << 30) return (snprintf(why, 256, "grid too large"), false);
    if (!(d->dx > 0) || !(d->dy > 0) || !std::isfinite(d->dx) || !std::isfinite(d->dy))
        return (snprintf(why, 256, "dx, dy must be finite and > 0"), false);
    if (!(d->g > 0) || !(d->cfl > 0 && d->cfl <= 1.0) || !(d->h_dry > 0) || !(d->dt_max > 0))
        return (snprintf(why, 256, "need g > 0, 0 < cfl <= 1, h_dry > 0, dt_max > 0"), false);
    for (int k = 0; k < 4; ++k)
        if (d->bc[k] != FPS_BC_WALL && d->bc[k] != FPS_BC_TRANSMISSIVE)
            return (snprintf(why, 256, "bc[%d] invalid", k), false);
    if (d->inflow_side < -1 || d->inflow_side > 3) return (snprintf(why, 256, "inflow_side invalid"), false);
    if (d->inflow_side >= 0) {
        int len = d->inflow_side <= 1 ? d->ny : d->nx;
        if (d->inflow_c0 < 0 || d->inflow_c1 > len || d->inflow_c0 >= d->inflow_c1)
            return (snprintf(why, 256, "inflow cell range invalid"), false);
    }
    if (!(d->n_base >= 0) || d->np_cap < 0) return (snprintf(why, 256, "n_base, np_cap must be >= 0"), false);
    return true;
}

// Per-scenario part of the workspace (offsets from the member's base).
struct Layout {
    size_t st, partials, wet, h2, qx2, qy2, h1, qx1, qy1, np, bin_count, bin_start, rank, key, perm_u, xy, slot,
        wmask, codes, line, stats, doors, csum, total;
    int64_t nbins_max;
    int32_t line_cap;
};

Layout member_layout(const fps_grid_desc* d, int32_t max_agents)
{
    Layout L{};
    const int64_t nc = (int64_t)d->nx * d->ny;
    L.nbins_max = nc;   // bins are whole cells, at least one cell wide
    L.line_cap = 2 * (d->nx + d->ny);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t na = (size_t)std::max(max_agents, 0);
    L.st = take(sizeof(DevState));
    L.partials = take(sizeof(double) * 4 * (size_t)std::max(fv_tiles(d->nx, d->ny, 1), fv_tiles2(d->nx, d->ny, 1)));
    L.wet = take(sizeof(int32_t) * kWetSlots * kWetStride);
    L.h2 = take(sizeof(float) * nc);
    L.qx2 = take(sizeof(float) * nc);
    L.qy2 = take(sizeof(float) * nc);
    L.h1 = take(sizeof(float) * nc);
    L.qx1 = take(sizeof(float) * nc);
    L.qy1 = take(sizeof(float) * nc);
    L.np = take(sizeof(int32_t) * nc);
    L.bin_count = take(max_agents > 0 ? sizeof(int32_t) * L.nbins_max : 0);
    L.bin_start = take(max_agents > 0 ? sizeof(int32_t) * (L.nbins_max + 1) : 0);
    L.rank = take(sizeof(int32_t) * na);
    L.key = take(sizeof(int32_t) * na);
    L.perm_u = take(sizeof(int32_t) * na);
    L.xy = take(sizeof(float2) * na);
    L.slot = take(sizeof(int32_t) * na);
    L.wmask = take(max_agents > 0 ? sizeof(uint4) * nc : 0);
    L.codes = take(max_agents > 0 ? (size_t)kCodeDest * nc : 0);
    L.line = take(sizeof(int32_t) * L.line_cap);
    L.stats = take(sizeof(int32_t) * 16);
    L.doors = take(sizeof(int32_t) * 2 * kMaxDoor);
    L.csum = take(max_agents > 0 ? sizeof(int32_t) * (size_t)(L.nbins_max / kChunkBins + 2) : 0);
    L.total = o;
    return L;
}

size_t engine_header_bytes(int S)
{
    return align256(sizeof(Scn) * S) + align256(sizeof(int) * (S + 1)) * 3;
}

template <class T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

// carve one member from its part of the workspace; nothing touches the device
fps_sim* new_member(Engine* e, int idx, const fps_grid_desc* d, const fps_ped_params& P,
                    int32_t max_agents, void* base)
{
    fps_sim* s = new (std::nothrow) fps_sim();
    if (!s) return nullptr;
    Layout L = member_layout(d, max_agents);
    s->eng = e;
    s->idx = idx;
    s->G = *d;
    s->P = P;
    s->max_agents = max_agents;
    s->st = at<DevState>(base, L.st);
    s->partials = at<double>(base, L.partials);
    s->wet = at<int32_t>(base, L.wet);
    s->h2 = at<float>(base, L.h2);
    s->qx2 = at<float>(base, L.qx2);
    s->qy2 = at<float>(base, L.qy2);
    s->h1 = at<float>(base, L.h1);
    s->qx1 = at<float>(base, L.qx1);
    s->qy1 = at<float>(base, L.qy1);
    s->np = at<int32_t>(base, L.np);
    s->bin_count = at<int32_t>(base, L.bin_count);
    s->bin_start = at<int32_t>(base, L.bin_start);
    s->rank = at<int32_t>(base, L.rank);
    s->key = at<int32_t>(base, L.key);
    s->perm_u = at<int32_t>(base, L.perm_u);
    s->xy = at<float2>(base, L.xy);
    s->slot = at<int32_t>(base, L.slot);
    s->wmask = at<uint4>(base, L.wmask);
    s->codes = at<uint8_t>(base, L.codes);
    s->line = at<int32_t>(base, L.line);
    s->stats = at<int32_t>(base, L.stats);
    s->doors = at<int32_t>(base, L.doors);
    s->csum = at<int32_t>(base, L.csum);
    s->line_cap = L.line_cap;
    s->H = fv_rows_per_wave(d->nx, d->ny);
    s->bsx = std::max(1, (int)std::ceil(P.r_cut / d->dx - 1e-9));
    s->bsy = std::max(1, (int)std::ceil(P.r_cut / d->dy - 1e-9));
    s->nbx = (d->nx + s->bsx - 1) / s->bsx;
    s->nby = (d->ny + s->bsy - 1) / s->bsy;
    s->nbins = s->nbx * s->nby;
    s->Rx = s->bsx;
    s->Ry = s->bsy;
    s->n_inflow = d->inflow_side >= 0 ? d->inflow_c1 - d->inflow_c0 : 0;
    s->storage_dest = s->barrier_dest = -1;
    s->t_end = 0.0;
    s->jmask = nullptr;
    s->jb = 0;
    s->hyd_n = 0;
    return s;
}

// zero the member's device state and scratch counters (at creation)
int init_member_device(fps_sim* s)
{
    DevState h0{};
    h0.dt = (float)s->G.dt_max;
    h0.dt_prev = (float)s->G.dt_max;
    h0.active = 1;
    hipStream_t st = s->eng->stream;
    HIPCHK(s, hipMemcpyAsync(s->st, &h0, sizeof(h0), hipMemcpyHostToDevice, st));
    HIPCHK(s, launch_fill_i32(s->np, 0, (int64_t)s->G.nx * s->G.ny, st));
    HIPCHK(s, launch_fill_i32(s->wet, 0, (int64_t)kWetSlots * kWetStride, st));
    // the second flood buffer starts as a dry state (a judge region updates
    // only part of it and reads the rest)
    for (float* f : {s->h2, s->qx2, s->qy2})
        HIPCHK(s, launch_fill_i32(reinterpret_cast<int32_t*>(f), 0, (int64_t)s->G.nx * s->G.ny, st));
    if (s->max_agents > 0)
        HIPCHK(s, launch_fill_i32(s->bin_count, 0, (int64_t)s->G.nx * s->G.ny, st));
    HIPCHK(s, hipStreamSynchronize(st));
    return FPS_OK;
}

void fill_scn(const fps_sim* s, Scn& c)
{
    c = Scn{};
    FvParams& p = c.fv;
    p.h[0] = s->h; p.h[1] = s->h2;
    p.qx[0] = s->qx; p.qx[1] = s->qx2;
    p.qy[0] = s->qy; p.qy[1] = s->qy2;
    p.h1 = s->h1; p.qx1 = s->qx1; p.qy1 = s->qy1;
    p.z = s->z;
    p.np = s->np;
    p.st = s->st;
    p.partials = s->partials;
    p.wet = s->wet;
    p.nx = s->G.nx; p.ny = s->G.ny; p.H = s->H;
    const bool order2 = s->eng->order2;
    p.nsx = (s->G.nx + fv_strip(order2) - 1) / fv_strip(order2);
    p.ntiles = order2 ? fv_tiles2(s->G.nx, s->G.ny, s->H) : fv_tiles(s->G.nx, s->G.ny, s->H);
    for (int k = 0; k < 4; ++k) p.bc[k] = s->G.bc[k];
    p.inflow_side = s->G.inflow_side;
    p.c0 = s->G.inflow_c0;
    p.c1 = s->G.inflow_c1;
    p.n_inflow = s->n_inflow;
    p.np_cap = s->G.np_cap;
    p.dx = (float)s->G.dx; p.dy = (float)s->G.dy;
    p.inv_dx = (float)(1.0 / s->G.dx); p.inv_dy = (float)(1.0 / s->G.dy);
    p.g = (float)s->G.g; p.half_g = (float)(0.5 * s->G.g);
    p.eps = (float)s->G.h_dry; p.cfl = (float)s->G.cfl; p.dt_max = (float)s->G.dt_max;
    p.n_base = (float)s->G.n_base;
    p.dxdy = s->G.dx * s->G.dy;
    p.jmask = s->jmask;
    p.jb = s->jb > 0 ? s->jb : 1;
    p.jbx = (s->G.nx + p.jb - 1) / p.jb;
    p.jby = (s->G.ny + p.jb - 1) / p.jb;

    PedParams& q = c.ped;
    q.x = s->x; q.y = s->y; q.vx = s->vx; q.vy = s->vy; q.vbase = s->vbase;
    q.role = s->role; q.state = s->state; q.cls = s->cls; q.dest = s->dest; q.timer = s->timer;
    q.na = s->na;
    q.np = s->np;
    q.dist = s->dist; q.walk = s->walk; q.n_dest = s->n_dest; q.n_exit = s->n_exit;
    q.bin_start = s->bin_start; q.xy = s->xy; q.slot = s->slot; q.wmask = s->wmask;
    q.bin_count = s->bin_count; q.rank = s->rank; q.key = s->key;
    q.nx = s->G.nx; q.ny = s->G.ny;
    q.bsx = s->bsx; q.bsy = s->bsy; q.nbx = s->nbx; q.nby = s->nby; q.Rx = s->Rx; q.Ry = s->Ry;
    q.use_wmask = s->use_wmask;
    q.codes = s->codes; q.use_codes = s->use_codes;
    q.dx = (float)s->G.dx; q.dy = (float)s->G.dy; q.eps = (float)s->G.h_dry;
    q.tau = (float)s->P.tau; q.a_over_m = (float)s->P.a_over_m; q.inv_b = (float)(1.0 / s->P.b_range);
    q.two_r = (float)(2.0 * s->P.radius); q.radius = (float)s->P.radius;
    q.r_cut = (float)s->P.r_cut; q.r_arrive = (float)s->P.r_arrive;
    for (int k = 0; k < 5; ++k) q.v_class[k] = (float)s->P.v_class[k];
    for (int k = 0; k < 3; ++k) q.hr_t[k] = (float)s->P.hr_t[k];
    q.pick_s = (float)s->P.pick_s; q.drop_s = (float)s->P.drop_s;
    q.storage_dest = s->storage_dest; q.barrier_dest = s->barrier_dest;
    q.doors = s->doors; q.n_door = s->na > 0 ? s->n_door : 0; q.door_rate = s->door_rate;
    q.stab = s->P.stability;
    q.body_h = s->body_h; q.body_m = s->body_m;
    q.stab_kd = (float)(0.5 * s->P.rho_w * s->P.c_drag);
    q.stab_mu = (float)s->P.mu_f; q.stab_rw = (float)s->P.rho_w; q.stab_rb = (float)s->P.rho_body;
    q.stab_g = (float)s->G.g; q.body_h0 = (float)s->P.body_h0; q.body_m0 = (float)s->P.body_m0;
    q.wade = s->P.wading; q.wade_k = (float)s->P.wade_k;
    q.door_seed = s->door_seed;

    BinParams& b = c.bins;
    b.x = s->x; b.y = s->y; b.state = s->state; b.role = s->role;
    b.bin_count = s->bin_count; b.bin_start = s->bin_start; b.rank = s->rank; b.key = s->key;
    b.perm_u = s->perm_u; b.xy = s->xy; b.slot = s->slot; b.np = s->np; b.csum = s->csum;
    b.na = s->na; b.nbins = s->nbins; b.nx = s->G.nx; b.ny = s->G.ny;
    b.bsx = s->bsx; b.bsy = s->bsy; b.nbx = s->nbx;
    b.dx = (float)s->G.dx; b.dy = (float)s->G.dy;

    BarrierParams& r = c.bar;
    r.z = s->z; r.line = s->line; r.nline = s->nline; r.n_layers = s->n_layers;
    r.bags_per = s->bags_per; r.t_bag = s->t_bag; r.t_last = s->t_last;

    c.na = s->na;
    // many bins: scanned by many blocks, and the agents placed by the placement kernels
    const bool mb = s->na > 0 && s->nbins > kMbScanBins;
    b.nchunk = mb ? (s->nbins + kChunkBins - 1) / kChunkBins : 0;
    c.inline_place = s->na <= kInlinePlace && !mb;
    c.lds_bins = c.inline_place && s->na > 0 && s->nbins <= kLdsScanBins &&
                 (int64_t)s->nbins + 1 + s->na <= kLdsBinWords;
    c.ped.need_rank = !c.lds_bins;       // the LDS binning counts the keys itself
}

void drop_graph(Engine* e)
{
    if (e->exec) (void)hipGraphExecDestroy(e->exec);
    e->exec = nullptr;
    e->exec_steps = 0;
}

// rebuild the device parameter records and launch geometry after any change
int upload(Engine* e)
{
    if (!e->dirty) return FPS_OK;
    e->tile_off_h.assign(e->S + 1, 0);
    e->agent_off_h.assign(e->S + 1, 0);
    e->chunk_off_h.assign(e->S + 1, 0);
    e->scn_h.resize(e->S);
    e->max_cells = 0;
    e->any_big = false;
    e->any_doors = false;
    e->fin_lds_bytes = 0;
    for (int k = 0; k < e->S; ++k) {
        fps_sim* s = e->m[k];
        fill_scn(s, e->scn_h[k]);
        e->tile_off_h[k + 1] = e->tile_off_h[k] + e->scn_h[k].fv.ntiles;
        e->agent_off_h[k + 1] = e->agent_off_h[k] + (s->na + kPedBlock - 1) / kPedBlock * kPedBlock;
        e->max_cells = std::max(e->max_cells, (int64_t)s->G.nx * s->G.ny);
        e->chunk_off_h[k + 1] = e->chunk_off_h[k] + e->scn_h[k].bins.nchunk;
        e->any_big = e->any_big || (s->na > 0 && !e->scn_h[k].inline_place);
        e->any_doors = e->any_doors || e->scn_h[k].ped.n_door > 0;
        if (e->scn_h[k].lds_bins)
            e->fin_lds_bytes = std::max(e->fin_lds_bytes, (int)(sizeof(int) * (s->nbins + 1 + s->na)));
    }
    HIPCHK_E(e, prepare_finalize(e->fin_lds_bytes));
    e->total_tiles = e->tile_off_h[e->S];
    e->total_agents = e->agent_off_h[e->S];
    e->total_chunks = e->chunk_off_h[e->S];
    e->fv_blocks = fv_blocks_for_tiles(e->total_tiles);
    HIPCHK_E(e, hipMemcpyAsync(e->scn_d, e->scn_h.data(), sizeof(Scn) * e->S, hipMemcpyHostToDevice, e->stream));
    HIPCHK_E(e, hipMemcpyAsync(e->tile_off_d, e->tile_off_h.data(), sizeof(int) * (e->S + 1),
                               hipMemcpyHostToDevice, e->stream));
    HIPCHK_E(e, hipMemcpyAsync(e->agent_off_d, e->agent_off_h.data(), sizeof(int) * (e->S + 1),
                               hipMemcpyHostToDevice, e->stream));
    HIPCHK_E(e, hipMemcpyAsync(e->chunk_off_d, e->chunk_off_h.data(), sizeof(int) * (e->S + 1),
                               hipMemcpyHostToDevice, e->stream));
    HIPCHK_E(e, hipStreamSynchronize(e->stream));
    e->dirty = false;
    drop_graph(e);
    return FPS_OK;
}

Batch batch_of(const Engine* e, int s_only = -1)
{
    Batch b{};
    b.scn = e->scn_d;
    b.tile_off = e->tile_off_d;
    b.agent_off = e->agent_off_d;
    b.chunk_off = e->chunk_off_d;
    b.total_chunks = e->total_chunks;
    b.S = e->S;
    b.total_tiles = e->total_tiles;
    b.total_agents = e->total_agents;
    b.fv_blocks = e->fv_blocks;
    b.fin_lds_bytes = e->fin_lds_bytes;
    b.s_only = s_only;
    b.hll = e->hll;
    b.order2 = e->order2;
    if (s_only >= 0) b.fv_blocks = fv_blocks_for_tiles(e->scn_h[s_only].fv.ntiles);
    if (e->S == 1) b.one = e->scn_h[0];
    return b;
}

void mark_dirty(fps_sim* s) { s->eng->dirty = true; }

// recompute dt (and the inflow of the next step) of one member from its state
int prime(fps_sim* s)
{
    if (!s->fields_bound) return FPS_OK;
    Engine* e = s->eng;
    int rc = upload(e);
    if (rc != FPS_OK) return fail(s, rc, "%s", e->err);
    Batch b = batch_of(e);
    HIPCHK(s, launch_fv_scan(b, s->idx, e->scn_h[s->idx].fv.ntiles, e->stream));
    HIPCHK(s, launch_finalize(b, 1, s->idx, 1, e->stream));
    return FPS_OK;
}

BinParams bin_params(const fps_sim* s)
{
    Scn c;
    fill_scn(s, c);
    return c.bins;
}

int rebuild_bins(fps_sim* s)
{
    if (s->na <= 0) return FPS_OK;
    hipStream_t st = s->eng->stream;
    BinParams b = bin_params(s);
    HIPCHK(s, launch_fill_i32(s->bin_count, 0, s->nbins, st));
    HIPCHK(s, launch_bin_keys(b, st));
    HIPCHK(s, launch_bin_scan(b, st));
    HIPCHK(s, launch_bin_place(b, st));
    HIPCHK(s, launch_bin_sort(b, st));
    HIPCHK(s, launch_fill_i32(s->np, 0, (int64_t)s->G.nx * s->G.ny, st));
    HIPCHK(s, launch_count(b, st));
    return FPS_OK;
}

struct KernelEvents {
    hipEvent_t ev[5][2];
    double ms[5];
    int n[5];
};

// the launches of one step of every scenario
int step_launches(Engine* e, hipStream_t st, KernelEvents* K)
{
    Batch b = batch_of(e);
    auto rec = [&](int k, int w) {
        if (K) (void)hipEventRecord(K->ev[k][w], st);
    };
    rec(0, 0);
    HIPCHK_E(e, launch_fv(b, st));
    rec(0, 1);
    if (e->total_agents > 0) {
        rec(1, 0);
        HIPCHK_E(e, launch_ped(b, st));
        if (e->any_doors) HIPCHK_E(e, launch_doors(b, st));
        rec(1, 1);
    }
    rec(2, 0);
    if (e->total_chunks > 0) HIPCHK_E(e, launch_bin_chunk_sum(b, st));
    HIPCHK_E(e, launch_finalize(b, 0, 0, e->S, st));
    if (e->total_chunks > 0) HIPCHK_E(e, launch_bin_chunk_scan(b, st));
    rec(2, 1);
    if (e->any_big) {
        rec(3, 0);
        HIPCHK_E(e, launch_bin_place_all(b, st));
        rec(3, 1);
        rec(4, 0);
        HIPCHK_E(e, launch_bin_sort_all(b, st));
        rec(4, 1);
    }
    if (K) {
        const bool used[5] = {true, e->total_agents > 0, true, e->any_big, e->any_big};
        for (int k = 0; k < 5; ++k) {
            if (!used[k]) continue;
            float ms = 0.0f;
            (void)hipEventSynchronize(K->ev[k][1]);
            (void)hipEventElapsedTime(&ms, K->ev[k][0], K->ev[k][1]);
            K->ms[k] += ms;
            K->n[k] += 1;
        }
    }
    return FPS_OK;
}

int capture(Engine* e, int steps)
{
    drop_graph(e);
    if (!e->cap) {
        HIPCHK_E(e, hipStreamCreateWithFlags(&e->cap, hipStreamNonBlocking));
        HIPCHK_E(e, hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming));
        HIPCHK_E(e, hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming));
    }
    hipGraph_t g = nullptr;
    HIPCHK_E(e, hipStreamBeginCapture(e->cap, hipStreamCaptureModeThreadLocal));
    int rc = FPS_OK;
    for (int k = 0; k < steps && rc == FPS_OK; ++k) rc = step_launches(e, e->cap, nullptr);
    hipError_t ce = hipStreamEndCapture(e->cap, &g);
    if (rc != FPS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (ce != hipSuccess) return efail(e, FPS_E_DEVICE, "graph capture failed: %s", hipGetErrorString(ce));
    hipError_t ie = hipGraphInstantiate(&e->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
        e->exec = nullptr;
        return efail(e, FPS_E_DEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
    }
    e->exec_steps = steps;
    return FPS_OK;
}

int engine_ready(Engine* e)
{
    for (fps_sim* s : e->m) {
        if (!s->fields_bound) return efail(e, FPS_E_STATE, "scenario %d: fields not bound", s->idx);
        if (s->na > 0 && !s->nav_bound)
            return efail(e, FPS_E_STATE, "scenario %d: agents need a navigation map", s->idx);
        if (s->numeric_fault)
            return efail(e, FPS_E_STATE, "scenario %d: numeric fault latched; rebind fields", s->idx);
    }
    return FPS_OK;
}

int run_steps(Engine* e, int32_t n, KernelEvents* K)
{
    if (n < 0) return efail(e, FPS_E_INVALID, "n_steps < 0");
    int rc = engine_ready(e);
    if (rc != FPS_OK) return rc;
    rc = upload(e);
    if (rc != FPS_OK) return rc;
    int done = 0;
    if (!K && e->graph_chunk > 0 && n >= e->graph_chunk) {
        if (!e->exec || e->exec_steps != e->graph_chunk) {
            rc = capture(e, e->graph_chunk);
            if (rc != FPS_OK) return rc;
        }
        HIPCHK_E(e, hipEventRecord(e->ev_in, e->stream));
        HIPCHK_E(e, hipStreamWaitEvent(e->cap, e->ev_in, 0));
        for (; done + e->exec_steps <= n; done += e->exec_steps) HIPCHK_E(e, hipGraphLaunch(e->exec, e->cap));
        HIPCHK_E(e, hipEventRecord(e->ev_out, e->cap));
        HIPCHK_E(e, hipStreamWaitEvent(e->stream, e->ev_out, 0));
    }
    for (; done < n; ++done) {
        rc = step_launches(e, e->stream, K);
        if (rc != FPS_OK) return rc;
    }
    if (n > 0) HIPCHK_E(e, launch_sync_back(batch_of(e), e->max_cells, e->stream));
    return FPS_OK;
}

int profiled(Engine* e, int32_t n, double* ms_out)
{
    KernelEvents K{};
    for (int k = 0; k < 5; ++k)
        for (int w = 0; w < 2; ++w) HIPCHK_E(e, hipEventCreate(&K.ev[k][w]));
    int rc = run_steps(e, n, &K);
    (void)hipStreamSynchronize(e->stream);
    for (int k = 0; k < 5; ++k) {
        ms_out[k] = K.n[k] ? K.ms[k] / K.n[k] : 0.0;
        for (int w = 0; w < 2; ++w) (void)hipEventDestroy(K.ev[k][w]);
    }
    return rc;
}

// mean device ms of one flood-update launch of member s with H rows per wave,
// measured on its bound state (outputs go to the scratch buffer; nothing is
// committed: the caller re-primes the member afterwards)
int time_rows(fps_sim* s, int H, int reps, float* ms_out)
{
    Engine* e = s->eng;
    s->H = H;
    mark_dirty(s);
    int rc = upload(e);
    if (rc != FPS_OK) return fail(s, rc, "%s", e->err);
    Batch b = batch_of(e, s->idx);
    hipEvent_t e0, e1;
    HIPCHK(s, hipEventCreate(&e0));
    HIPCHK(s, hipEventCreate(&e1));
    for (int r = 0; r < 2; ++r) HIPCHK(s, launch_fv(b, e->stream));
    HIPCHK(s, hipEventRecord(e0, e->stream));
    for (int r = 0; r < reps; ++r) HIPCHK(s, launch_fv(b, e->stream));
    HIPCHK(s, hipEventRecord(e1, e->stream));
    HIPCHK(s, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK(s, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / reps;
    return FPS_OK;
}

int current_arch(char* arch, size_t n)
{
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return -1;
    snprintf(arch, n, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
        if (*c == ':' || *c == ' ') *c = '\0';
    return 0;
}

// one line of a tuning cache file (false at the end of the file)
bool read_line(FILE* f, std::string& line)
{
    line.clear();
    int c;
    while ((c = fgetc(f)) != EOF && c != '\n') line.push_back((char)c);
    return c != EOF || !line.empty();
}

bool valid_rows(int H) { return H >= 1 && H <= 64 && !(H & (H - 1)); }

// a grid size as one key: nx in the upper 32 bits, ny in the lower
int64_t size_key(int nx, int ny) { return (int64_t)nx << 32 | (uint32_t)ny; }

// Cache lines of one grid: "<arch> <nx> <ny> <rows> <ms>"; the last match wins.
bool cache_lookup(const char* path, const char* arch, int nx, int ny, int* H, double* ms)
{
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    std::string line;
    bool found = false;
    while (read_line(f, line)) {
        std::istringstream in(line);
        std::string a;
        int cx, cy, ch;
        double cm;
        if ((in >> a >> cx >> cy >> ch >> cm) && a == arch && cx == nx && cy == ny && valid_rows(ch)) {
            *H = ch;
            *ms = cm;
            found = true;
        }
    }
    fclose(f);
    return found;
}

// An ensemble's mix of grids: FNV-1a over the members' (nx, ny) in member order.
uint64_t mix_key(const Engine* e)
{
    uint64_t h = 1469598103934665603ull;
    for (const fps_sim* s : e->m)
        for (int v : {s->G.nx, s->G.ny})
            for (int b = 0; b < 4; ++b) {
                h ^= (uint64_t)((uint32_t)v >> (8 * b) & 0xffu);
                h *= 1099511628211ull;
            }
    return h;
}

// Cache lines of an ensemble: "<arch> ens <mix key, hex> <n sizes> (<nx> <ny> <rows>)... <ms>".
bool ens_cache_lookup(const char* path, const char* arch, uint64_t key, std::vector<int64_t>& sizes,
                      std::vector<int>& rows)
{
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    std::string line;
    bool found = false;
    while (read_line(f, line)) {
        std::istringstream in(line);
        std::string a, tag;
        uint64_t k = 0;
        int n = 0;
        if (!(in >> a >> tag >> std::hex >> k >> std::dec >> n) || a != arch || tag != "ens" || k != key || n < 1)
            continue;
        std::vector<int64_t> sz;
        std::vector<int> hs;
        bool ok = true;
        for (int i = 0; i < n && ok; ++i) {
            int cx, cy, ch;
            ok = (in >> cx >> cy >> ch) && valid_rows(ch);
            sz.push_back(size_key(cx, cy));
            hs.push_back(ch);
        }
        if (ok) {
            sizes = sz;
            rows = hs;
            found = true;
        }
    }
    fclose(f);
    return found;
}

int tune_member(fps_sim* s, const char* cache_path, int* rows_out, double* ms_out)
{
    if (!s->fields_bound) return fail(s, FPS_E_STATE, "fps_autotune: fields not bound");
    char arch[64] = "unknown";
    if (current_arch(arch, sizeof(arch)) != 0) return fail(s, FPS_E_DEVICE, "no HIP device");
    int best = -1;
    double best_ms = 0.0;
    if (!cache_lookup(cache_path, arch, s->G.nx, s->G.ny, &best, &best_ms)) {
        HIPCHK(s, hipStreamSynchronize(s->eng->stream));
        const int64_t cells = (int64_t)s->G.nx * s->G.ny;
        const int reps = cells > (1 << 24) ? 5 : 20;
        // the sweep is timed three times, interleaved, and each H keeps its
        // fastest pass: neighbouring H often differ by a few per cent, about
        // as much as one pass drifts with the clock
        constexpr int kPasses = 3;
        int Hs[8], nH = 0;
        double tmin[8];
        for (int H = 1; H <= 64; H <<= 1) {
            if (H > 1 && (H >> 1) >= s->G.ny) break;
            tmin[nH] = 0.0;
            Hs[nH++] = H;
        }
        for (int pass = 0; pass < kPasses; ++pass)
            for (int k = 0; k < nH; ++k) {
                float ms = 0.0f;
                int rc = time_rows(s, Hs[k], reps, &ms);
                if (rc != FPS_OK) return rc;
                if (pass == 0 || ms < tmin[k]) tmin[k] = ms;
            }
        best = -1;
        for (int k = 0; k < nH; ++k)
            if (best < 0 || tmin[k] < best_ms) {
                best = Hs[k];
                best_ms = tmin[k];
            }
        if (cache_path) {
            FILE* f = fopen(cache_path, "a");
            if (f) {
                fprintf(f, "%s %d %d %d %.6f\n", arch, s->G.nx, s->G.ny, best, best_ms);
                fclose(f);
            }
        }
    }
    s->H = best;
    mark_dirty(s);
    int rc = prime(s);   // timing launches wrote scratch partials and the wet flag
    if (rc != FPS_OK) return rc;
    if (rows_out) *rows_out = best;
    if (ms_out) *ms_out = best_ms;
    return FPS_OK;
}

void destroy_engine(Engine* e)
{
    if (!e) return;
    (void)hipStreamSynchronize(e->stream);
    drop_graph(e);
    if (e->cap) {
        (void)hipStreamSynchronize(e->cap);
        (void)hipStreamDestroy(e->cap);
    }
    if (e->ev_in) (void)hipEventDestroy(e->ev_in);
    if (e->ev_out) (void)hipEventDestroy(e->ev_out);
    for (fps_sim* s : e->m) delete s;
    e->m.clear();
}

int build_engine(Engine* e, int32_t S, const fps_grid_desc* descs, const fps_ped_params* peds,
                 const int32_t* max_agents, void* ws, size_t ws_bytes, void* stream)
{
    char why[256];
    if (S < 1) return efail(e, FPS_E_INVALID, "need at least one scenario");
    if (!descs) return efail(e, FPS_E_INVALID, "descs is NULL");
    for (int k = 0; k < S; ++k) {
        if (!valid_desc(&descs[k], why)) return efail(e, FPS_E_INVALID, "scenario %d: %s", k, why);
        if (max_agents && max_agents[k] < 0) return efail(e, FPS_E_INVALID, "scenario %d: max_agents < 0", k);
        if (peds) {
            const fps_ped_params& P = peds[k];
            if (!(P.tau > 0) || !(P.b_range > 0) || !(P.r_cut > 0) || !(P.radius >= 0) || !(P.r_arrive >= 0))
                return efail(e, FPS_E_INVALID, "scenario %d: pedestrian constants out of range", k);
            if ((P.stability != 0 && P.stability != 1) || !(P.c_drag >= 0) || !(P.mu_f > 0) || !(P.rho_w > 0) ||
                !(P.rho_body > 0) || !(P.body_h0 > 0) || !(P.body_m0 > 0))
                return efail(e, FPS_E_INVALID, "scenario %d: stability constants out of range", k);
            if ((P.wading != 0 && P.wading != 1) || !(P.wade_k > 0) || (P.wading && !(P.c_drag > 0)))
                return efail(e, FPS_E_INVALID, "scenario %d: wading constants out of range", k);
        }
    }
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
        return efail(e, FPS_E_INVALID, "workspace NULL or not 256-byte aligned");
    size_t need = engine_header_bytes(S);
    for (int k = 0; k < S; ++k) need += member_layout(&descs[k], max_agents ? max_agents[k] : 0).total;
    if (ws_bytes < need) return efail(e, FPS_E_CAPACITY, "workspace %zu bytes < %zu needed", ws_bytes, need);
    e->S = S;
    e->stream = static_cast<hipStream_t>(stream);
    size_t o = 0;
    e->scn_d = at<Scn>(ws, o);
    o += align256(sizeof(Scn) * S);
    e->tile_off_d = at<int>(ws, o);
    o += align256(sizeof(int) * (S + 1));
    e->agent_off_d = at<int>(ws, o);
    o += align256(sizeof(int) * (S + 1));
    e->chunk_off_d = at<int>(ws, o);
    o += align256(sizeof(int) * (S + 1));
    for (int k = 0; k < S; ++k) {
        fps_ped_params P;
        if (peds) P = peds[k];
        else fps_ped_params_default(&P);
        int32_t ma = max_agents ? max_agents[k] : 0;
        fps_sim* s = new_member(e, k, &descs[k], P, ma, at<char>(ws, o));
        if (!s) return efail(e, FPS_E_DEVICE, "out of host memory");
        e->m.push_back(s);
        o += member_layout(&descs[k], ma).total;
        int rc = init_member_device(s);
        if (rc != FPS_OK) return efail(e, rc, "%s", s->err);
    }
    return FPS_OK;
}

int write_state_i32(fps_sim* s, int32_t* field, int32_t v)
{
    HIPCHK(s, hipMemcpyAsync(field, &v, sizeof(v), hipMemcpyHostToDevice, s->eng->stream));
    HIPCHK(s, hipStreamSynchronize(s->eng->stream));
    return FPS_OK;
}

// the free slots of the door flow, counted from the bound agents' states
int recount_outside(fps_sim* s)
{
    hipStream_t st = s->eng->stream;
    HIPCHK(s, launch_fill_i32(&s->st->n_outside, 0, 1, st));
    if (s->na > 0) HIPCHK(s, launch_count_state(s->state, s->na, FPS_ST_OUTSIDE, &s->st->n_outside, st));
    HIPCHK(s, hipStreamSynchronize(st));
    return FPS_OK;
}

// reps back-to-back launches of the whole ensemble's flood update on the
// current state (outputs to scratch; the state is not advanced)
int time_ensemble_flood(Engine* e, int reps, float* ms_out)
{
    int rc = upload(e);
    if (rc != FPS_OK) return rc;
    const Batch b = batch_of(e);
    hipEvent_t e0, e1;
    HIPCHK_E(e, hipEventCreate(&e0));
    HIPCHK_E(e, hipEventCreate(&e1));
    for (int r = 0; r < 2; ++r) HIPCHK_E(e, launch_fv(b, e->stream));
    HIPCHK_E(e, hipEventRecord(e0, e->stream));
    for (int r = 0; r < reps; ++r) HIPCHK_E(e, launch_fv(b, e->stream));
    HIPCHK_E(e, hipEventRecord(e1, e->stream));
    HIPCHK_E(e, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCHK_E(e, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_out = ms / reps;
    return FPS_OK;
}
}  // namespace

extern "C" {

void fps_ped_params_default(fps_ped_params* o)
{
    if (!o) return;
    o->tau = 0.5;
    o->a_over_m = 25.0;
    o->b_range = 0.08;
    o->radius = 0.25;
    o->r_cut = 1.0;
    o->r_arrive = 1.0;
    const double v[5] = {0.0, 1.8, 0.9, 0.45, 0.0};
    for (int k = 0; k < 5; ++k) o->v_class[k] = v[k];
    o->hr_t[0] = 0.75;
    o->hr_t[1] = 1.5;
    o->hr_t[2] = 2.5;
    o->pick_s = 30.0;
    o->drop_s = 30.0;
    o->stability = 0;
    o->c_drag = 1.1;
    o->mu_f = 0.45;
    o->rho_w = 1000.0;
    o->rho_body = 1000.0;
    o->body_h0 = 1.71;
    o->body_m0 = 70.0;
    o->wading = 0;
    o->wade_k = 0.1;
}

size_t fps_workspace_bytes(const fps_grid_desc* desc, int32_t max_agents)
{
    char why[256];
    if (!valid_desc(desc, why) || max_agents < 0) return 0;
    return engine_header_bytes(1) + member_layout(desc, max_agents).total;
}

size_t fps_ens_workspace_bytes(int32_t S, const fps_grid_desc* descs, const int32_t* max_agents)
{
    char why[256];
    if (S < 1 || !descs) return 0;
    size_t total = engine_header_bytes(S);
    for (int k = 0; k < S; ++k) {
        if (!valid_desc(&descs[k], why)) return 0;
        int32_t ma = max_agents ? max_agents[k] : 0;
        if (ma < 0) return 0;
        total += member_layout(&descs[k], ma).total;
    }
    return total;
}

int fps_create(const fps_grid_desc* desc, const fps_ped_params* ped, int32_t max_agents,
               void* ws, size_t ws_bytes, void* stream, fps_sim** out)
{
    if (!out) return fail(nullptr, FPS_E_INVALID, "fps_create: out is NULL");
    *out = nullptr;
    Engine* e = new (std::nothrow) Engine();
    if (!e) return fail(nullptr, FPS_E_DEVICE, "fps_create: out of host memory");
    e->standalone = true;
    int rc = build_engine(e, 1, desc, ped, &max_agents, ws, ws_bytes, stream);
    if (rc != FPS_OK) {
        fail(nullptr, rc, "fps_create: %s", e->err);
        destroy_engine(e);
        delete e;
        return rc;
    }
    *out = e->m[0];
    return FPS_OK;
}

void fps_destroy(fps_sim* s)
{
    if (!s || !s->eng->standalone) return;   // members belong to their ensemble
    Engine* e = s->eng;
    destroy_engine(e);
    delete e;
}

int fps_ens_create(int32_t S, const fps_grid_desc* descs, const fps_ped_params* peds,
                   const int32_t* max_agents, void* ws, size_t ws_bytes, void* stream, fps_ens** out)
{
    if (!out) return fail(nullptr, FPS_E_INVALID, "fps_ens_create: out is NULL");
    *out = nullptr;
    fps_ens* e = new (std::nothrow) fps_ens();
    if (!e) return fail(nullptr, FPS_E_DEVICE, "fps_ens_create: out of host memory");
    int rc = build_engine(e, S, descs, peds, max_agents, ws, ws_bytes, stream);
    if (rc != FPS_OK) {
        fail(nullptr, rc, "fps_ens_create: %s", e->err);
        destroy_engine(e);
        delete e;
        return rc;
    }
    *out = e;
    return FPS_OK;
}

void fps_ens_destroy(fps_ens* e)
{
    if (!e) return;
    destroy_engine(e);
    delete e;
}

fps_sim* fps_ens_member(fps_ens* e, int32_t s)
{
    if (!e || s < 0 || s >= e->S) return nullptr;
    return e->m[s];
}

int fps_ens_step(fps_ens* e, int32_t n_steps)
{
    if (!e) return fail(nullptr, FPS_E_INVALID, "fps_ens_step: ens is NULL");
    return run_steps(e, n_steps, nullptr);
}

int fps_ens_step_profiled(fps_ens* e, int32_t n_steps, double* ms_out)
{
    if (!e || !ms_out) return fail(nullptr, FPS_E_INVALID, "fps_ens_step_profiled: NULL argument");
    return profiled(e, n_steps, ms_out);
}

int fps_ens_set_graph(fps_ens* e, int32_t steps_per_graph)
{
    if (!e) return fail(nullptr, FPS_E_INVALID, "fps_ens_set_graph: ens is NULL");
    if (steps_per_graph < 0 || steps_per_graph > 4096) return efail(e, FPS_E_INVALID, "steps_per_graph out of range");
    e->graph_chunk = steps_per_graph;
    drop_graph(e);
    return FPS_OK;
}

int fps_ens_set_flux(fps_ens* e, int32_t flux)
{
    if (!e) return fail(nullptr, FPS_E_INVALID, "fps_ens_set_flux: ens is NULL");
    if (flux != FPS_FLUX_HLLC && flux != FPS_FLUX_HLL) return efail(e, FPS_E_INVALID, "unknown flux %d", flux);
    e->hll = flux == FPS_FLUX_HLL;
    drop_graph(e);      // the captured launches name the kernel of the old flux
    return FPS_OK;
}

int fps_ens_autotune(fps_ens* e, const char* cache_path)
{
    if (!e) return fail(nullptr, FPS_E_INVALID, "fps_ens_autotune: ens is NULL");
    for (fps_sim* s : e->m)
        if (!s->fields_bound) return efail(e, FPS_E_STATE, "fps_ens_autotune: scenario %d: fields not bound", s->idx);
    HIPCHK_E(e, hipStreamSynchronize(e->stream));
    // the best heights depend on the whole mix of grids: the cache is keyed by it
    char arch[64] = "unknown";
    if (current_arch(arch, sizeof(arch)) != 0) return efail(e, FPS_E_DEVICE, "no HIP device");
    const uint64_t key = mix_key(e);
    std::vector<int64_t> c_sizes;
    std::vector<int> c_rows;
    if (ens_cache_lookup(cache_path, arch, key, c_sizes, c_rows)) {
        for (fps_sim* s : e->m) {
            const int64_t k = size_key(s->G.nx, s->G.ny);
            for (size_t i = 0; i < c_sizes.size(); ++i)
                if (c_sizes[i] == k) s->H = c_rows[i];
            mark_dirty(s);
        }
        return FPS_OK;
    }
    // The flood update of an ensemble is one launch over the tiles of every
    // member, which fills the chip: tune the rows per wave for that launch's
    // duration, not for each member alone (alone, a small grid is latency
    // bound and prefers short marches).  One height for every member first,
    // then each distinct grid size moved by factors of two while the launch
    // gets shorter by more than 1 %.
    int64_t cells = 0;
    for (fps_sim* s : e->m) cells += (int64_t)s->G.nx * s->G.ny;
    const int reps = cells > (1 << 26) ? 3 : 10;
    auto set_all = [&](int H) {
        for (fps_sim* s : e->m) {
            s->H = H;
            mark_dirty(s);
        }
    };
    // the common height: three interleaved passes over the heights, each
    // keeping its fastest (neighbouring heights differ by a few per cent,
    // about as much as one pass drifts with the clock)
    constexpr int kPasses = 3;
    float tmin[7] = {};
    for (int pass = 0; pass < kPasses; ++pass)
        for (int i = 0; i < 7; ++i) {
            set_all(1 << i);
            float ms = 0.0f;
            int rc = time_ensemble_flood(e, reps, &ms);
            if (rc != FPS_OK) return rc;
            if (pass == 0 || ms < tmin[i]) tmin[i] = ms;
        }
    int best_h = 1;
    float best = tmin[0];
    for (int i = 1; i < 7; ++i)
        if (tmin[i] < best) {
            best = tmin[i];
            best_h = 1 << i;
        }
    set_all(best_h);
    std::vector<int64_t> sizes;      // distinct grid sizes (size_key)
    for (fps_sim* s : e->m) {
        const int64_t key = size_key(s->G.nx, s->G.ny);
        if (std::find(sizes.begin(), sizes.end(), key) == sizes.end()) sizes.push_back(key);
    }
    if (sizes.size() > 1) {
        for (int pass = 0; pass < 2; ++pass) {
            bool moved = false;
            for (int64_t key : sizes) {
                int cur_h = 0;
                for (fps_sim* s : e->m)
                    if (size_key(s->G.nx, s->G.ny) == key) cur_h = s->H;
                for (int H : {cur_h * 2, cur_h / 2}) {
                    if (H < 1 || H > 64) continue;
                    for (fps_sim* s : e->m)
                        if (size_key(s->G.nx, s->G.ny) == key) {
                            s->H = H;
                            mark_dirty(s);
                        }
                    float ms = 0.0f;
                    int rc = time_ensemble_flood(e, reps, &ms);
                    if (rc != FPS_OK) return rc;
                    if (ms < 0.99f * best) {
                        best = ms;
                        cur_h = H;
                        moved = true;
                    }
                    for (fps_sim* s : e->m)
                        if (size_key(s->G.nx, s->G.ny) == key) {
                            s->H = cur_h;
                            mark_dirty(s);
                        }
                }
            }
            if (!moved) break;
        }
    }
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "%s ens %llx %d", arch, (unsigned long long)key, (int)sizes.size());
            for (int64_t k : sizes) {
                int h = 1;
                for (fps_sim* s : e->m)
                    if (size_key(s->G.nx, s->G.ny) == k) h = s->H;
                fprintf(f, " %d %d %d", (int)(k >> 32), (int)(uint32_t)k, h);
            }
            fprintf(f, " %.6f\n", (double)best);
            fclose(f);
        }
    }
    // the timing launches wrote scratch partials and the wetness flags
    for (fps_sim* s : e->m) {
        int rc = prime(s);
        if (rc != FPS_OK) return efail(e, rc, "%s", s->err);
    }
    return FPS_OK;
}

int fps_ens_time_flood(fps_ens* e, int32_t reps, double* ms_per_launch)
{
    if (!e || !ms_per_launch || reps < 1) return fail(nullptr, FPS_E_INVALID, "fps_ens_time_flood: bad argument");
    for (fps_sim* s : e->m)
        if (!s->fields_bound) return efail(e, FPS_E_STATE, "fps_ens_time_flood: scenario %d: fields not bound", s->idx);
    float ms = 0.0f;
    int rc = time_ensemble_flood(e, reps, &ms);
    if (rc != FPS_OK) return rc;
    *ms_per_launch = ms;
    // the timing launches wrote scratch partials and the wetness flags
    for (fps_sim* s : e->m) {
        rc = prime(s);
        if (rc != FPS_OK) return efail(e, rc, "%s", s->err);
    }
    return FPS_OK;
}

int fps_ens_active(fps_ens* e, int32_t* n_active)
{
    if (!e || !n_active) return fail(nullptr, FPS_E_INVALID, "fps_ens_active: NULL argument");
    HIPCHK_E(e, hipStreamSynchronize(e->stream));
    int32_t n = 0;
    for (fps_sim* s : e->m) {
        int32_t a = 0;
        HIPCHK_E(e, hipMemcpy(&a, &s->st->active, sizeof(a), hipMemcpyDeviceToHost));
        n += a;
    }
    *n_active = n;
    return FPS_OK;
}

const char* fps_ens_last_error(const fps_ens* e) { return e ? e->err : g_err; }

int fps_bind_fields(fps_sim* s, float* h, float* hu, float* hv, float* z)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_bind_fields: sim is NULL");
    if (!h || !hu || !hv || !z) return fail(s, FPS_E_INVALID, "fps_bind_fields: NULL field");
    // the same buffers again (new contents): launch parameters and captured
    // graphs stay valid
    const bool same = s->fields_bound && s->h == h && s->qx == hu && s->qy == hv && s->z == z;
    s->h = h; s->qx = hu; s->qy = hv; s->z = z;
    s->fields_bound = true;
    s->numeric_fault = false;
    if (!same) mark_dirty(s);
    int rc = write_state_i32(s, &s->st->status, 0);
    if (rc == FPS_OK) rc = write_state_i32(s, &s->st->settled, 0);
    if (rc == FPS_OK) rc = write_state_i32(s, &s->st->cur, 0);
    if (rc == FPS_OK) rc = write_state_i32(s, &s->st->frozen, 0);
    if (rc != FPS_OK) return rc;
    return prime(s);
}

int fps_set_flood_frozen(fps_sim* s, int32_t frozen)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_flood_frozen: sim is NULL");
    if (frozen != 0 && frozen != 1) return fail(s, FPS_E_INVALID, "fps_set_flood_frozen: 0 or 1");
    if (!s->fields_bound) return fail(s, FPS_E_STATE, "fps_set_flood_frozen: fields not bound");
    int rc = write_state_i32(s, &s->st->frozen, frozen);
    if (rc != FPS_OK) return rc;
    if (frozen) {
        // held steps have the fixed length dt_max and add no inflow
        const float dt = (float)s->G.dt_max;
        HIPCHK(s, hipMemcpyAsync(&s->st->dt, &dt, sizeof(dt), hipMemcpyHostToDevice, s->eng->stream));
        HIPCHK(s, hipStreamSynchronize(s->eng->stream));
        return FPS_OK;
    }
    return prime(s);     // the time step of the current state again
}

int fps_set_hydrograph(fps_sim* s, const double* t, const double* q, int32_t npts)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_hydrograph: sim is NULL");
    if (npts < 0 || npts > kMaxHydro) return fail(s, FPS_E_INVALID, "hydrograph: 0..%d points", kMaxHydro);
    if (npts > 0 && (!t || !q)) return fail(s, FPS_E_INVALID, "hydrograph: NULL arrays");
    for (int k = 0; k < npts; ++k) {
        if (!std::isfinite(t[k]) || !std::isfinite(q[k]))
            return fail(s, FPS_E_INVALID, "hydrograph: non-finite point %d", k);
        if (k > 0 && !(t[k] > t[k - 1])) return fail(s, FPS_E_INVALID, "hydrograph: times must increase");
    }
    double tt[kMaxHydro] = {0}, qq[kMaxHydro] = {0};
    for (int k = 0; k < npts; ++k) {
        tt[k] = t[k];
        qq[k] = q[k];
    }
    for (int k = 0; k < kMaxHydro; ++k) {
        s->hyd_t[k] = tt[k];
        s->hyd_q[k] = qq[k];
    }
    s->hyd_n = npts;
    hipStream_t st = s->eng->stream;
    HIPCHK(s, hipMemcpyAsync(s->st->hyd_t, tt, sizeof(tt), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(s->st->hyd_q, qq, sizeof(qq), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(&s->st->nh, &npts, sizeof(npts), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipStreamSynchronize(st));
    return prime(s);
}

int fps_set_navigation(fps_sim* s, int32_t n_dest, int32_t n_exit, const float* dist,
                       const uint8_t* walkable)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_navigation: sim is NULL");
    if (n_dest < 1 || n_exit < 1 || n_exit > n_dest || !dist || !walkable)
        return fail(s, FPS_E_INVALID, "fps_set_navigation: need 1 <= n_exit <= n_dest and arrays");
    s->n_dest = n_dest;
    s->n_exit = n_exit;
    s->dist = dist;
    s->walk = walkable;
    s->nav_bound = true;
    s->use_wmask = s->max_agents > 0 && (2 * s->Rx + 1) * (2 * s->Ry + 1) <= kMaskBits;
    if (s->use_wmask)
        HIPCHK(s, launch_wall_mask(walkable, s->wmask, s->G.nx, s->G.ny, s->Rx, s->Ry, s->eng->stream));
    s->use_codes = s->max_agents > 0 && n_dest <= kCodeDest;
    if (s->use_codes)
        HIPCHK(s, launch_nav_codes(dist, walkable, n_dest, s->G.nx, s->G.ny, (float)s->P.r_arrive, s->Rx, s->Ry,
                                   s->codes, s->eng->stream));
    mark_dirty(s);
    return FPS_OK;
}

int fps_bind_agents(fps_sim* s, int32_t n, float* x, float* y, float* vx, float* vy, float* v_base,
                    uint8_t* role, uint8_t* state, uint8_t* hr_class, int32_t* dest, float* timer)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_bind_agents: sim is NULL");
    if (n < 0 || n > s->max_agents)
        return fail(s, FPS_E_CAPACITY, "fps_bind_agents: %d agents, capacity %d", n, s->max_agents);
    if (n > 0 && (!x || !y || !vx || !vy || !v_base || !role || !state || !hr_class || !dest || !timer))
        return fail(s, FPS_E_INVALID, "fps_bind_agents: NULL array");
    hipStream_t st = s->eng->stream;
    if (n > 0) {
        if (!s->nav_bound) return fail(s, FPS_E_STATE, "fps_bind_agents: set the navigation map first");
        HIPCHK(s, launch_fill_i32(s->stats, 0, 2, st));
        HIPCHK(s, launch_check_agents(x, y, role, state, dest, n, (float)(s->G.nx * s->G.dx),
                                      (float)(s->G.ny * s->G.dy), s->n_dest, s->stats, st));
        int32_t bad[2] = {0, 0};
        HIPCHK(s, hipMemcpyAsync(bad, s->stats, sizeof(bad), hipMemcpyDeviceToHost, st));
        HIPCHK(s, hipStreamSynchronize(st));
        if (bad[0]) return fail(s, FPS_E_INVALID, "fps_bind_agents: %d agents outside the domain", bad[0]);
        if (bad[1])
            return fail(s, FPS_E_INVALID, "fps_bind_agents: %d agents with invalid role/state/dest", bad[1]);
    }
    s->na = n;
    s->body_h = s->body_m = nullptr;      // bodies follow the agents: set them again
    s->x = x; s->y = y; s->vx = vx; s->vy = vy; s->vbase = v_base;
    s->role = role; s->state = state; s->cls = hr_class; s->dest = dest; s->timer = timer;
    mark_dirty(s);
    int rc = rebuild_bins(s);
    return rc != FPS_OK ? rc : recount_outside(s);
}

int fps_set_bodies(fps_sim* s, const float* height, const float* mass)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_bodies: sim is NULL");
    if (!height != !mass) return fail(s, FPS_E_INVALID, "fps_set_bodies: give both arrays or neither");
    HIPCHK(s, hipStreamSynchronize(s->eng->stream));
    s->body_h = height;
    s->body_m = mass;
    mark_dirty(s);
    return FPS_OK;
}

int fps_set_doors(fps_sim* s, int32_t n_doors, const int32_t* cells, const int32_t* dests, int32_t per_step,
                  uint64_t seed)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_doors: sim is NULL");
    if (n_doors != 0 && (n_doors < 2 || n_doors > kMaxDoor))
        return fail(s, FPS_E_INVALID, "fps_set_doors: n_doors must be 0 or in [2, %d], got %d", kMaxDoor, n_doors);
    int32_t tab[2 * kMaxDoor] = {};
    if (n_doors > 0) {
        if (!cells || !dests) return fail(s, FPS_E_INVALID, "fps_set_doors: NULL array");
        if (per_step < 0) return fail(s, FPS_E_INVALID, "fps_set_doors: per_step must be >= 0, got %d", per_step);
        if (!s->nav_bound) return fail(s, FPS_E_STATE, "fps_set_doors: set the navigation map first");
        if (s->max_agents > (1 << 24))
            return fail(s, FPS_E_CAPACITY, "fps_set_doors: at most 2^24 agents (capacity %d)", s->max_agents);
        if (s->G.nx > (1 << 20) || s->G.ny > (1 << 20))
            return fail(s, FPS_E_CAPACITY, "fps_set_doors: at most 2^20 cells along a side");
        const int64_t nc = (int64_t)s->G.nx * s->G.ny;
        for (int k = 0; k < n_doors; ++k) {
            if (cells[k] < 0 || cells[k] >= nc)
                return fail(s, FPS_E_INVALID, "fps_set_doors: door %d: cell %d outside the grid", k, cells[k]);
            if (dests[k] < s->n_exit || dests[k] >= s->n_dest)
                return fail(s, FPS_E_INVALID, "fps_set_doors: door %d: destination %d not in [%d, %d)", k,
                            dests[k], s->n_exit, s->n_dest);
            tab[k] = cells[k];
            tab[kMaxDoor + k] = dests[k];
        }
    }
    hipStream_t st = s->eng->stream;
    HIPCHK(s, hipMemcpyAsync(s->doors, tab, sizeof(tab), hipMemcpyHostToDevice, st));
    int rc = write_state_i32(s, &s->st->doors_closed, 0);
    if (rc != FPS_OK) return rc;
    s->n_door = n_doors;
    s->door_rate = per_step;
    s->door_seed = seed;
    mark_dirty(s);
    return recount_outside(s);
}

int fps_set_barrier(fps_sim* s, const int32_t* cells, int32_t ncells, int32_t storage_dest,
                    int32_t barrier_dest, int32_t n_layers, float layer_thickness,
                    float last_thickness, int32_t bags_per)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_barrier: sim is NULL");
    if (ncells < 0 || (ncells > 0 && !cells)) return fail(s, FPS_E_INVALID, "fps_set_barrier: cells");
    if (ncells > s->line_cap) return fail(s, FPS_E_CAPACITY, "fps_set_barrier: %d cells > %d", ncells, s->line_cap);
    if (n_layers < 1 || bags_per < 1 || !(layer_thickness >= 0) || !(last_thickness >= 0))
        return fail(s, FPS_E_INVALID, "fps_set_barrier: layers/bags/thickness out of range");
    if (storage_dest < 0 || barrier_dest < 0 || (s->nav_bound && (storage_dest >= s->n_dest || barrier_dest >= s->n_dest)))
        return fail(s, FPS_E_INVALID, "fps_set_barrier: destination index out of range");
    const int64_t nc = (int64_t)s->G.nx * s->G.ny;
    for (int k = 0; k < ncells; ++k)
        if (cells[k] < 0 || cells[k] >= nc) return fail(s, FPS_E_INVALID, "fps_set_barrier: cell %d out of grid", k);
    hipStream_t st = s->eng->stream;
    if (ncells > 0)
        HIPCHK(s, hipMemcpyAsync(s->line, cells, sizeof(int32_t) * ncells, hipMemcpyHostToDevice, st));
    int32_t zero4[4] = {0, 0, 0, 0};
    HIPCHK(s, hipMemcpyAsync(&s->st->layers_done, zero4, sizeof(zero4), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipStreamSynchronize(st));
    s->nline = ncells;
    s->storage_dest = storage_dest;
    s->barrier_dest = barrier_dest;
    s->n_layers = n_layers;
    s->t_bag = layer_thickness;
    s->t_last = last_thickness;
    s->bags_per = bags_per;
    mark_dirty(s);
    return FPS_OK;
}

int fps_set_time(fps_sim* s, double t, int64_t step)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_time: sim is NULL");
    if (!std::isfinite(t) || step < 0) return fail(s, FPS_E_INVALID, "fps_set_time: bad time/step");
    hipStream_t st = s->eng->stream;
    HIPCHK(s, hipMemcpyAsync(&s->st->t, &t, sizeof(t), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(&s->st->step, &step, sizeof(step), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipStreamSynchronize(st));
    int rc = write_state_i32(s, &s->st->active, !(s->t_end > 0.0) || t < s->t_end);
    if (rc != FPS_OK) return rc;
    return prime(s);
}

namespace {
// unit discharge of the hydrograph at time t: piecewise linear between the
// breakpoints, the end values held outside them (as the flood update does)
static double host_hydro_q(const fps_sim* s, double t)
{
    const int n = s->hyd_n;
    if (n <= 0) return 0.0;
    if (t <= s->hyd_t[0]) return s->hyd_q[0];
    if (t >= s->hyd_t[n - 1]) return s->hyd_q[n - 1];
    for (int k = 0; k + 1 < n; ++k)
        if (t >= s->hyd_t[k] && t <= s->hyd_t[k + 1]) {
            const double w = (t - s->hyd_t[k]) / (s->hyd_t[k + 1] - s->hyd_t[k]);
            return s->hyd_q[k] + w * (s->hyd_q[k + 1] - s->hyd_q[k]);
        }
    return s->hyd_q[n - 1];
}
}  // namespace

int fps_inflow_depth(fps_sim* s, double t0, double t1, double* depth)
{
    if (!s || !depth) return fail(s, FPS_E_INVALID, "fps_inflow_depth: NULL argument");
    if (!std::isfinite(t0) || !std::isfinite(t1) || t1 < t0)
        return fail(s, FPS_E_INVALID, "fps_inflow_depth: need finite t0 <= t1");
    *depth = 0.0;
    if (s->G.inflow_side < 0 || s->hyd_n <= 0) return FPS_OK;
    // exact integral of the piecewise-linear discharge over [t0, t1]
    double total = 0.0, lo = t0;
    for (int k = 0; k < s->hyd_n; ++k) {
        const double tk = s->hyd_t[k];
        if (tk > lo && tk < t1) {
            total += 0.5 * (host_hydro_q(s, lo) + host_hydro_q(s, tk)) * (tk - lo);
            lo = tk;
        }
    }
    total += 0.5 * (host_hydro_q(s, lo) + host_hydro_q(s, t1)) * (t1 - lo);
    const double dn = s->G.inflow_side <= FPS_SIDE_E ? s->G.dx : s->G.dy;
    *depth = total / dn;
    return FPS_OK;
}

int fps_set_judge_region(fps_sim* s, const uint8_t* mask, int32_t block)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_judge_region: sim is NULL");
    if (mask && (block < 1 || block > 4096))
        return fail(s, FPS_E_INVALID, "fps_set_judge_region: block must be in [1, 4096]");
    if (mask && s->eng->order2)
        return fail(s, FPS_E_STATE, "fps_set_judge_region: not with the second-order variant");
    s->jmask = mask;
    s->jb = mask ? block : 0;
    mark_dirty(s);
    return FPS_OK;
}

int fps_set_occupancy(fps_sim* s, const int32_t* counts)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_occupancy: sim is NULL");
    if (s->na > 0) return fail(s, FPS_E_STATE, "fps_set_occupancy: agents are bound; counts come from them");
    hipStream_t st = s->eng->stream;
    const size_t nc = (size_t)s->G.nx * s->G.ny;
    if (counts) HIPCHK(s, hipMemcpyAsync(s->np, counts, sizeof(int32_t) * nc, hipMemcpyDeviceToDevice, st));
    else HIPCHK(s, launch_fill_i32(s->np, 0, (int64_t)nc, st));
    return FPS_OK;
}

int fps_set_end_time(fps_sim* s, double t_end)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_end_time: sim is NULL");
    if (!std::isfinite(t_end)) return fail(s, FPS_E_INVALID, "fps_set_end_time: t_end not finite");
    hipStream_t st = s->eng->stream;
    double t = 0.0;
    HIPCHK(s, hipMemcpyAsync(&s->st->t_end, &t_end, sizeof(t_end), hipMemcpyHostToDevice, st));
    HIPCHK(s, hipMemcpyAsync(&t, &s->st->t, sizeof(t), hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipStreamSynchronize(st));
    s->t_end = t_end;
    return write_state_i32(s, &s->st->active, !(t_end > 0.0) || t < t_end);
}

// the order of every scenario of an engine (1 or 2)
static int set_order(Engine* e, int32_t order, char* err)
{
    if (order != 1 && order != 2) return (snprintf(err, 512, "order must be 1 or 2, got %d", order), FPS_E_INVALID);
    if (order == 2)
        for (fps_sim* s : e->m)
            if (s->jmask)
                return (snprintf(err, 512, "scenario %d has a judge region (first order only)", s->idx),
                        FPS_E_STATE);
    e->order2 = order == 2;
    for (fps_sim* s : e->m) mark_dirty(s);     // the tiles of the march depend on the order
    drop_graph(e);      // the captured launches name the kernels of the old order
    return FPS_OK;
}

int fps_set_order(fps_sim* s, int32_t order)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_order: sim is NULL");
    if (!s->eng->standalone) return fail(s, FPS_E_STATE, "fps_set_order: member of an ensemble; use fps_ens_set_order");
    return set_order(s->eng, order, s->err);
}

int fps_ens_set_order(fps_ens* e, int32_t order)
{
    if (!e) return fail(nullptr, FPS_E_INVALID, "fps_ens_set_order: ens is NULL");
    return set_order(e, order, e->err);
}

int fps_set_flux(fps_sim* s, int32_t flux)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_flux: sim is NULL");
    if (flux != FPS_FLUX_HLLC && flux != FPS_FLUX_HLL) return fail(s, FPS_E_INVALID, "fps_set_flux: unknown flux %d", flux);
    if (!s->eng->standalone) return fail(s, FPS_E_STATE, "fps_set_flux: member of an ensemble; use fps_ens_set_flux");
    s->eng->hll = flux == FPS_FLUX_HLL;
    drop_graph(s->eng);
    return FPS_OK;
}

int fps_step(fps_sim* s, int32_t n_steps)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_step: sim is NULL");
    if (!s->eng->standalone) return fail(s, FPS_E_STATE, "fps_step: member of an ensemble; use fps_ens_step");
    int rc = run_steps(s->eng, n_steps, nullptr);
    if (rc != FPS_OK) return fail(s, rc, "fps_step: %s", s->eng->err);
    return FPS_OK;
}

int fps_step_profiled(fps_sim* s, int32_t n_steps, double* ms_out)
{
    if (!s || !ms_out) return fail(s, FPS_E_INVALID, "fps_step_profiled: NULL argument");
    if (!s->eng->standalone) return fail(s, FPS_E_STATE, "fps_step_profiled: member of an ensemble");
    int rc = profiled(s->eng, n_steps, ms_out);
    if (rc != FPS_OK) return fail(s, rc, "fps_step_profiled: %s", s->eng->err);
    return FPS_OK;
}

int fps_set_graph(fps_sim* s, int32_t steps_per_graph)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_graph: sim is NULL");
    if (steps_per_graph < 0 || steps_per_graph > 4096)
        return fail(s, FPS_E_INVALID, "fps_set_graph: steps_per_graph out of range");
    s->eng->graph_chunk = steps_per_graph;
    drop_graph(s->eng);
    return FPS_OK;
}

int fps_get_diag(fps_sim* s, fps_diag* out)
{
    if (!s || !out) return fail(s, FPS_E_INVALID, "fps_get_diag: NULL argument");
    hipStream_t st = s->eng->stream;
    HIPCHK(s, launch_fill_i32(s->stats, 0, 16, st));
    if (s->na > 0) HIPCHK(s, launch_agent_stats(s->state, s->cls, s->na, s->stats, st));
    DevState d;
    int32_t stats[16];
    HIPCHK(s, hipMemcpyAsync(&d, s->st, sizeof(d), hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipMemcpyAsync(stats, s->stats, sizeof(stats), hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipStreamSynchronize(st));
    std::memset(out, 0, sizeof(*out));
    out->t = d.t;
    out->step = d.step;
    out->ped_steps = (int64_t)d.ped_steps;
    out->dt_last = d.dt_prev;
    out->dt_next = d.dt;
    out->mass = d.mass;
    out->v_in = d.v_in;
    out->v_out = d.v_out;
    out->v_clip = d.v_clip;
    out->any_wet = d.any_wet;
    out->n_agents = s->na;
    for (int k = 0; k <= FPS_CLS_UNSTABLE; ++k) out->class_count[k] = stats[k];
    for (int k = 0; k <= FPS_ST_OUTSIDE; ++k) out->state_count[k] = stats[6 + k];
    out->barrier_layers_done = d.layers_done;
    out->barrier_active_cell = d.active_cell;
    out->barrier_bags = d.bags;
    out->barrier_done = d.done;
    out->drops_total = d.drops_total;
    out->status = d.status;
    out->active = d.active;
    out->flood_steps = d.flood_steps;
    out->doors_closed = d.doors_closed;
    out->door_entries = d.door_in;
    out->door_leaves = d.door_out;
    if (d.status != FPS_OK) {
        s->numeric_fault = true;
        return fail(s, FPS_E_NUMERIC, "non-finite state or time step detected on the device");
    }
    return FPS_OK;
}

int fps_get_time(fps_sim* s, double* t, double* dt_next)
{
    if (!s || !t || !dt_next) return fail(s, FPS_E_INVALID, "fps_get_time: NULL argument");
    hipStream_t st = s->eng->stream;
    double tt = 0.0;
    float dt = 0.0f;
    HIPCHK(s, hipMemcpyAsync(&tt, &s->st->t, sizeof(tt), hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipMemcpyAsync(&dt, &s->st->dt, sizeof(dt), hipMemcpyDeviceToHost, st));
    HIPCHK(s, hipStreamSynchronize(st));
    *t = tt;
    *dt_next = dt;
    return FPS_OK;
}

int fps_hazard_field(fps_sim* s, float* hr_out)
{
    if (!s || !hr_out) return fail(s, FPS_E_INVALID, "fps_hazard_field: NULL argument");
    if (!s->fields_bound) return fail(s, FPS_E_STATE, "fps_hazard_field: fields not bound");
    HIPCHK(s, launch_hazard(s->h, s->qx, s->qy, hr_out, (int64_t)s->G.nx * s->G.ny, (float)s->G.h_dry,
                            s->eng->stream));
    return FPS_OK;
}

int fps_get_counts(fps_sim* s, int32_t* counts)
{
    if (!s || !counts) return fail(s, FPS_E_INVALID, "fps_get_counts: NULL argument");
    HIPCHK(s, hipMemcpyAsync(counts, s->np, sizeof(int32_t) * (size_t)s->G.nx * s->G.ny,
                             hipMemcpyDeviceToDevice, s->eng->stream));
    return FPS_OK;
}

int fps_get_bins(fps_sim* s, int32_t* bin_start, int32_t* perm, int32_t* nbins_out)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_get_bins: sim is NULL");
    if (nbins_out) *nbins_out = s->nbins;
    if (s->na <= 0) return FPS_OK;
    if (bin_start)
        HIPCHK(s, hipMemcpyAsync(bin_start, s->bin_start, sizeof(int32_t) * (s->nbins + 1),
                                 hipMemcpyDeviceToDevice, s->eng->stream));
    if (perm) HIPCHK(s, launch_perm_from_slots(s->key, s->slot, s->na, perm, s->eng->stream));
    return FPS_OK;
}

int fps_time_flood(fps_sim* s, int32_t reps, double* ms_per_launch)
{
    if (!s || !ms_per_launch || reps < 1) return fail(s, FPS_E_INVALID, "fps_time_flood: bad argument");
    if (!s->fields_bound) return fail(s, FPS_E_STATE, "fps_time_flood: fields not bound");
    float ms = 0.0f;
    int rc = time_rows(s, s->H, reps, &ms);
    if (rc != FPS_OK) return rc;
    *ms_per_launch = ms;
    return prime(s);    // the timing launches wrote scratch partials and the wetness flags
}

int fps_set_rows_per_wave(fps_sim* s, int32_t rows)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_rows_per_wave: sim is NULL");
    if (rows < 1 || rows > 64 || (rows & (rows - 1)))
        return fail(s, FPS_E_INVALID, "fps_set_rows_per_wave: rows must be a power of two in [1, 64]");
    HIPCHK(s, hipStreamSynchronize(s->eng->stream));
    s->H = rows;
    mark_dirty(s);
    return FPS_OK;
}

int fps_get_rows_per_wave(fps_sim* s, int32_t* rows)
{
    if (!s || !rows) return fail(s, FPS_E_INVALID, "fps_get_rows_per_wave: NULL argument");
    *rows = s->H;
    return FPS_OK;
}

int fps_autotune(fps_sim* s, const char* cache_path, int32_t* rows_out, double* ms_out)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_autotune: sim is NULL");
    int rows = 0;
    double ms = 0.0;
    int rc = tune_member(s, cache_path, &rows, &ms);
    if (rc != FPS_OK) return rc;
    if (rows_out) *rows_out = rows;
    if (ms_out) *ms_out = ms;
    return FPS_OK;
}

int fps_stream_probe(float* buf, int64_t n, int64_t stride, int32_t n_in, int32_t n_out, int32_t reps, void* stream,
                     double* ms_per_pass)
{
    const bool shape = (n_in == 1 && n_out == 1) || (n_in == 4 && n_out == 3) || (n_in == 5 && n_out == 3);
    if (!buf || !ms_per_pass || n < 4 || n % 4 || stride < n || stride % 4 || !shape || reps < 1 ||
        (reinterpret_cast<uintptr_t>(buf) & 15))
        return fail(nullptr, FPS_E_INVALID, "fps_stream_probe: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        cus = 256;
    const int blocks = (int)std::min<int64_t>((n / 4 + 255) / 256, (int64_t)cus * 16);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return fail(nullptr, FPS_E_DEVICE, "fps_stream_probe: event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(nullptr, FPS_E_DEVICE, "fps_stream_probe: event");
    }
    hipError_t e = launch_stream_probe(buf, n, stride, n_in, n_out, blocks, st);
    if (e == hipSuccess) e = launch_stream_probe(buf, n, stride, n_in, n_out, blocks, st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_stream_probe(buf, n, stride, n_in, n_out, blocks, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return fail(nullptr, FPS_E_DEVICE, "fps_stream_probe: %s", hipGetErrorString(e));
    *ms_per_pass = ms / reps;
    return FPS_OK;
}

const char* fps_status_string(int status)
{
    switch (status) {
    case FPS_OK: return "ok";
    case FPS_E_INVALID: return "invalid argument";
    case FPS_E_DEVICE: return "device error";
    case FPS_E_STATE: return "invalid state";
    case FPS_E_CAPACITY: return "capacity exceeded";
    case FPS_E_NUMERIC: return "numeric fault";
    default: return "unknown status";
    }
}

const char* fps_last_error(const fps_sim* s) { return s ? s->err : g_err; }

}  // extern "C"
