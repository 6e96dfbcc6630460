// C-ABI of libfps (declared in include/fps.h): handle, workspace carving,
// argument validation and the stream-ordered step loop.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "fps_internal.h"

using namespace fps;

struct fps_sim {
    fps_grid_desc G;
    fps_ped_params P;
    int32_t max_agents;
    hipStream_t stream;
    char err[512];
    // workspace carve
    DevState* st;
    double* partials;
    float *h2, *qx2, *qy2;
    int32_t* np;
    int32_t *bin_count, *bin_start, *rank, *key, *perm_u, *perm;
    float2* xy;
    int32_t* slot;
    uint4* wmask;
    bool use_wmask;
    int32_t* line;
    int32_t* stats;
    int32_t line_cap;
    int H, nblocks_fv;
    int nbins, bsx, bsy, nbx, nby, Rx, Ry;
    int n_inflow;
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
    bool numeric_fault;
};

namespace {

char g_err[512] = "";

int fail(fps_sim* s, int code, const char* fmt, ...)
{
    char* buf = s ? s->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define HIPCHK(sim, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(sim, FPS_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

bool valid_desc(const fps_grid_desc* d, char* why)
{
    if (!d) return (snprintf(why, 256, "desc is NULL"), false);
    if (d->nx < 1 || d->ny < 1) return (snprintf(why, 256, "nx, ny must be >= 1"), false);
    if ((int64_t)d->nx * d->ny > (int64_t)1 << 31) return (snprintf(why, 256, "grid too large"), false);
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

struct Layout {
    size_t st, partials, h2, qx2, qy2, np, bin_count, bin_start, rank, key, perm_u, perm, xy, slot,
        wmask, line, stats, total;
    int nblocks, H;
    int64_t nbins_max;
    int32_t line_cap;
};

Layout make_layout(const fps_grid_desc* d, int32_t max_agents)
{
    Layout L{};
    const int64_t nc = (int64_t)d->nx * d->ny;
    L.H = fv_rows_per_wave(d->nx, d->ny);
    L.nblocks = fv_blocks(d->nx, d->ny, L.H);
    L.nbins_max = nc;   // bins are whole cells, at least one cell wide
    L.line_cap = 2 * (d->nx + d->ny);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    L.st = take(sizeof(DevState));
    L.partials = take(sizeof(double) * 4 * (size_t)L.nblocks);
    L.h2 = take(sizeof(float) * nc);
    L.qx2 = take(sizeof(float) * nc);
    L.qy2 = take(sizeof(float) * nc);
    L.np = take(sizeof(int32_t) * nc);
    size_t na = (size_t)std::max(max_agents, 0);
    L.bin_count = take(max_agents > 0 ? sizeof(int32_t) * L.nbins_max : 0);
    L.bin_start = take(max_agents > 0 ? sizeof(int32_t) * (L.nbins_max + 1) : 0);
    L.rank = take(sizeof(int32_t) * na);
    L.key = take(sizeof(int32_t) * na);
    L.perm_u = take(sizeof(int32_t) * na);
    L.perm = take(sizeof(int32_t) * na);
    L.xy = take(sizeof(float2) * na);
    L.slot = take(sizeof(int32_t) * na);
    L.wmask = take(max_agents > 0 ? sizeof(uint4) * nc : 0);
    L.line = take(sizeof(int32_t) * L.line_cap);
    L.stats = take(sizeof(int32_t) * 16);
    L.total = o;
    return L;
}

template <class T>
T* at(void* base, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(base) + off); }

FvParams fv_params(const fps_sim* s, int mode, const float* h, const float* qx, const float* qy,
                   float* ho, float* qxo, float* qyo)
{
    FvParams p{};
    p.h = h; p.qx = qx; p.qy = qy;
    p.ho = ho; p.qxo = qxo; p.qyo = qyo;
    p.z = s->z;
    p.np = s->np;
    p.st = s->st;
    p.partials = s->partials;
    p.nx = s->G.nx; p.ny = s->G.ny; p.H = s->H;
    p.nsx = (s->G.nx + kStrip - 1) / kStrip;
    p.ntiles = p.nsx * ((s->G.ny + s->H - 1) / s->H);
    p.nblocks = s->nblocks_fv;
    for (int k = 0; k < 4; ++k) p.bc[k] = s->G.bc[k];
    p.inflow_side = s->G.inflow_side;
    p.c0 = s->G.inflow_c0;
    p.c1 = s->G.inflow_c1;
    p.n_inflow = s->n_inflow;
    p.np_cap = s->G.np_cap;
    p.mode = mode;
    p.dx = (float)s->G.dx; p.dy = (float)s->G.dy;
    p.inv_dx = (float)(1.0 / s->G.dx); p.inv_dy = (float)(1.0 / s->G.dy);
    p.g = (float)s->G.g; p.half_g = (float)(0.5 * s->G.g);
    p.eps = (float)s->G.h_dry; p.cfl = (float)s->G.cfl; p.dt_max = (float)s->G.dt_max;
    p.n_base = (float)s->G.n_base;
    p.dxdy = s->G.dx * s->G.dy;
    return p;
}

PedParams ped_params(const fps_sim* s, const float* h, const float* qx, const float* qy)
{
    PedParams p{};
    p.x = s->x; p.y = s->y; p.vx = s->vx; p.vy = s->vy; p.vbase = s->vbase;
    p.role = s->role; p.state = s->state; p.cls = s->cls; p.dest = s->dest; p.timer = s->timer;
    p.na = s->na;
    p.h = h; p.qx = qx; p.qy = qy;
    p.z = s->z;
    p.np = s->np;
    p.dist = s->dist; p.walk = s->walk; p.n_dest = s->n_dest; p.n_exit = s->n_exit;
    p.bin_start = s->bin_start; p.xy = s->xy; p.slot = s->slot; p.wmask = s->wmask;
    p.use_wmask = s->use_wmask;
    p.bin_count = s->bin_count; p.rank = s->rank; p.key = s->key;
    p.st = s->st;
    p.nx = s->G.nx; p.ny = s->G.ny;
    p.bsx = s->bsx; p.bsy = s->bsy; p.nbx = s->nbx; p.nby = s->nby; p.Rx = s->Rx; p.Ry = s->Ry;
    p.nblocks = (s->na + kPedBlock - 1) / kPedBlock;
    p.dx = (float)s->G.dx; p.dy = (float)s->G.dy; p.eps = (float)s->G.h_dry;
    p.tau = (float)s->P.tau; p.a_over_m = (float)s->P.a_over_m; p.inv_b = (float)(1.0 / s->P.b_range);
    p.two_r = (float)(2.0 * s->P.radius); p.radius = (float)s->P.radius;
    p.r_cut = (float)s->P.r_cut; p.r_arrive = (float)s->P.r_arrive;
    for (int k = 0; k < 5; ++k) p.v_class[k] = (float)s->P.v_class[k];
    for (int k = 0; k < 3; ++k) p.hr_t[k] = (float)s->P.hr_t[k];
    p.pick_s = (float)s->P.pick_s; p.drop_s = (float)s->P.drop_s;
    p.storage_dest = s->storage_dest; p.barrier_dest = s->barrier_dest;
    p.fv_partials = s->partials;
    p.fv_blocks = s->nblocks_fv;
    return p;
}

BinParams bin_params(const fps_sim* s)
{
    BinParams b{};
    b.x = s->x; b.y = s->y; b.state = s->state; b.role = s->role;
    b.bin_count = s->bin_count; b.bin_start = s->bin_start; b.rank = s->rank; b.key = s->key;
    b.perm_u = s->perm_u; b.perm = s->perm; b.xy = s->xy; b.slot = s->slot; b.np = s->np;
    b.na = s->na; b.nbins = s->nbins; b.nx = s->G.nx; b.ny = s->G.ny;
    b.bsx = s->bsx; b.bsy = s->bsy; b.nbx = s->nbx;
    b.dx = (float)s->G.dx; b.dy = (float)s->G.dy;
    return b;
}

FinParams fin_params(const fps_sim* s, const FvParams& fv, int mode)
{
    FinParams f{};
    f.fv = fv;
    f.bar.z = s->z;
    f.bar.line = s->line;
    f.bar.nline = s->nline;
    f.bar.n_layers = s->n_layers;
    f.bar.bags_per = s->bags_per;
    f.bar.t_bag = s->t_bag;
    f.bar.t_last = s->t_last;
    f.bins = bin_params(s);
    f.do_barrier = mode == 0 && s->na > 0;
    f.do_scan = mode == 0 && s->na > 0;
    return f;
}

// recompute dt (and the inflow of the next step) from the bound state
int prime(fps_sim* s)
{
    if (!s->fields_bound) return FPS_OK;
    FvParams p = fv_params(s, 1, s->h, s->qx, s->qy, nullptr, nullptr, nullptr);
    HIPCHK(s, launch_fv(p, s->stream));
    HIPCHK(s, launch_finalize(fin_params(s, p, 1), s->stream));
    return FPS_OK;
}

int rebuild_bins(fps_sim* s)
{
    if (s->na <= 0) return FPS_OK;
    BinParams b = bin_params(s);
    HIPCHK(s, launch_fill_i32(s->bin_count, 0, s->nbins, s->stream));
    HIPCHK(s, launch_bin_keys(b, s->stream));
    HIPCHK(s, launch_bin_scan(b, s->stream));
    HIPCHK(s, launch_bin_place(b, s->stream));
    HIPCHK(s, launch_bin_sort(b, s->stream));
    HIPCHK(s, launch_fill_i32(s->np, 0, (int64_t)s->G.nx * s->G.ny, s->stream));
    HIPCHK(s, launch_count(b, s->stream));
    return FPS_OK;
}

struct KernelEvents {
    hipEvent_t ev[5][2];
    double ms[5];
    int n[5];
};

// one coupled step: flood update from (in) to (out), pedestrians, end of step
// (reductions, barrier, bin scan), then placement of the agents in the bins
int step_once(fps_sim* s, const float* hi, const float* qxi, const float* qyi, float* ho,
              float* qxo, float* qyo, KernelEvents* K)
{
    hipStream_t st = s->stream;
    auto rec = [&](int k, int w) {
        if (K) (void)hipEventRecord(K->ev[k][w], st);
    };
    auto harvest = [&](int k) {
        if (!K) return;
        float ms = 0.0f;
        (void)hipEventSynchronize(K->ev[k][1]);
        (void)hipEventElapsedTime(&ms, K->ev[k][0], K->ev[k][1]);
        K->ms[k] += ms;
        K->n[k] += 1;
    };
    FvParams fp = fv_params(s, 0, hi, qxi, qyi, ho, qxo, qyo);
    rec(0, 0);
    HIPCHK(s, launch_fv(fp, st));
    rec(0, 1);
    if (s->na > 0) {
        PedParams pp = ped_params(s, ho, qxo, qyo);
        rec(1, 0);
        HIPCHK(s, launch_ped(pp, st));
        rec(1, 1);
    }
    rec(2, 0);
    HIPCHK(s, launch_finalize(fin_params(s, fp, 0), st));
    rec(2, 1);
    if (s->na > 0) {
        BinParams b = bin_params(s);
        rec(3, 0);
        HIPCHK(s, launch_bin_place(b, st));
        rec(3, 1);
        rec(4, 0);
        HIPCHK(s, launch_bin_sort(b, st));
        rec(4, 1);
    }
    harvest(0);
    harvest(2);
    if (s->na > 0) {
        harvest(1);
        harvest(3);
        harvest(4);
    }
    return FPS_OK;
}

int run_steps(fps_sim* s, int32_t n, KernelEvents* K)
{
    if (!s->fields_bound) return fail(s, FPS_E_STATE, "fps_step: fields not bound");
    if (s->na > 0 && !s->nav_bound) return fail(s, FPS_E_STATE, "fps_step: agents need a navigation map");
    if (s->numeric_fault) return fail(s, FPS_E_STATE, "fps_step: numeric fault latched; rebind fields");
    if (n < 0) return fail(s, FPS_E_INVALID, "fps_step: n_steps < 0");
    for (int32_t k = 0; k < n; ++k) {
        int rc;
        if ((k & 1) == 0) rc = step_once(s, s->h, s->qx, s->qy, s->h2, s->qx2, s->qy2, K);
        else rc = step_once(s, s->h2, s->qx2, s->qy2, s->h, s->qx, s->qy, K);
        if (rc != FPS_OK) return rc;
    }
    if (n & 1) {
        size_t bytes = sizeof(float) * (size_t)s->G.nx * s->G.ny;
        HIPCHK(s, hipMemcpyAsync(s->h, s->h2, bytes, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(s, hipMemcpyAsync(s->qx, s->qx2, bytes, hipMemcpyDeviceToDevice, s->stream));
        HIPCHK(s, hipMemcpyAsync(s->qy, s->qy2, bytes, hipMemcpyDeviceToDevice, s->stream));
    }
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
}

size_t fps_workspace_bytes(const fps_grid_desc* desc, int32_t max_agents)
{
    char why[256];
    if (!valid_desc(desc, why) || max_agents < 0) return 0;
    return make_layout(desc, max_agents).total;
}

int fps_create(const fps_grid_desc* desc, const fps_ped_params* ped, int32_t max_agents,
               void* ws, size_t ws_bytes, void* stream, fps_sim** out)
{
    char why[256];
    if (!out) return fail(nullptr, FPS_E_INVALID, "fps_create: out is NULL");
    *out = nullptr;
    if (!valid_desc(desc, why)) return fail(nullptr, FPS_E_INVALID, "fps_create: %s", why);
    if (max_agents < 0) return fail(nullptr, FPS_E_INVALID, "fps_create: max_agents < 0");
    fps_ped_params P;
    if (ped) P = *ped;
    else fps_ped_params_default(&P);
    if (!(P.tau > 0) || !(P.b_range > 0) || !(P.r_cut > 0) || !(P.radius >= 0) || !(P.r_arrive >= 0))
        return fail(nullptr, FPS_E_INVALID, "fps_create: pedestrian constants out of range");
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
        return fail(nullptr, FPS_E_INVALID, "fps_create: workspace NULL or not 256-byte aligned");
    Layout L = make_layout(desc, max_agents);
    if (ws_bytes < L.total)
        return fail(nullptr, FPS_E_CAPACITY, "fps_create: workspace %zu bytes < %zu needed", ws_bytes,
                    L.total);
    fps_sim* s = new (std::nothrow) fps_sim();
    if (!s) return fail(nullptr, FPS_E_DEVICE, "fps_create: out of host memory");
    s->G = *desc;
    s->P = P;
    s->max_agents = max_agents;
    s->stream = static_cast<hipStream_t>(stream);
    s->st = at<DevState>(ws, L.st);
    s->partials = at<double>(ws, L.partials);
    s->h2 = at<float>(ws, L.h2);
    s->qx2 = at<float>(ws, L.qx2);
    s->qy2 = at<float>(ws, L.qy2);
    s->np = at<int32_t>(ws, L.np);
    s->bin_count = at<int32_t>(ws, L.bin_count);
    s->bin_start = at<int32_t>(ws, L.bin_start);
    s->rank = at<int32_t>(ws, L.rank);
    s->key = at<int32_t>(ws, L.key);
    s->perm_u = at<int32_t>(ws, L.perm_u);
    s->perm = at<int32_t>(ws, L.perm);
    s->xy = at<float2>(ws, L.xy);
    s->slot = at<int32_t>(ws, L.slot);
    s->wmask = at<uint4>(ws, L.wmask);
    s->line = at<int32_t>(ws, L.line);
    s->stats = at<int32_t>(ws, L.stats);
    s->line_cap = L.line_cap;
    s->H = L.H;
    s->nblocks_fv = L.nblocks;
    s->bsx = std::max(1, (int)std::ceil(P.r_cut / desc->dx - 1e-9));
    s->bsy = std::max(1, (int)std::ceil(P.r_cut / desc->dy - 1e-9));
    s->nbx = (desc->nx + s->bsx - 1) / s->bsx;
    s->nby = (desc->ny + s->bsy - 1) / s->bsy;
    s->nbins = s->nbx * s->nby;
    s->Rx = s->bsx;
    s->Ry = s->bsy;
    s->n_inflow = desc->inflow_side >= 0 ? desc->inflow_c1 - desc->inflow_c0 : 0;
    s->storage_dest = s->barrier_dest = -1;
    DevState h0{};
    h0.dt = (float)desc->dt_max;
    h0.dt_prev = (float)desc->dt_max;
    hipError_t e = hipMemcpyAsync(s->st, &h0, sizeof(h0), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) {
        int rc = FPS_OK;
        if (launch_fill_i32(s->np, 0, (int64_t)desc->nx * desc->ny, s->stream) != hipSuccess) rc = -1;
        if (max_agents > 0 && launch_fill_i32(s->bin_count, 0, L.nbins_max, s->stream) != hipSuccess) rc = -1;
        if (rc != FPS_OK) e = hipErrorLaunchFailure;
    }
    if (e != hipSuccess) {
        delete s;
        return fail(nullptr, FPS_E_DEVICE, "fps_create: %s", hipGetErrorString(e));
    }
    *out = s;
    return FPS_OK;
}

void fps_destroy(fps_sim* s)
{
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    delete s;
}

int fps_bind_fields(fps_sim* s, float* h, float* hu, float* hv, float* z)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_bind_fields: sim is NULL");
    if (!h || !hu || !hv || !z) return fail(s, FPS_E_INVALID, "fps_bind_fields: NULL field");
    s->h = h; s->qx = hu; s->qy = hv; s->z = z;
    s->fields_bound = true;
    s->numeric_fault = false;
    int32_t zero = 0;
    HIPCHK(s, hipMemcpyAsync(&s->st->status, &zero, sizeof(zero), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return prime(s);
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
    HIPCHK(s, hipMemcpyAsync(s->st->hyd_t, tt, sizeof(tt), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(s->st->hyd_q, qq, sizeof(qq), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(&s->st->nh, &npts, sizeof(npts), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
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
        HIPCHK(s, launch_wall_mask(walkable, s->wmask, s->G.nx, s->G.ny, s->Rx, s->Ry, s->stream));
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
    if (n > 0) {
        if (!s->nav_bound) return fail(s, FPS_E_STATE, "fps_bind_agents: set the navigation map first");
        HIPCHK(s, launch_fill_i32(s->stats, 0, 2, s->stream));
        HIPCHK(s, launch_check_agents(x, y, role, state, dest, n, (float)(s->G.nx * s->G.dx),
                                      (float)(s->G.ny * s->G.dy), s->n_dest, s->stats, s->stream));
        int32_t bad[2] = {0, 0};
        HIPCHK(s, hipMemcpyAsync(bad, s->stats, sizeof(bad), hipMemcpyDeviceToHost, s->stream));
        HIPCHK(s, hipStreamSynchronize(s->stream));
        if (bad[0]) return fail(s, FPS_E_INVALID, "fps_bind_agents: %d agents outside the domain", bad[0]);
        if (bad[1])
            return fail(s, FPS_E_INVALID, "fps_bind_agents: %d agents with invalid role/state/dest", bad[1]);
    }
    s->na = n;
    s->x = x; s->y = y; s->vx = vx; s->vy = vy; s->vbase = v_base;
    s->role = role; s->state = state; s->cls = hr_class; s->dest = dest; s->timer = timer;
    return rebuild_bins(s);
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
    if (ncells > 0)
        HIPCHK(s, hipMemcpyAsync(s->line, cells, sizeof(int32_t) * ncells, hipMemcpyHostToDevice, s->stream));
    int32_t zero4[4] = {0, 0, 0, 0};
    HIPCHK(s, hipMemcpyAsync(&s->st->active, zero4, sizeof(zero4), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    s->nline = ncells;
    s->storage_dest = storage_dest;
    s->barrier_dest = barrier_dest;
    s->n_layers = n_layers;
    s->t_bag = layer_thickness;
    s->t_last = last_thickness;
    s->bags_per = bags_per;
    return FPS_OK;
}

int fps_set_time(fps_sim* s, double t, int64_t step)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_set_time: sim is NULL");
    if (!std::isfinite(t) || step < 0) return fail(s, FPS_E_INVALID, "fps_set_time: bad time/step");
    HIPCHK(s, hipMemcpyAsync(&s->st->t, &t, sizeof(t), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipMemcpyAsync(&s->st->step, &step, sizeof(step), hipMemcpyHostToDevice, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
    return prime(s);
}

int fps_step(fps_sim* s, int32_t n_steps)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_step: sim is NULL");
    return run_steps(s, n_steps, nullptr);
}

int fps_step_profiled(fps_sim* s, int32_t n_steps, double* ms_out)
{
    if (!s || !ms_out) return fail(s, FPS_E_INVALID, "fps_step_profiled: NULL argument");
    KernelEvents K{};
    for (int k = 0; k < 5; ++k)
        for (int w = 0; w < 2; ++w) HIPCHK(s, hipEventCreate(&K.ev[k][w]));
    int rc = run_steps(s, n_steps, &K);
    (void)hipStreamSynchronize(s->stream);
    for (int k = 0; k < 5; ++k) {
        ms_out[k] = K.n[k] ? K.ms[k] / K.n[k] : 0.0;
        for (int w = 0; w < 2; ++w) (void)hipEventDestroy(K.ev[k][w]);
    }
    return rc;
}

int fps_get_diag(fps_sim* s, fps_diag* out)
{
    if (!s || !out) return fail(s, FPS_E_INVALID, "fps_get_diag: NULL argument");
    HIPCHK(s, launch_fill_i32(s->stats, 0, 16, s->stream));
    if (s->na > 0) HIPCHK(s, launch_agent_stats(s->state, s->cls, s->na, s->stats, s->stream));
    DevState d;
    int32_t stats[16];
    HIPCHK(s, hipMemcpyAsync(&d, s->st, sizeof(d), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipMemcpyAsync(stats, s->stats, sizeof(stats), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(s, hipStreamSynchronize(s->stream));
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
    for (int k = 0; k < 5; ++k) out->class_count[k] = stats[k];
    for (int k = 0; k < 6; ++k) out->state_count[k] = stats[5 + k];
    out->barrier_layers_done = d.layers_done;
    out->barrier_active_cell = d.active;
    out->barrier_bags = d.bags;
    out->barrier_done = d.done;
    out->drops_total = d.drops_total;
    out->status = d.status;
    if (d.status != FPS_OK) {
        s->numeric_fault = true;
        return fail(s, FPS_E_NUMERIC, "non-finite state or time step detected on the device");
    }
    return FPS_OK;
}

int fps_hazard_field(fps_sim* s, float* hr_out)
{
    if (!s || !hr_out) return fail(s, FPS_E_INVALID, "fps_hazard_field: NULL argument");
    if (!s->fields_bound) return fail(s, FPS_E_STATE, "fps_hazard_field: fields not bound");
    HIPCHK(s, launch_hazard(s->h, s->qx, s->qy, hr_out, (int64_t)s->G.nx * s->G.ny, (float)s->G.h_dry,
                            s->stream));
    return FPS_OK;
}

int fps_get_counts(fps_sim* s, int32_t* counts)
{
    if (!s || !counts) return fail(s, FPS_E_INVALID, "fps_get_counts: NULL argument");
    HIPCHK(s, hipMemcpyAsync(counts, s->np, sizeof(int32_t) * (size_t)s->G.nx * s->G.ny,
                             hipMemcpyDeviceToDevice, s->stream));
    return FPS_OK;
}

int fps_get_bins(fps_sim* s, int32_t* bin_start, int32_t* perm, int32_t* nbins_out)
{
    if (!s) return fail(nullptr, FPS_E_INVALID, "fps_get_bins: sim is NULL");
    if (nbins_out) *nbins_out = s->nbins;
    if (s->na <= 0) return FPS_OK;
    if (bin_start)
        HIPCHK(s, hipMemcpyAsync(bin_start, s->bin_start, sizeof(int32_t) * (s->nbins + 1),
                                 hipMemcpyDeviceToDevice, s->stream));
    if (perm)
        HIPCHK(s, hipMemcpyAsync(perm, s->perm, sizeof(int32_t) * s->na, hipMemcpyDeviceToDevice,
                                 s->stream));
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
