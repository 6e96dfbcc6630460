// Pedestrian step and neighbour binning on gfx950 (sec. 2.3-2.4, Table 1).
//
// 1, 4 or 16 lanes per agent (fewer when there are many agents): they share
// its neighbour and obstacle loops, and do the rest of its work in step.  Each agent reads the flood
// state of the navigation cell that contains it, takes its hazard class and
// walking speed (Table 1, HR = (max(|u|,|v|) + 0.5) h), follows its
// destination's distance field, is repelled by neighbours found in the 3x3
// bins around it and by obstacle cells, and moves.  Evacuee counts per cell
// (the N_p of the roughness rule) are kept by integer atomics on the old and
// new cells; responders deliver sandbags that the end-of-step kernel applies
// to the barrier line in order.
//
// Readings (the paper defers the pedestrian model to Karmakharm et al. 2010
// and Helbing's social force): exact relaxation v <- v0 e + (v - v0 e)
// exp(-dt/tau); repulsion A/m exp((2r - d)/B) from agents and A/m exp((r -
// d)/B) from the nearest point of obstacle cells within r_cut; |v| <= v0;
// axis-wise rejection of moves into obstacles or out of the domain; arrival
// when the destination distance at the new cell is <= r_arrive; evacuees stand
// until some cell is wet; dry cells: hazard class DRY at the agent's own speed.
// Before the flood, walkers of the door flow (sec. 3.2) walk at their own
// speed to the door they leave by; the door kernel below lets free slots in.
//
// Binning is a stable counting sort by (bin, agent id): integer histogram with
// atomic ranks, one-block exclusive scan, placement by rank, then each agent
// finds its final slot by counting the smaller ids of its own bin, so the
// result is deterministic and equal to a stable sort.
#include "fps_device.h"

// No contraction of a * b + c into fused multiply-adds in this file: the
// compiler would choose them per instantiation (the kernel is built for 1, 4
// and 16 lanes per agent, one scenario or many), and the pedestrian dynamics
// grow a last-bit difference into a different walk within a few steps.  With
// every multiply and add rounded on its own, every instantiation gives the
// same bits.
#pragma clang fp contract(off)

namespace fps {
namespace {

__device__ __forceinline__ int cell_of(float x, float d, int n)
{
    // IEEE division and floor in FP32; may return -1 or n (outside)
    float f = floorf(x / d);
    if (f < -1.0f) return -1;
    if (f > (float)n) return n;
    return (int)f;
}

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__device__ __forceinline__ float dist_at(const PedParams& p, int d, int i, int j)
{
    return p.dist[((size_t)d * p.ny + j) * p.nx + i];
}

__device__ __forceinline__ int nearest_exit(const PedParams& p, int ci, int cj)
{
    int best = 0;
    float bd = dist_at(p, 0, ci, cj);
    for (int e = 1; e < p.n_exit; ++e) {
        float de = dist_at(p, e, ci, cj);
        if (de < bd) {
            bd = de;
            best = e;
        }
    }
    return best;
}

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// The eight neighbour offsets in the tie order of the heading rule (E, N, W, S, NE, NW, SW, SE),
// packed two bits an offset (offset + 1) so that a run-time index selects one
// without a table in memory.
constexpr int kOffX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
constexpr int kOffY[8] = {0, 1, 0, -1, 1, 1, -1, -1};
constexpr uint32_t pack_offsets(const int (&o)[8])
{
    uint32_t v = 0;
    for (int k = 0; k < 8; ++k) v |= (uint32_t)(o[k] + 1) << (2 * k);
    return v;
}
constexpr uint32_t kOffXPacked = pack_offsets(kOffX), kOffYPacked = pack_offsets(kOffY);
__device__ __forceinline__ int off_of(uint32_t packed, int k) { return (int)((packed >> (2 * k)) & 3u) - 1; }

// Heading and arrival codes of a destination's distance field (sec. 2.1 navigation):
// the decisions the pedestrian step takes from the field at a cell, taken
// once per cell when the navigation map is set.  Bits 0-3: the neighbour to
// head for (0-7 in the order above: the first of the smallest distances
// below the cell's own), 8 for the cell's own centre (the destination, at
// distance 0), 15 for none; bit 4: the distance is within the arrival
// radius; bit 5: no obstacle cell within the repulsion window around the
// cell; bit 6: the cell is walkable (the last two the same for every
// destination).  The FP32 comparisons are those the step would make, in the
// same order, so the decisions are the same.
constexpr int kCodeNone = 15, kCodeHere = 8, kCodeArrive = 16, kCodeClear = 32, kCodeWalk = 64;

// Repulsion of one neighbour or obstacle point at offset (rx, ry) from the
// agent: A/m exp((r0 - d)/B) along the unit offset, zero outside (0, r_cut).
__device__ __forceinline__ void repel(const PedParams& p, float rx, float ry, float r0, float& fx, float& fy)
{
    const float d = __builtin_amdgcn_sqrtf(rx * rx + ry * ry);
    if (!(d > 0.0f) || !(d < p.r_cut)) return;
    const float w = p.a_over_m * __expf((r0 - d) * p.inv_b) * rcp(d);
    fx += w * rx;
    fy += w * ry;
}

// The partner of a lane at butterfly distance O within its group, by a DPP
// move: lane ^ 1 and lane ^ 2 by quad permutes; at distances 4 and 8 the
// half-row and row mirrors (lane 7 - k, 15 - k) serve, since by then every
// lane of an aligned group of O holds the same value.
template <int O>
__device__ __forceinline__ float lane_partner(float v)
{
    constexpr int kCtrl = O == 1 ? 0xB1 : O == 2 ? 0x4E : O == 4 ? 0x141 : 0x140;
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xF, 0xF, true));
}

// One butterfly level over the slot index: across lanes below L, within the
// lane from L on.
template <int O, int L>
__device__ __forceinline__ void slot_level(float (&v)[kSlots / L])
{
    constexpr int J = kSlots / L;
    if constexpr (O < L) {
#pragma unroll
        for (int j = 0; j < J; ++j) v[j] += lane_partner<O>(v[j]);
    } else {
        float w[J];
#pragma unroll
        for (int j = 0; j < J; ++j) w[j] = v[j] + v[j ^ (O / L)];
#pragma unroll
        for (int j = 0; j < J; ++j) v[j] = w[j];
    }
}

// The kSlots partial sums of an agent, slot s = q + jL held by lane q of its
// group as v[j], added by a butterfly over the slot index (levels 1, 2, 4,
// 8).  Every slot ends with the total, with the same bits for any L (each
// level adds the same two values).
template <int L>
__device__ __forceinline__ float slot_sum(float (&v)[kSlots / L])
{
    static_assert(kSlots == 16, "four butterfly levels");
    slot_level<1, L>(v);
    slot_level<2, L>(v);
    slot_level<4, L>(v);
    slot_level<8, L>(v);
    return v[0];
}

// Row of cell b (< wcells) of a window wdth cells wide: b * ceil(2^20 /
// wdth) >> 20 is exact while b < 2^20 / wdth, so windows of fewer cells than
// that use it; larger ones divide.
__device__ __forceinline__ int window_row(int b, int wdth, int wcells, uint32_t wmagic)
{
    return wcells <= (1 << 20) / wdth ? (int)(((uint64_t)(uint32_t)b * wmagic) >> 20) : b / wdth;
}

// The agent's record, read before anything else of the step.
struct AgentRec {
    float x, y, vx, vy, vbase, timer, body_h, body_m;
    int state, role, dest, slot;
};

__device__ __forceinline__ AgentRec load_agent(const PedParams& p, int a)
{
    AgentRec r;
    r.state = p.state[a];
    r.x = p.x[a];
    r.y = p.y[a];
    r.vx = p.vx[a];
    r.vy = p.vy[a];
    r.role = p.role[a];
    r.dest = p.dest[a];
    r.vbase = p.vbase[a];
    r.slot = p.slot[a];
    r.timer = p.timer[a];
    r.body_h = p.body_h0;
    r.body_m = p.body_m0;
    if ((p.stab || p.wade) && p.body_h) {
        r.body_h = p.body_h[a];
        r.body_m = p.body_m[a];
    }
    return r;
}

// One agent, one step, on the L lanes of its group (q = lane in the group).
// Every lane evaluates the agent's own state; the lanes share the neighbour
// and obstacle loops and the group sum combines their forces; lane 0 stores.
// The loads come in four dependent rounds: the agent record; everything
// addressed by its cell (flood state, the nine distances of its destination
// field, the obstacle mask, the bin bounds of the three bin rows); the
// neighbours' positions (with one lane per agent, also the discharge of a wet
// cell); the cells of the move.  Cell and bin indices use IEEE
// division so they match the FP32 decisions of the oracle exactly.
template <int L>
__device__ void agent_step(const PedParams& p, const AgentRec& rec, const float* __restrict__ fh,
                           const float* __restrict__ fqx, const float* __restrict__ fqy, int a, int q,
                           float dt, int any_wet, int done, int& drop, int& left)
{
    const bool lead = q == 0;
    const int st0 = rec.state;
    const float x = rec.x, y = rec.y;
    float vx = rec.vx, vy = rec.vy;
    const int role = rec.role;
    int dest = rec.dest;
    const float vbase = rec.vbase;
    const int self = rec.slot;
    if (st0 == FPS_ST_EXITED || st0 == FPS_ST_OUTSIDE) {
        if (lead) p.key[a] = -1;
        return;
    }
    const int ci = clampi(cell_of(x, p.dx, p.nx), 0, p.nx - 1);
    const int cj = clampi(cell_of(y, p.dy, p.ny), 0, p.ny - 1);
    const size_t c = (size_t)cj * p.nx + ci;
    const size_t nc = (size_t)p.nx * p.ny;
    // the agent's state and destination, from its record alone (the new
    // destination of an agent without one reads the exits' distances), so
    // that the record is complete before the next round of loads goes out
    int st = st0;
    if (dest < 0) {
        if (role == FPS_ROLE_EVACUEE) {
            dest = nearest_exit(p, ci, cj);
            st = FPS_ST_EVAC;
        } else {
            dest = p.storage_dest;
            st = FPS_ST_TO_STORAGE;
        }
    }
    if (role == FPS_ROLE_RESPONDER && done && st != FPS_ST_EVAC) {
        st = FPS_ST_EVAC;
        dest = nearest_exit(p, ci, cj);
    }
    // the flood has reached the site: walkers of the pre-flood flow become
    // evacuees heading for the nearest exit
    if (st == FPS_ST_SHOPPING && any_wet) {
        st = FPS_ST_EVAC;
        dest = nearest_exit(p, ci, cj);
    }
    bool moving = true;
    if (st == FPS_ST_PICKING || st == FPS_ST_DROPPING) {
        float tm = rec.timer - dt;
        if (lead) p.timer[a] = tm;
        if (tm > 0.0f) {
            moving = false;
        } else if (st == FPS_ST_PICKING) {
            st = FPS_ST_TO_BARRIER;
            dest = p.barrier_dest;
        } else {
            drop = 1;
            st = FPS_ST_TO_STORAGE;
            dest = p.storage_dest;
        }
    }
    if (moving && role == FPS_ROLE_EVACUEE && st == FPS_ST_EVAC && !any_wet) moving = false;
    // an agent without a valid destination (e.g. a responder with no barrier set) stands
    if (dest < 0 || dest >= p.n_dest) moving = false;
    // second load round: everything addressed by the cell.
    // A 32 x 32 -> 64-bit product: the 64 x 64 one leaves its upper addend
    // undefined, and the register chosen for it can be a load still in flight
    const uint64_t doff = (uint64_t)(uint32_t)(moving ? dest : 0) * (uint64_t)(uint32_t)nc;
    const float* D = p.dist + doff;
    const uint8_t* K = p.codes + doff;
    const float h = fh[c];
    float qxc = 0.0f, qyc = 0.0f;     // the cell's discharge: this round with several lanes per agent
    if constexpr (L > 1) {
        qxc = fqx[c];
        qyc = fqy[c];
    }
    const int kc = moving && p.use_codes ? (int)K[c] : 0;       // the cell's code of the destination
    uint4 m4 = make_uint4(0, 0, 0, 0);
    if (p.use_wmask) {
        // with one lane per agent (many agents: the step is bound by memory
        // traffic) the obstacle mask is read only where the code says an
        // obstacle is near, a round later; with several lanes (few agents:
        // bound by latency) it goes out with this round
        if constexpr (L == 1) {
            if (!(kc & kCodeClear)) m4 = p.wmask[c];
        } else {
            m4 = p.wmask[c];
        }
    }
    const int bi = ci / p.bsx, bj = cj / p.bsy;
    const int qi0 = max(bi - 1, 0), qi1 = min(bi + 1, p.nbx - 1);
    // both bounds of every bin row are loaded (a row outside the grid reads
    // the agent's own row and is then made empty), so that the six loads go
    // out together: a load under a condition would make the empty-row copy
    // wait for the one before it
    int seg0[3], seg1[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const int qj = bj - 1 + r;
        const bool ok = qj >= 0 && qj < p.nby;
        const int row = ok ? qj : bj;
        const int s0 = p.bin_start[row * p.nbx + qi0], s1 = p.bin_start[row * p.nbx + qi1 + 1];
        seg0[r] = s0;
        seg1[r] = ok ? s1 : s0;
    }
    // the direction: from the cell's heading code of the destination (one
    // byte), or, for destinations beyond the coded ones, from the nine
    // distances of its field; the loads go out before the wait for the cell's
    // flood state (the hazard class below), so that they travel in the same
    // round as the cell's.
    float ex = 0.0f, ey = 0.0f;    // desired direction
    if (moving) {
        bool has_target;
        int ti, tj;
        if (p.use_codes) {
            const int code = kc & 15;
            has_target = code <= kCodeHere;
            const bool here_c = code == kCodeHere;
            ti = here_c ? ci : ci + off_of(kOffXPacked, code & 7);
            tj = here_c ? cj : cj + off_of(kOffYPacked, code & 7);
        } else {
            float dk[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int qi = ci + kOffX[k], qj = cj + kOffY[k];
                const bool in = qi >= 0 && qj >= 0 && qi < p.nx && qj < p.ny;
                const float val = D[(size_t)clampi(qj, 0, p.ny - 1) * p.nx + clampi(qi, 0, p.nx - 1)];
                dk[k] = in ? val : __builtin_inff();
            }
            const float here = D[c];
            // steepest descent: the first of the smallest neighbour distances
            // below the agent's own; on the destination (distance 0) the target
            // is the agent's cell.  Selected without a branch on the agent's own
            // distance (which would hold the other eight loads back until it
            // arrives) and with the offsets as constants (no offset table read).
            float best = here;
            int box = 0, boy = 0;
            bool found = false;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (dk[k] < best) {
                    best = dk[k];
                    box = kOffX[k];
                    boy = kOffY[k];
                    found = true;
                }
            }
            const bool at_goal = here == 0.0f;
            has_target = at_goal || found;
            ti = at_goal ? ci : ci + box;
            tj = at_goal ? cj : cj + boy;
        }
        if (has_target) {
            float tx = ((float)ti + 0.5f) * p.dx - x, ty = ((float)tj + 0.5f) * p.dy - y;
            float len2 = tx * tx + ty * ty;
            if (len2 > 0.0f) {
                float il = __builtin_amdgcn_rsqf(len2);
                ex = tx * il;
                ey = ty * il;
            }
        }
    }
    // the direction is needed here: this keeps the compiler from moving its
    // loads below the neighbour loop, where they would form a round of their own
    asm volatile("" : "+v"(ex), "+v"(ey));
    // with one lane per agent (many agents: the step is bound by memory
    // traffic) the cell's discharge is read only where the cell is wet, in
    // the round of the neighbours' positions
    if constexpr (L == 1) {
        if (h > p.eps) {
            qxc = fqx[c];
            qyc = fqy[c];
        }
    }
    // the forces first (they do not depend on the hazard class), so that
    // the discharge loads travel with the neighbour loads
    float fsx = 0.0f, fsy = 0.0f;
    if (moving) {
        // repulsion from the neighbours in the 3x3 bins (the three bins of one
        // bin row are one contiguous run of the sorted positions; the runs of
        // the three rows are numbered one after the other), then from the
        // obstacle cells of the window [-Rx, Rx] x [-Ry, Ry] around the cell
        // (row-major; nearest point of the obstacle cell to the agent).  Entry
        // k of each list goes into slot k mod kSlots, in list order; the slots
        // are then added by a fixed tree.  Lane q holds slots q, q + L, ...,
        // so the sum has the same bits whatever the number L of lanes.
        constexpr int J = kSlots / L;
        constexpr int U = J >= 8 ? 1 : 2;      // slot batches per round of loads
        float fx[J], fy[J];
#pragma unroll
        for (int j = 0; j < J; ++j) {
            fx[j] = 0.0f;
            fy[j] = 0.0f;
        }
        const int n0 = seg1[0] - seg0[0], n01 = n0 + seg1[1] - seg0[1];
        const int ntot = n01 + seg1[2] - seg0[2];
        for (int k0 = 0; k0 < ntot; k0 += U * kSlots) {
            int sl[U][J];
            float2 o[U][J];
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j) {
                    const int kk = k0 + u * kSlots + q + j * L;
                    sl[u][j] = kk < n0 ? seg0[0] + kk : kk < n01 ? seg0[1] + (kk - n0) : seg0[2] + (kk - n01);
                    o[u][j] = kk < ntot ? p.xy[sl[u][j]] : make_float2(x, y);
                }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int j = 0; j < J; ++j)
                    if (sl[u][j] != self) repel(p, x - o[u][j].x, y - o[u][j].y, p.two_r, fx[j], fy[j]);
        }
        const int wdth = 2 * p.Rx + 1, wcells = (kc & kCodeClear) ? 0 : wdth * (2 * p.Ry + 1);
        const uint32_t wmagic = ((1u << 20) + (uint32_t)wdth - 1u) / (uint32_t)wdth;
        for (int b0 = 0; b0 < wcells; b0 += kSlots) {
#pragma unroll
            for (int j = 0; j < J; ++j) {
                const int b = b0 + q + j * L;
                if (b >= wcells) continue;
                const int row = window_row(b, wdth, wcells, wmagic), col = b - row * wdth;
                const int wi = ci + col - p.Rx, wj = cj + row - p.Ry;
                bool obst;
                if (p.use_wmask) {
                    const uint32_t word = b < 32 ? m4.x : b < 64 ? m4.y : b < 96 ? m4.z : m4.w;
                    obst = (word >> (b & 31)) & 1u;
                } else {
                    obst = wi >= 0 && wj >= 0 && wi < p.nx && wj < p.ny && !p.walk[(size_t)wj * p.nx + wi];
                }
                if (obst) {
                    const float px = fminf(fmaxf(x, (float)wi * p.dx), (float)(wi + 1) * p.dx);
                    const float py = fminf(fmaxf(y, (float)wj * p.dy), (float)(wj + 1) * p.dy);
                    repel(p, x - px, y - py, p.radius, fx[j], fy[j]);
                }
            }
        }
        fsx = slot_sum<L>(fx);
        fsy = slot_sum<L>(fy);
    }
    // hazard of the containing cell (Table 1)
    int cls;
    float v0;
    if (!(h > p.eps)) {
        cls = FPS_CLS_DRY;
        v0 = vbase;
    } else {
        float u = qxc / h, v = qyc / h;
        float hr = (fmaxf(fabsf(u), fabsf(v)) + 0.5f) * h;
        cls = hr < p.hr_t[0] ? FPS_CLS_LOW
            : hr < p.hr_t[1] ? FPS_CLS_MEDIUM
            : hr < p.hr_t[2] ? FPS_CLS_HIGH : FPS_CLS_HIGHEST;
        // constant indices keep the parameter copy in registers
        v0 = cls == FPS_CLS_LOW ? p.v_class[FPS_CLS_LOW]
           : cls == FPS_CLS_MEDIUM ? p.v_class[FPS_CLS_MEDIUM]
           : cls == FPS_CLS_HIGH ? p.v_class[FPS_CLS_HIGH] : p.v_class[FPS_CLS_HIGHEST];
        if (p.stab || p.wade) {
            // the body: an upright cylinder of its volume, its weight less buoyancy
            const float bh = rec.body_h, bm = rec.body_m;
            const float area = bm / (p.stab_rb * bh);
            const float b = 2.0f * sqrtf(area * 0.318309886f);
            const float w_eff = p.stab_g * (bm - p.stab_rw * area * h);
            if (p.stab) {
                // stability rule: sliding, toppling about its edge, or water to its height
                const float u = sqrtf(qxc * qxc + qyc * qyc) / h;
                const float drag = p.stab_kd * b * h * u * u;
                const bool unstable = h >= bh || drag > p.stab_mu * w_eff || drag * (0.5f * h) > w_eff * (0.5f * b);
                if (unstable) {
                    cls = FPS_CLS_UNSTABLE;
                    v0 = 0.0f;
                }
            }
            if (p.wade) {
                // wading rule: no faster than the drag of wading lets the feet push
                const float vw = w_eff > 0.0f ? sqrtf(p.wade_k * w_eff / (p.stab_kd * b * h)) : 0.0f;
                v0 = fminf(v0, vw);
            }
        }
    }
    if (lead) p.cls[a] = (uint8_t)cls;
    float xn = x, yn = y;
    int ni = ci, nj = cj;
    if (!moving) {
        vx = 0.0f;
        vy = 0.0f;
    } else {
        // relaxation toward the desired velocity, then the forces
        float k = __expf(-dt / p.tau);
        vx = v0 * ex + (vx - v0 * ex) * k;
        vy = v0 * ey + (vy - v0 * ey) * k;
        vx += dt * fsx;
        vy += dt * fsy;
        float sp2 = vx * vx + vy * vy;
        if (sp2 > v0 * v0) {
            if (v0 > 0.0f) {
                float sc = v0 * __builtin_amdgcn_rsqf(sp2);
                vx *= sc;
                vy *= sc;
            } else {
                vx = 0.0f;
                vy = 0.0f;
            }
        }
        // move, rejecting an axis that lands in an obstacle or outside.  The
        // cells the outcome can depend on are read together (one round of
        // loads instead of three dependent ones), then selected.
        xn = x + dt * vx;
        const int ni_try = cell_of(xn, p.dx, p.nx);
        const int ny_try = cell_of(y + dt * vy, p.dy, p.ny);
        const bool in_x = ni_try >= 0 && ni_try < p.nx, in_y = ny_try >= 0 && ny_try < p.ny;
        const size_t ix = (size_t)clampi(ni_try, 0, p.nx - 1), iy = (size_t)clampi(ny_try, 0, p.ny - 1);
        const size_t nxs = (size_t)p.nx;
        bool w_x, w_xy, w_y;                    // walkable: (ni_try, cj), (ni_try, ny_try), (ci, ny_try)
        bool arr_xy, arr_x, arr_y, arr_0;       // arrival at each cell the move may end in
        if (p.use_codes) {
            const int k_xy = K[iy * nxs + ix], k_x = K[(size_t)cj * nxs + ix], k_y = K[iy * nxs + ci];
            w_x = k_x & kCodeWalk;
            w_xy = k_xy & kCodeWalk;
            w_y = k_y & kCodeWalk;
            arr_xy = k_xy & kCodeArrive;
            arr_x = k_x & kCodeArrive;
            arr_y = k_y & kCodeArrive;
            arr_0 = kc & kCodeArrive;
        } else {
            w_x = p.walk[(size_t)cj * nxs + ix];
            w_xy = p.walk[iy * nxs + ix];
            w_y = p.walk[iy * nxs + ci];
            arr_xy = D[iy * nxs + ix] <= p.r_arrive;
            arr_x = D[(size_t)cj * nxs + ix] <= p.r_arrive;
            arr_y = D[iy * nxs + ci] <= p.r_arrive;
            arr_0 = D[(size_t)cj * nxs + ci] <= p.r_arrive;
        }
        const bool okx = in_x && w_x;
        ni = okx ? ni_try : ci;
        if (!okx) {
            xn = x;
            vx = 0.0f;
        }
        yn = y + dt * vy;
        const bool oky = in_y && (okx ? w_xy : w_y);
        nj = oky ? ny_try : cj;
        if (!oky) {
            yn = y;
            vy = 0.0f;
        }
        const bool arrive = okx ? (oky ? arr_xy : arr_x) : (oky ? arr_y : arr_0);
        if (arrive) {
            if (st == FPS_ST_EVAC) {
                st = FPS_ST_EXITED;
            } else if (st == FPS_ST_TO_STORAGE) {
                st = FPS_ST_PICKING;
                if (lead) p.timer[a] = p.pick_s;
                vx = 0.0f;
                vy = 0.0f;
            } else if (st == FPS_ST_TO_BARRIER) {
                st = FPS_ST_DROPPING;
                if (lead) p.timer[a] = p.drop_s;
                vx = 0.0f;
                vy = 0.0f;
            } else if (st == FPS_ST_SHOPPING) {
                st = FPS_ST_OUTSIDE;      // left by its door: the slot is free again
                left = 1;
            }
        }
    }
    if (!lead) return;
    p.x[a] = xn;
    p.y[a] = yn;
    p.vx[a] = vx;
    p.vy[a] = vy;
    p.state[a] = (uint8_t)st;
    p.dest[a] = dest;
    // evacuee counts per cell (roughness write-back)
    const size_t cn = (size_t)nj * p.nx + ni;
    const bool was = role == FPS_ROLE_EVACUEE && st0 == FPS_ST_EVAC;
    const bool now = role == FPS_ROLE_EVACUEE && st == FPS_ST_EVAC;
    if (was && !(now && cn == c)) atomicSub(&p.np[c], 1);
    if (now && !(was && cn == c)) atomicAdd(&p.np[cn], 1);
    // bin key of the new position; the global binning also needs the
    // histogram and each agent's rank in its bin (the LDS binning counts the
    // keys itself)
    if (st != FPS_ST_EXITED && st != FPS_ST_OUTSIDE) {
        int b = (nj / p.bsy) * p.nbx + ni / p.bsx;
        p.key[a] = b;
        if (p.need_rank) p.rank[a] = atomicAdd(&p.bin_count[b], 1);
    } else {
        p.key[a] = -1;
    }
}

// One wave (= one block) per kWave / L agents of one scenario: the agent
// ranges of the scenarios are padded to whole multiples of kWave agents in the
// flattened index, so no block straddles two scenarios.
template <bool kOne, int L>
__global__ __launch_bounds__(kWave) void ped_step_kernel(Batch B)
{
    const int g0 = blockIdx.x * (kWave / L);
    if (g0 >= B.total_agents) return;
    const int sc = kOne ? 0 : find_scenario(B.agent_off, B.S, g0);
    const Scn& S = scn_at<kOne>(B, sc);
    const int q = (int)threadIdx.x & (L - 1);
    const int a = g0 - (kOne ? 0 : B.agent_off[sc]) + (int)threadIdx.x / L;
    const PedParams P = S.ped;     // by value: not reloaded after the agent's stores
    // the agent's record in the same round of loads as the scenario's state words
    AgentRec rec{};
    if (a < S.na) rec = load_agent(P, a);
    const DevState* st = S.fv.st;
    if (!st->active) return;
    const bool skipped = flood_skipped(st);
    // the flood state this step's pedestrians see: the new one, or the
    // unchanged one when the dry step skipped the flood update
    const int fb = skipped ? st->cur : (st->cur ^ 1);
    const float dt = st->dt;            // the step length of this step
    const int done = st->done;
    // evacuation trigger: some cell is wet after this step's flood update
    // one wetness flag per lane (the flood update sets them per group of blocks)
    // (a skipped update left the state, and its wetness, as they were)
    const int wet = skipped ? st->any_wet : (__ballot(S.fv.wet[kWetStride * threadIdx.x] != 0) != 0ull);
    int drop = 0, left = 0;
    if (a < S.na)
        agent_step<L>(P, rec, fb ? S.fv.h[1] : S.fv.h[0], fb ? S.fv.qx[1] : S.fv.qx[0], fb ? S.fv.qy[1] : S.fv.qy[0],
                   a, q, dt, wet, done, drop, left);
    // one wave per block: the sandbag drops of the wave (lane 0 of each
    // group), one atomic; the agent-steps of the step are the agents that
    // start it outside the exits, which the bins hold: one add per scenario,
    // by its first block, instead of a same-address atomic from every block
    const unsigned long long drops = __popcll(__ballot(drop && q == 0));
    const unsigned long long leaves = __popcll(__ballot(left && q == 0));
    if (threadIdx.x == 0) {
        DevState* stw = S.fv.st;
        if (drops) atomicAdd(&stw->drops, (int)drops);
        if (leaves) {
            atomicAdd(&stw->n_outside, (int)leaves);
            atomicAdd(reinterpret_cast<unsigned long long*>(&stw->door_out), leaves);
        }
        if (a == 0) atomicAdd(&stw->ped_steps, (unsigned long long)P.bin_start[P.nbx * P.nby]);
    }
}

// --- pre-flood door flow (sec. 3, sec. 3.2) ---------------------------------
// SplitMix64 (Steele, Lea & Flood 2014): output number c + 1 of the generator
// started from seed, i.e. its output mix applied to seed + (c + 1) * gamma.
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// draw k of slot a in step n (k = 0: entry door, 1: leaving door, 2, 3: offsets in the cell)
__device__ __forceinline__ uint64_t door_draw(uint64_t seed, int64_t n, int a, int k)
{
    return splitmix64_at(seed, ((uint64_t)n << 26) | ((uint64_t)(uint32_t)a << 2) | (uint64_t)k);
}

// an integer uniform in [0, m) from the upper 32 bits (multiply-shift)
__device__ __forceinline__ int draw_below(uint64_t u, int m)
{
    return (int)(((u >> 32) * (uint64_t)(uint32_t)m) >> 32);
}

// a point of the central half of a cell: 0.25 + 0.5 * (upper 24 bits) / 2^24
__device__ __forceinline__ float draw_mid(uint64_t u)
{
    return 0.25f + 0.5f * ((float)(uint32_t)(u >> 40) * 0x1p-24f);
}

// The entries of one step, one block per scenario, after the pedestrian step
// (so slots freed by walkers who left this step may enter at once) and before
// the end-of-step binning (which takes the entrants in through their keys).
// Every free slot draws a door; at each door the first door_rate slots in
// slot order that drew it enter.  The slots are scanned in chunks of the
// block: per door, a ballot gives each slot its rank in its wave, the wave
// counts in LDS its rank in the chunk, and the running count per door its
// rank in the step.  The scan stops once every door is full.
template <bool kOne>
__global__ __launch_bounds__(kScanThreads) void door_kernel(Batch B)
{
    constexpr int kW = kScanThreads / kWave;
    __shared__ int taken[kMaxDoor];
    __shared__ int wcnt[kW][kMaxDoor];
    const Scn& S = scn_at<kOne>(B, kOne ? 0 : (int)blockIdx.x);
    const PedParams& P = S.ped;
    const int nd = P.n_door;
    DevState* st = S.fv.st;
    if (nd == 0 || !st->active || st->doors_closed) return;
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x >> 6;
    // the same wetness as the pedestrian step of this step
    const bool skipped = flood_skipped(st);
    const bool wet = skipped ? st->any_wet != 0 : __ballot(S.fv.wet[kWetStride * lane] != 0) != 0ull;
    if (wet) {
        if (threadIdx.x == 0) st->doors_closed = 1;
        return;
    }
    if (st->n_outside <= 0) return;
    const int64_t n = st->step;
    const uint64_t seed = P.door_seed;
    const int rate = P.door_rate, na = P.na;
    if (threadIdx.x < kMaxDoor) taken[threadIdx.x] = 0;
    for (int base = 0; base < na; base += kScanThreads) {
        __syncthreads();
        bool full = true;
        for (int k = 0; k < nd; ++k) full = full && taken[k] >= rate;
        if (full) break;
        const int a = base + (int)threadIdx.x;
        const bool out = a < na && P.state[a] == FPS_ST_OUTSIDE;
        const int d = out ? draw_below(door_draw(seed, n, a, 0), nd) : -1;
        int below = 0;
        for (int k = 0; k < nd; ++k) {
            const uint64_t m = __ballot(d == k);
            if (lane == 0) wcnt[w][k] = __popcll(m);
            if (d == k) below = __popcll(m & ((1ull << lane) - 1ull));
        }
        __syncthreads();
        if (d >= 0) {
            int r = taken[d] + below;
            for (int v = 0; v < w; ++v) r += wcnt[v][d];
            if (r < rate) {
                const int dc = P.doors[d];
                const int ci = dc % P.nx, cj = dc / P.nx;
                const int j = draw_below(door_draw(seed, n, a, 1), nd - 1);
                const int leave = j < d ? j : j + 1;
                P.x[a] = ((float)ci + draw_mid(door_draw(seed, n, a, 2))) * P.dx;
                P.y[a] = ((float)cj + draw_mid(door_draw(seed, n, a, 3))) * P.dy;
                P.vx[a] = 0.0f;
                P.vy[a] = 0.0f;
                P.timer[a] = 0.0f;
                P.state[a] = FPS_ST_SHOPPING;
                P.cls[a] = FPS_CLS_DRY;
                P.dest[a] = P.doors[kMaxDoor + leave];
                const int b = (cj / P.bsy) * P.nbx + ci / P.bsx;
                P.key[a] = b;
                if (P.need_rank) P.rank[a] = atomicAdd(&P.bin_count[b], 1);
            }
        }
        __syncthreads();
        if ((int)threadIdx.x < nd) {
            int t = 0;
            for (int v = 0; v < kW; ++v) t += wcnt[v][threadIdx.x];
            taken[threadIdx.x] += t;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int e = 0;
        for (int k = 0; k < nd; ++k) e += min(taken[k], rate);
        st->n_outside -= e;
        st->door_in += e;
    }
}

// agents in one state (ballot counts, one atomic per wave)
__global__ void count_state_kernel(const uint8_t* state, int na, int value, int32_t* out)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const int n = __popcll(__ballot(a < na && state[a] == value));
    if ((threadIdx.x & (kWave - 1)) == 0 && n) atomicAdd(out, n);
}

// --- binning ---------------------------------------------------------------
__global__ void bin_keys_kernel(BinParams b)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= b.na) return;
    if (b.state[a] == FPS_ST_EXITED || b.state[a] == FPS_ST_OUTSIDE) {
        b.key[a] = -1;
        return;
    }
    int ci = clampi(cell_of(b.x[a], b.dx, b.nx), 0, b.nx - 1);
    int cj = clampi(cell_of(b.y[a], b.dy, b.ny), 0, b.ny - 1);
    int k = (cj / b.bsy) * b.nbx + ci / b.bsx;
    b.key[a] = k;
    b.rank[a] = atomicAdd(&b.bin_count[k], 1);
}

__global__ __launch_bounds__(kScanThreads) void bin_scan_kernel(BinParams b) { block_scan_bins(b); }

__global__ void bin_place_kernel(BinParams b)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < b.na) place_agent(b, a);
}

__global__ void bin_sort_kernel(BinParams b)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < b.na) sort_agent(b, a);
}

// Ensemble versions for scenarios with more agents than the finalize places
// inline (same padded flattened index as the pedestrian step).
__global__ __launch_bounds__(kPedBlock) void bin_place_all_kernel(Batch B)
{
    const int g0 = blockIdx.x * kPedBlock;
    if (g0 >= B.total_agents) return;
    const int sc = find_scenario(B.agent_off, B.S, g0);
    const Scn& S = B.scn[sc];
    if (S.inline_place) return;
    const int a = g0 - B.agent_off[sc] + (int)threadIdx.x;
    if (a < S.na) {
        const BinParams b = S.bins;    // by value: not reloaded after the stores
        place_agent(b, a);
    }
}
__global__ __launch_bounds__(kPedBlock) void bin_sort_all_kernel(Batch B)
{
    const int g0 = blockIdx.x * kPedBlock;
    if (g0 >= B.total_agents) return;
    const int sc = find_scenario(B.agent_off, B.S, g0);
    const Scn& S = B.scn[sc];
    if (S.inline_place) return;
    const int a = g0 - B.agent_off[sc] + (int)threadIdx.x;
    if (a < S.na) {
        const BinParams b = S.bins;
        sort_agent(b, a);
    }
}

// --- multi-block bin scan (scenarios with more than kMbScanBins bins) --------
// Instead of one block per scenario walking all its bins: the count of every
// chunk of kChunkBins bins (one block each), the exclusive scan of the chunk
// counts (the scenario's end-of-step block, which also writes the total), and
// the scan of every chunk from its offset (one block each), which clears the
// histogram behind it.  Integer sums: the bin starts are those of the
// one-block scan.  A scenario that does not step (past its end time) keeps
// its bins: the chunk-count launch records whether it stepped, since the end
// of the step may mark it inactive before the chunk scan runs.
constexpr int kChunkThreads = kChunkBins / 16;

__device__ __forceinline__ void chunk_counts(const BinParams& b, int k0, int (&v)[16])
{
    if (k0 + 16 <= b.nbins) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int4 w = *reinterpret_cast<const int4*>(b.bin_count + k0 + 4 * q);
            v[4 * q] = w.x; v[4 * q + 1] = w.y; v[4 * q + 2] = w.z; v[4 * q + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = k0 + e < b.nbins ? b.bin_count[k0 + e] : 0;
    }
}

__global__ __launch_bounds__(kChunkThreads) void bin_chunk_sum_kernel(Batch B)
{
    __shared__ int wt[kChunkThreads / kWave];
    const int g = blockIdx.x;
    const int sc = find_scenario(B.chunk_off, B.S, g);
    const Scn& S = B.scn[sc];
    const BinParams b = S.bins;
    const int c = g - B.chunk_off[sc];
    const int active = S.fv.st->active != 0;
    if (c == 0 && threadIdx.x == 0) b.csum[b.nchunk] = active;
    if (!active) return;
    int v[16];
    chunk_counts(b, c * kChunkBins + 16 * (int)threadIdx.x, v);
    int t = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) t += v[e];
    const int incl = wave_inclusive_scan(t);
    if ((threadIdx.x & (kWave - 1)) == kWave - 1) wt[threadIdx.x >> 6] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        int sum = 0;
        for (int w = 0; w < kChunkThreads / kWave; ++w) sum += wt[w];
        b.csum[c] = sum;
    }
}

__global__ __launch_bounds__(kChunkThreads) void bin_chunk_scan_kernel(Batch B)
{
    __shared__ int wt[kChunkThreads / kWave];
    const int g = blockIdx.x;
    const int sc = find_scenario(B.chunk_off, B.S, g);
    const Scn& S = B.scn[sc];
    const BinParams b = S.bins;
    const int c = g - B.chunk_off[sc];
    if (!b.csum[b.nchunk]) return;
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x >> 6;
    const int k0 = c * kChunkBins + 16 * (int)threadIdx.x;
    int v[16];
    chunk_counts(b, k0, v);
    const bool full = k0 + 16 <= b.nbins;
    if (full) {
#pragma unroll
        for (int q = 0; q < 4; ++q) *reinterpret_cast<int4*>(b.bin_count + k0 + 4 * q) = make_int4(0, 0, 0, 0);
    } else {
        for (int e = 0; e < 16; ++e)
            if (k0 + e < b.nbins) b.bin_count[k0 + e] = 0;
    }
    int t = 0;
#pragma unroll
    for (int e = 0; e < 16; ++e) t += v[e];
    const int incl = wave_inclusive_scan(t);
    if (lane == kWave - 1) wt[wid] = incl;
    __syncthreads();
    int run = b.csum[c] + incl - t;
    for (int w = 0; w < wid; ++w) run += wt[w];
    if (full) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            int4 w;
            w.x = run; run += v[4 * q];
            w.y = run; run += v[4 * q + 1];
            w.z = run; run += v[4 * q + 2];
            w.w = run; run += v[4 * q + 3];
            *reinterpret_cast<int4*>(b.bin_start + k0 + 4 * q) = w;
        }
    } else {
        for (int e = 0; e < 16; ++e) {
            if (k0 + e < b.nbins) b.bin_start[k0 + e] = run;
            run += v[e];
        }
    }
}

// the agents in bin order from each binned agent's slot (the step keeps only
// the slots; this list is for reading the bins out)
__global__ void perm_from_slots_kernel(const int32_t* key, const int32_t* slot, int na, int32_t* perm)
{
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < na && key[a] >= 0) perm[slot[a]] = a;
}

__global__ void count_kernel(BinParams b)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= b.na) return;
    if (b.role[a] != FPS_ROLE_EVACUEE || b.state[a] != FPS_ST_EVAC) return;
    int ci = clampi(cell_of(b.x[a], b.dx, b.nx), 0, b.nx - 1);
    int cj = clampi(cell_of(b.y[a], b.dy, b.ny), 0, b.ny - 1);
    atomicAdd(&b.np[(size_t)cj * b.nx + ci], 1);
}

__global__ void fill_i32_kernel(int32_t* p, int32_t v, int64_t n)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; k < n; k += (int64_t)gridDim.x * blockDim.x) p[k] = v;
}

__global__ void hazard_kernel(const float* h, const float* qx, const float* qy, float* hr,
                              int64_t n, float eps)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        float d = h[k];
        float r = 0.0f;
        if (d > eps) r = (fmaxf(fabsf(qx[k] / d), fabsf(qy[k] / d)) + 0.5f) * d;
        hr[k] = r;
    }
}

// Counts per hazard class (agents inside: neither exited nor outside) and per state: each wave counts
// its agents by ballots, one lane adds the wave's counts (integer sums, so
// the order does not matter).
__global__ void agent_stats_kernel(const uint8_t* state, const uint8_t* cls, int na, int32_t* out)
{
    constexpr int kCls = FPS_CLS_UNSTABLE + 1;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = a < na;
    const int s = in ? min((int)state[a], (int)FPS_ST_OUTSIDE) : -1;
    const int c = in && s != FPS_ST_EXITED && s != FPS_ST_OUTSIDE ? min((int)cls[a], kCls - 1) : -1;
    const bool first = (threadIdx.x & (kWave - 1)) == 0;
#pragma unroll
    for (int k = 0; k <= FPS_ST_OUTSIDE; ++k) {
        const int n = __popcll(__ballot(s == k));
        if (first && n) atomicAdd(&out[kCls + k], n);
    }
#pragma unroll
    for (int k = 0; k < kCls; ++k) {
        const int n = __popcll(__ballot(c == k));
        if (first && n) atomicAdd(&out[k], n);
    }
}

// Per cell, one bit per offset (di, dj) in [-Rx, Rx] x [-Ry, Ry], row-major
// from (-Rx, -Ry): set where that cell lies in the grid and is not walkable.
__global__ void wall_mask_kernel(const uint8_t* walk, uint4* mask, int nx, int ny, int Rx, int Ry)
{
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (int64_t)nx * ny) return;
    int i = (int)(c % nx), j = (int)(c / nx);
    uint32_t m[4] = {0, 0, 0, 0};
    int bit = 0;
    for (int dj = -Ry; dj <= Ry; ++dj)
        for (int di = -Rx; di <= Rx; ++di, ++bit) {
            int wi = i + di, wj = j + dj;
            if (wi < 0 || wj < 0 || wi >= nx || wj >= ny) continue;
            if (!walk[(size_t)wj * nx + wi]) m[bit >> 5] |= 1u << (bit & 31);
        }
    mask[c] = make_uint4(m[0], m[1], m[2], m[3]);
}

__global__ void nav_code_kernel(const float* __restrict__ dist, const uint8_t* __restrict__ walk, int n_dest, int nx,
                                int ny, float r_arrive, int Rx, int Ry, uint8_t* __restrict__ codes)
{
    const int64_t nc = (int64_t)nx * ny;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nc * n_dest) return;
    const int64_t d = g / nc, c = g - d * nc;
    const int ci = (int)(c % nx), cj = (int)(c / nx);
    const float* D = dist + d * nc;
    const float here = D[c];
    float best = here;
    int kb = -1;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int qi = ci + kOffX[k], qj = cj + kOffY[k];
        if (qi < 0 || qj < 0 || qi >= nx || qj >= ny) continue;
        const float v = D[(int64_t)qj * nx + qi];
        if (v < best) {
            best = v;
            kb = k;
        }
    }
    int code = here == 0.0f ? kCodeHere : kb >= 0 ? kb : kCodeNone;
    if (here <= r_arrive) code |= kCodeArrive;
    if (walk[c]) code |= kCodeWalk;
    bool clear = true;        // no obstacle cell in the window (cells outside the grid are none)
    for (int wj = max(cj - Ry, 0); wj <= min(cj + Ry, ny - 1) && clear; ++wj)
        for (int wi = max(ci - Rx, 0); wi <= min(ci + Rx, nx - 1); ++wi)
            clear = clear && walk[(int64_t)wj * nx + wi];
    if (clear) code |= kCodeClear;
    codes[g] = (uint8_t)code;
}

__global__ void check_agents_kernel(const float* x, const float* y, const uint8_t* role,
                                    const uint8_t* state, const int32_t* dest, int na, float lx,
                                    float ly, int n_dest, int32_t* bad)
{
    int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= na) return;
    float xa = x[a], ya = y[a];
    if (!(xa >= 0.0f && xa < lx && ya >= 0.0f && ya < ly)) atomicAdd(&bad[0], 1);
    const bool door_flow = state[a] == FPS_ST_SHOPPING || state[a] == FPS_ST_OUTSIDE;
    if (role[a] > FPS_ROLE_RESPONDER || state[a] > FPS_ST_OUTSIDE || dest[a] < -1 || dest[a] >= n_dest ||
        (door_flow && role[a] != FPS_ROLE_EVACUEE))
        atomicAdd(&bad[1], 1);
}

inline int blocks_for(int64_t n, int t) { return (int)((n + t - 1) / t); }

template <int L>
void launch_ped_lanes(const Batch& b, hipStream_t s)
{
    const dim3 grid(b.total_agents / (kWave / L));
    if (b.S == 1) hipLaunchKernelGGL((ped_step_kernel<true, L>), grid, dim3(kWave), 0, s, b);
    else hipLaunchKernelGGL((ped_step_kernel<false, L>), grid, dim3(kWave), 0, s, b);
}

}  // namespace

// Lanes per agent, by measurement: 16 for small crowds (latency bound: the
// lanes share an agent's neighbour and obstacle loops), 4 up to 2^18 agents
// (the 64-scenario sweep with 170 k agents: 58 us per step against 66 with
// 1 lane and 88 with 16), then 1, where the agents' own work fills the chip.
int ped_lanes(int64_t total_agents)
{
    return total_agents <= 8192 ? 16 : total_agents <= 262144 ? 4 : 1;
}

hipError_t launch_ped(const Batch& b, hipStream_t s)
{
    if (b.total_agents > 0) {
        switch (ped_lanes(b.total_agents)) {
        case 16: launch_ped_lanes<16>(b, s); break;
        case 4: launch_ped_lanes<4>(b, s); break;
        default: launch_ped_lanes<1>(b, s); break;
        }
    }
    return hipGetLastError();
}
hipError_t launch_doors(const Batch& b, hipStream_t s)
{
    if (b.S == 1) hipLaunchKernelGGL((door_kernel<true>), dim3(1), dim3(kScanThreads), 0, s, b);
    else hipLaunchKernelGGL((door_kernel<false>), dim3(b.S), dim3(kScanThreads), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_count_state(const uint8_t* state, int na, int value, int32_t* out, hipStream_t s)
{
    if (na > 0) hipLaunchKernelGGL(count_state_kernel, dim3(blocks_for(na, 256)), dim3(256), 0, s, state, na, value, out);
    return hipGetLastError();
}
hipError_t launch_nav_codes(const float* dist, const uint8_t* walk, int n_dest, int nx, int ny, float r_arrive,
                            int Rx, int Ry, uint8_t* codes, hipStream_t s)
{
    const int64_t n = (int64_t)nx * ny * n_dest;
    if (n > 0)
        hipLaunchKernelGGL(nav_code_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dist, walk, n_dest,
                           nx, ny, r_arrive, Rx, Ry, codes);
    return hipGetLastError();
}
hipError_t launch_perm_from_slots(const int32_t* key, const int32_t* slot, int na, int32_t* perm, hipStream_t s)
{
    if (na > 0)
        hipLaunchKernelGGL(perm_from_slots_kernel, dim3(blocks_for(na, 256)), dim3(256), 0, s, key, slot, na, perm);
    return hipGetLastError();
}
hipError_t launch_bin_place_all(const Batch& b, hipStream_t s)
{
    if (b.total_agents > 0)
        hipLaunchKernelGGL(bin_place_all_kernel, dim3(b.total_agents / kPedBlock), dim3(kPedBlock), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_chunk_sum(const Batch& b, hipStream_t s)
{
    if (b.total_chunks > 0)
        hipLaunchKernelGGL(bin_chunk_sum_kernel, dim3(b.total_chunks), dim3(kChunkThreads), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_chunk_scan(const Batch& b, hipStream_t s)
{
    if (b.total_chunks > 0)
        hipLaunchKernelGGL(bin_chunk_scan_kernel, dim3(b.total_chunks), dim3(kChunkThreads), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_sort_all(const Batch& b, hipStream_t s)
{
    if (b.total_agents > 0)
        hipLaunchKernelGGL(bin_sort_all_kernel, dim3(b.total_agents / kPedBlock), dim3(kPedBlock), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_keys(const BinParams& b, hipStream_t s)
{
    if (b.na > 0) hipLaunchKernelGGL(bin_keys_kernel, dim3(blocks_for(b.na, 256)), dim3(256), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_scan(const BinParams& b, hipStream_t s)
{
    hipLaunchKernelGGL(bin_scan_kernel, dim3(1), dim3(kScanThreads), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_place(const BinParams& b, hipStream_t s)
{
    if (b.na > 0) hipLaunchKernelGGL(bin_place_kernel, dim3(blocks_for(b.na, 256)), dim3(256), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_bin_sort(const BinParams& b, hipStream_t s)
{
    if (b.na > 0) hipLaunchKernelGGL(bin_sort_kernel, dim3(blocks_for(b.na, 256)), dim3(256), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_count(const BinParams& b, hipStream_t s)
{
    if (b.na > 0) hipLaunchKernelGGL(count_kernel, dim3(blocks_for(b.na, 256)), dim3(256), 0, s, b);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s)
{
    if (n > 0) {
        int g = (int)std::min<int64_t>(blocks_for(n, 256), 4096);
        hipLaunchKernelGGL(fill_i32_kernel, dim3(g), dim3(256), 0, s, p, v, n);
    }
    return hipGetLastError();
}
hipError_t launch_hazard(const float* h, const float* qx, const float* qy, float* hr, int64_t n,
                         float eps, hipStream_t s)
{
    int g = (int)std::min<int64_t>(blocks_for(n, 256), 8192);
    hipLaunchKernelGGL(hazard_kernel, dim3(g), dim3(256), 0, s, h, qx, qy, hr, n, eps);
    return hipGetLastError();
}
hipError_t launch_agent_stats(const uint8_t* state, const uint8_t* cls, int na, int32_t* out14,
                              hipStream_t s)
{
    if (na > 0)
        hipLaunchKernelGGL(agent_stats_kernel, dim3(blocks_for(na, 256)), dim3(256), 0, s, state,
                           cls, na, out14);
    return hipGetLastError();
}
hipError_t launch_wall_mask(const uint8_t* walk, uint4* mask, int nx, int ny, int Rx, int Ry,
                            hipStream_t s)
{
    int64_t n = (int64_t)nx * ny;
    hipLaunchKernelGGL(wall_mask_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, walk, mask, nx, ny,
                       Rx, Ry);
    return hipGetLastError();
}
hipError_t launch_check_agents(const float* x, const float* y, const uint8_t* role,
                               const uint8_t* state, const int32_t* dest, int na, float lx,
                               float ly, int n_dest, int32_t* bad2, hipStream_t s)
{
    if (na > 0)
        hipLaunchKernelGGL(check_agents_kernel, dim3(blocks_for(na, 256)), dim3(256), 0, s, x, y,
                           role, state, dest, na, lx, ly, n_dest, bad2);
    return hipGetLastError();
}

}  // namespace fps
