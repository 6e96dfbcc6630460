/*
 * fps_oracle.c -- plain, slow, FP64 CPU oracle of the coupled flood-pedestrian
 * step of Shirvani, Kesserwani & Richmond, "Agent-based simulator of dynamic
 * flood-people interactions" (arXiv 1908.05232).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the GPU library.
 *
 * What the paper fixes, and where:
 *   - state U = [h, hu, hv], fluxes F, G, bed-slope and Manning sources: Eq. (1), sec. 2.2
 *   - explicit update from east/west/north/south fluxes: Eq. (2), sec. 2.2
 *   - Godunov-type, first-order, 4-neighbour stencil with wetting/drying and
 *     terrain treatment: sec. 2.2 (deferring to Wang et al. 2011)
 *   - CFL-adaptive step when wet, 1.0 s pedestrian step when dry: sec. 3
 *   - HR = (V + 0.5) h with V = max(|u|, |v|); classes and walking speeds: Table 1, sec. 2.4
 *   - roughness rule n = n0 + Np n0 with at most 20 counted evacuees: sec. 2.4
 *   - responder cycle storage -> 30 s pick -> barrier -> 30 s drop; layer fill
 *     along the barrier line, N_L layers: sec. 2.4, sec. 3.3
 *   - triangular inflow hydrograph: sec. 3.1
 *   - richer walking-speed and stability rules and variable body shapes are
 *     named as further work (sec. 2.4 note 1, sec. 4): the stability rule
 *     (S1-S4) and the wading rule (W1-W3) below are this oracle's reading
 *     of them
 *   - pre-flood flow: 7 entrance doors, entering and leaving by each with
 *     probability 1/7, 10 per door, 1,000 walkers, a 5-minute spin-up with
 *     no inflow, no entries once water is on the site: sec. 3, sec. 3.2, sec. 2.4
 * Readings where the paper is silent (each also listed in the design notes):
 *   R1 Riemann solver: HLLC (Toro) with dry-bed wave speeds.  HLL part written
 *      anchored at the left state, which is the same formula rearranged so that
 *      two identical states return F(U) exactly.  Variant (P->flux): plain HLL
 *      (Harten, Lax & van Leer 1983) for all three components, the tangential
 *      momentum averaged like the other two instead of taken from the upwind
 *      side of the contact.
 *   R2 wetting/drying + terrain: non-negative hydrostatic reconstruction
 *      (Audusse et al. 2004), z_f = max(zL, zR), h* = h - (z_f - z); a face side
 *      with h* <= h_dry counts as dry and h* := 0.  Velocities come from the
 *      unreconstructed cell (0 if h <= h_dry).
 *   R3 the bed slope enters as the one-sided pressure correction 1/2 g h*^2 of
 *      the same reconstruction (exactly zero for a lake at rest).
 *   R4 Eq. (2) prints "+ S" without a time factor; read as + dt S.
 *   R5 Manning friction: splitting point-implicit (Liang & Marche 2009) with a
 *      no-reversal limiter, applied after the flux update where h > h_dry.
 *   R6 dt = min(CFL * min_wet min(dx/(|u|+c), dy/(|v|+c)), dt_max), dt_max = 1 s;
 *      dt_max when nothing is wet.
 *   R7 g and h_dry are parameters (9.81 m/s^2 and 1e-5 m in every scenario).
 *   R8 boundaries by ghost cells: wall = mirror (normal discharge negated; the
 *      wall face carries zero mass and tangential flux exactly); transmissive
 *      = copy.  The "slip" north side of sec. 3.1 is read as transmissive.
 *   R9 inflow: a line mass source on the cells along the inflow segment,
 *      depth += (1/dn) * integral of q over the step; piecewise-linear q
 *      integrated exactly; no momentum added.
 *   R10 coupled order per step: flood update with n and z of the previous step,
 *      then pedestrians with the new flood state, then write-back of n and z.
 *   R11 hazard: a dry cell (h <= h_dry) is class DRY at the agent's own base
 *      speed; class intervals are half-open [from, to); above 20 stays HIGHEST.
 *   R12 V in HR = (V + 0.5) h is max(|u|, |v|) as printed, not the speed.
 *   R13 roughness: n_eff = n0 (1 + min(Np, cap)), recomputed every step from
 *      the active evacuees whose containing cell it is (not cumulative).
 *   R14 navigation: per-destination distance field (input); step toward the
 *      centre of the 8-neighbour with the smallest distance, ties in the order
 *      E, N, W, S, NE, NW, SW, SE; inside a destination cell toward its centre.
 *   R15 movement: social force of Helbing, Farkas & Vicsek (2000): exact
 *      relaxation to v0 e over tau, exponential repulsion from neighbours in
 *      the 3x3 bins and from obstacle cells within r_cut, |v| <= v0, explicit
 *      position update with an axis-wise rejection of moves into obstacles or
 *      out of the domain.
 *   R16 arrival when the distance field at the new cell is <= r_arrive.
 *   R17 evacuees stay put until any cell is wet (evacuation trigger, sec. 2.4).
 *   R18 barrier: completed drops of a step are summed, then applied in order;
 *      one bag per drop; a cell-layer takes bags_per bags; z += layer thickness.
 *   R19 cell / bin indices are decided in FP32 (the GPU kernel's precision):
 *      i = floor((float)x / (float)dx).
 *   R21 cleanup after the update: h := max(h, 0) (clipped volume recorded),
 *      q := 0 where h <= h_dry.
 * Readings of the pre-flood door flow (or_doors; the paper gives the counts,
 * not the mechanism):
 *   D1 the agents are slots: the most people inside at once (1,000); a slot
 *      outside (OR_ST_OUTSIDE) may enter, at most door_rate per door per step
 *      (the 10 per door, per 1 s pedestrian step while dry).
 *   D2 admission: every free slot draws a door, each with probability 1/n_door,
 *      every step; at each door the first door_rate slots in slot order that
 *      drew it enter, at a uniform point of the central half of the door cell,
 *      standing, hazard class DRY.  Entries follow the step's pedestrian moves,
 *      so a slot freed in a step may enter in the same step.
 *   D3 an entrant heads for a leaving door drawn uniformly from the other doors
 *      (so each door is the leaving door with probability 1/n_door overall);
 *      arriving there (R16) it goes back outside.  Walkers move like evacuees
 *      (R14, R15) at their own dry speed and add no roughness (R13 counts
 *      evacuees only).
 *   D4 trigger (R17): the first step after whose flood update a cell is wet
 *      closes the doors for good; every walker inside becomes an evacuee
 *      heading for the nearest exit in that step's move (the doors are not
 *      exits: the emergency exit stays open).
 *   D5 spin-up: the run starts 300 s before the hydrograph, which is zero
 *      until then; the dry steps are the 1 s pedestrian step.
 *   D6 random numbers: SplitMix64 (Steele, Lea & Flood 2014) in counter form:
 *      draw k (0 entry door, 1 leaving door, 2 and 3 offsets in x and y) of
 *      slot a in step n is output (n * 2^26 + a * 4 + k) + 1 of the generator
 *      seeded with door_seed; a choice among m is floor((u >> 32) * m / 2^32),
 *      an offset 0.25 + 0.5 * floor(u / 2^40) / 2^24, the position
 *      ((float)i + offset) * (float)dx in FP32 (R19's precision).
 * Readings of the stability rule (or_unstable; the paper names richer
 * walking-speed and stability rules and variable bodies as further work):
 *   S1 every person has a body: height and mass (a default body for those
 *      without one).
 *   S2 the body is an upright cylinder of its own volume (mass over the body
 *      density); standing in water of depth h it loses the weight of the
 *      water it displaces and meets the drag of the flow speed (the magnitude
 *      of the cell's velocity, not the max of its components) on its wetted
 *      frontal area, acting half way up the water.
 *   S3 it cannot stand when the drag exceeds the foot friction on its
 *      effective weight (sliding), when the drag's moment exceeds that
 *      weight's moment about the cylinder's edge (toppling), or when the
 *      water reaches its height.
 *   S4 a person who cannot stand does not walk (speed 0) and takes a sixth
 *      state in floodwater, UNSTABLE, in place of its Table 1 class; on dry
 *      cells and with the rule off the paper's Table 1 alone applies.
 * Readings of the wading rule (or_wade_speed; the walking-speed half of the
 * same further work):
 *   W1 wading through still water of depth h at speed v, the body of S2 meets
 *      the drag 1/2 rho_w c_drag b h v^2 on its wetted frontal width b.
 *   W2 its feet keep up a horizontal push of at most wade_k times its weight
 *      less buoyancy, W' = g (M - rho_w A h); the fastest it can wade is the
 *      speed at which the two balance, sqrt(2 wade_k W' / (rho_w c_drag b
 *      h)), and 0 once buoyancy takes the whole weight.
 *   W3 in a wet cell where the person stands, the walking speed is the
 *      smaller of Table 1's speed for its class and that cap; the class stays
 *      Table 1's (or UNSTABLE by S4, speed 0); on dry cells and with the rule
 *      off Table 1 alone applies.
 */
#include "fps_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Riemann flux (R1).  F = (mass, normal momentum, tangential momentum).     */
/* ------------------------------------------------------------------------ */
void or_hllc(double g, double hL, double uL, double vL, double hR, double uR, double vR,
             double F[3])
{
    if (hL == 0.0 && hR == 0.0) {
        F[0] = F[1] = F[2] = 0.0;
        return;
    }
    double cL = sqrt(g * hL), cR = sqrt(g * hR);
    double sL, sR;
    if (hL == 0.0) {                     /* dry left bed */
        sL = uR - 2.0 * cR;
        sR = uR + cR;
    } else if (hR == 0.0) {              /* dry right bed */
        sL = uL - cL;
        sR = uL + 2.0 * cL;
    } else {
        double us = 0.5 * (uL + uR) + cL - cR;
        double cs = 0.5 * (cL + cR) + 0.25 * (uL - uR);
        sL = fmin(uL - cL, us - cs);
        sR = fmax(uR + cR, us + cs);
    }
    /* physical fluxes of the two states */
    double qL = hL * uL, qR = hR * uR;
    double FL0 = qL, FL1 = qL * uL + 0.5 * g * hL * hL, FL2 = qL * vL;
    double FR0 = qR, FR1 = qR * uR + 0.5 * g * hR * hR, FR2 = qR * vR;
    if (sL >= 0.0) {
        F[0] = FL0; F[1] = FL1; F[2] = FL2;
        return;
    }
    if (sR <= 0.0) {
        F[0] = FR0; F[1] = FR1; F[2] = FR2;
        return;
    }
    /* HLL star flux (sR FL - sL FR + sL sR (UR - UL)) / (sR - sL), anchored at FL */
    double inv = 1.0 / (sR - sL);
    F[0] = FL0 + sL * ((FL0 - FR0) + sR * (hR - hL)) * inv;
    F[1] = FL1 + sL * ((FL1 - FR1) + sR * (qR - qL)) * inv;
    /* contact speed; the tangential velocity is carried across it */
    double sM = (sL * hR * (uR - sR) - sR * hL * (uL - sL)) /
                (hR * (uR - sR) - hL * (uL - sL));
    F[2] = F[0] * (sM >= 0.0 ? vL : vR);
}

/* HLL for all three components: the same wave speeds as or_hllc and the
   same left-anchored form of (sR FL - sL FR + sL sR (UR - UL)) / (sR - sL),
   with U = (h, h un, h ut); mass and normal momentum equal or_hllc's exactly. */
void or_hll(double g, double hL, double uL, double vL, double hR, double uR, double vR,
            double F[3])
{
    if (hL == 0.0 && hR == 0.0) {
        F[0] = F[1] = F[2] = 0.0;
        return;
    }
    double cL = sqrt(g * hL), cR = sqrt(g * hR);
    double sL, sR;
    if (hL == 0.0) {
        sL = uR - 2.0 * cR;
        sR = uR + cR;
    } else if (hR == 0.0) {
        sL = uL - cL;
        sR = uL + 2.0 * cL;
    } else {
        double us = 0.5 * (uL + uR) + cL - cR;
        double cs = 0.5 * (cL + cR) + 0.25 * (uL - uR);
        sL = fmin(uL - cL, us - cs);
        sR = fmax(uR + cR, us + cs);
    }
    double qL = hL * uL, qR = hR * uR;
    double FL[3] = {qL, qL * uL + 0.5 * g * hL * hL, qL * vL};
    double FR[3] = {qR, qR * uR + 0.5 * g * hR * hR, qR * vR};
    double UL[3] = {hL, qL, hL * vL};
    double UR[3] = {hR, qR, hR * vR};
    for (int k = 0; k < 3; ++k) {
        if (sL >= 0.0) F[k] = FL[k];
        else if (sR <= 0.0) F[k] = FR[k];
        else F[k] = FL[k] + sL * ((FL[k] - FR[k]) + sR * (UR[k] - UL[k])) * (1.0 / (sR - sL));
    }
}

/* one face: hydrostatic reconstruction (R2) then the flux.  hsL/hsR return the
   reconstructed depths each side sees, used by the bed-slope correction. */
void or_face(const or_params *P, double hL, double qnL, double qtL, double zL,
             double hR, double qnR, double qtR, double zR, int wall, double F[3],
             double *hsL, double *hsR)
{
    double eps = P->h_dry;
    double zf = fmax(zL, zR);
    double hl = hL - (zf - zL);
    double hr = hR - (zf - zR);
    if (!(hl > eps)) hl = 0.0;
    if (!(hr > eps)) hr = 0.0;
    double unL = 0.0, utL = 0.0, unR = 0.0, utR = 0.0;
    if (hL > eps) { unL = qnL / hL; utL = qtL / hL; }
    if (hR > eps) { unR = qnR / hR; utR = qtR / hR; }
    if (P->flux == OR_FLUX_HLL) or_hll(P->g, hl, unL, utL, hr, unR, utR, F);
    else or_hllc(P->g, hl, unL, utL, hr, unR, utR, F);
    if (wall) {                          /* R8: a wall passes no mass */
        F[0] = 0.0;
        F[2] = 0.0;
    }
    *hsL = hl;
    *hsR = hr;
}

/* exact integral of the piecewise-linear hydrograph over [a, b] (R9) */
static double hydro_q(int32_t nh, const double *ht, const double *hq, double t)
{
    if (nh <= 0) return 0.0;
    if (t <= ht[0]) return hq[0];
    if (t >= ht[nh - 1]) return hq[nh - 1];
    for (int32_t k = 0; k + 1 < nh; ++k) {
        if (t >= ht[k] && t <= ht[k + 1]) {
            double w = (t - ht[k]) / (ht[k + 1] - ht[k]);
            return hq[k] + w * (hq[k + 1] - hq[k]);
        }
    }
    return hq[nh - 1];
}

double or_hydro_integral(int32_t nh, const double *ht, const double *hq, double a, double b)
{
    if (nh <= 0 || !(b > a)) return 0.0;
    /* split [a, b] at the breakpoints inside it; trapezoids are exact on lines */
    double total = 0.0, lo = a;
    for (int32_t k = 0; k < nh; ++k) {
        if (ht[k] > lo && ht[k] < b) {
            total += 0.5 * (hydro_q(nh, ht, hq, lo) + hydro_q(nh, ht, hq, ht[k])) * (ht[k] - lo);
            lo = ht[k];
        }
    }
    total += 0.5 * (hydro_q(nh, ht, hq, lo) + hydro_q(nh, ht, hq, b)) * (b - lo);
    return total;
}

/* ------------------------------------------------------------------------ */
/* Hazard rate and class (Table 1, sec. 2.4; R11, R12)                        */
/* ------------------------------------------------------------------------ */
int32_t or_hr_class(const or_params *P, double h, double qx, double qy, double *hr_out)
{
    if (!(h > P->h_dry)) {
        if (hr_out) *hr_out = 0.0;
        return OR_CLS_DRY;
    }
    double u = qx / h, v = qy / h;
    double V = fmax(fabs(u), fabs(v));
    double hr = (V + 0.5) * h;
    if (hr_out) *hr_out = hr;
    if (hr < P->hr_t[0]) return OR_CLS_LOW;
    if (hr < P->hr_t[1]) return OR_CLS_MEDIUM;
    if (hr < P->hr_t[2]) return OR_CLS_HIGH;
    return OR_CLS_HIGHEST;
}

/* Stability of a person standing in flowing water (S1-S4; the paper leaves
   richer rules than Table 1 to later work and names mechanics-based criteria):
   the body an upright cylinder of height H and volume M / rho_body, so of
   cross-section A = M / (rho_body H) and diameter b = 2 sqrt(A / pi); in water
   of depth h it loses rho_w g A h of its weight to buoyancy and meets the drag
   D = 1/2 rho_w c_drag b h u^2 of the flow speed u, acting at h / 2.  It
   slides when D exceeds mu_f times its effective weight W' and topples when
   the moment D h / 2 exceeds W' b / 2 (the cylinder tipping about its edge);
   it cannot stand once h >= H. */
int32_t or_unstable(const or_params *P, double h, double qx, double qy, double height, double mass,
                    double *margin)
{
    if (margin) *margin = 1.0;
    if (!(h > P->h_dry)) return 0;
    if (h >= height) {
        if (margin) *margin = -1.0;
        return 1;
    }
    const double pi = 3.14159265358979323846;
    double u = sqrt(qx * qx + qy * qy) / h;
    double area = mass / (P->rho_body * height);
    double b = 2.0 * sqrt(area / pi);
    double w_eff = P->g * (mass - P->rho_w * area * h);
    double drag = 0.5 * P->rho_w * P->c_drag * b * h * u * u;
    double hold_slide = P->mu_f * w_eff, hold_topple = w_eff * 0.5 * b;
    double push_topple = drag * 0.5 * h;
    if (margin) {
        double m1 = (hold_slide - drag) / hold_slide, m2 = (hold_topple - push_topple) / hold_topple;
        *margin = m1 < m2 ? m1 : m2;
    }
    return drag > hold_slide || push_topple > hold_topple;
}

/* Wading speed cap (W1, W2): the body of S2 (cross-section A = M / (rho_body
   H), frontal width b = 2 sqrt(A / pi)) wading through still water of depth
   h at speed v meets the drag 1/2 rho_w c_drag b h v^2; its feet keep up a
   push of wade_k W' with W' = g (M - rho_w A h); the cap is the speed at which
   the two are equal, 0 where W' <= 0. */
double or_wade_speed(const or_params *P, double h, double height, double mass)
{
    const double pi = 3.14159265358979323846;
    double area = mass / (P->rho_body * height);
    double b = 2.0 * sqrt(area / pi);
    double w_eff = P->g * (mass - P->rho_w * area * h);
    if (!(w_eff > 0.0)) return 0.0;
    return sqrt(2.0 * P->wade_k * w_eff / (P->rho_w * P->c_drag * b * h));
}

/* roughness write-back (sec. 2.4; R13) */
double or_n_eff(const or_params *P, int32_t np)
{
    int32_t k = np < P->np_cap ? np : P->np_cap;
    return P->n_base + (double)k * P->n_base;
}

/* Manning friction, splitting point-implicit (R5) */
void or_friction(const or_params *P, double dt, double h, double n, double *qx, double *qy)
{
    if (!(h > P->h_dry)) return;
    double u = *qx / h, v = *qy / h;
    double V2 = u * u + v * v;
    if (!(V2 > 0.0)) return;
    double speed = sqrt(V2);
    double Cf = P->g * n * n / cbrt(h);
    double Sx = -Cf * u * speed;
    double Sy = -Cf * v * speed;
    double Dx = 1.0 + dt * (Cf / h) * (2.0 * u * u + v * v) / speed;
    double Dy = 1.0 + dt * (Cf / h) * (2.0 * v * v + u * u) / speed;
    double dqx = dt * Sx / Dx;
    double dqy = dt * Sy / Dy;
    if (fabs(dqx) > fabs(*qx)) dqx = -*qx;
    if (fabs(dqy) > fabs(*qy)) dqy = -*qy;
    *qx += dqx;
    *qy += dqy;
}

/* ------------------------------------------------------------------------ */
/* Time step (sec. 3; R6)                                                     */
/* ------------------------------------------------------------------------ */
double or_compute_dt(const or_sim *S)
{
    const or_params *P = &S->P;
    int64_t nc = (int64_t)P->nx * P->ny;
    double lam = INFINITY;
    int any = 0;
#pragma omp parallel for schedule(static) reduction(min : lam) reduction(| : any)
    for (int64_t c = 0; c < nc; ++c) {
        double h = S->h[c];
        if (!(h > P->h_dry)) continue;
        double u = S->qx[c] / h, v = S->qy[c] / h;
        double cel = sqrt(P->g * h);
        double lx = P->dx / (fabs(u) + cel);
        double ly = P->dy / (fabs(v) + cel);
        lam = fmin(lam, fmin(lx, ly));
        any = 1;
    }
    if (!any) return P->dt_max;
    return fmin(P->cfl * lam, P->dt_max);
}

double or_mass(const or_sim *S)
{
    int64_t nc = (int64_t)S->P.nx * S->P.ny;
    double m = 0.0;
    for (int64_t c = 0; c < nc; ++c) m += S->h[c];
    return m * S->P.dx * S->P.dy;
}

/* ------------------------------------------------------------------------ */
/* Finite-volume update, Eq. (2) with R1-R9, R21                              */
/* ------------------------------------------------------------------------ */
/* the ghost of interior cell c across side s (R8) */
static void ghost(const or_sim *S, int32_t side, int64_t c, double *h, double *qx, double *qy,
                  double *z, int *wall)
{
    *h = S->h[c];
    *qx = S->qx[c];
    *qy = S->qy[c];
    *z = S->z[c];
    *wall = S->P.bc[side] == OR_WALL;
    if (*wall) {
        if (side <= 1) *qx = -*qx;       /* west / east: x is normal */
        else *qy = -*qy;                 /* south / north: y is normal */
    }
}

static void fv_step2(or_sim *S, double dt);

void or_fv_step(or_sim *S, double dt)
{
    if (S->P.order == 2) {
        fv_step2(S, dt);
        return;
    }
    const or_params *P = &S->P;
    const int32_t nx = P->nx, ny = P->ny;
    const double g = P->g, eps = P->h_dry;
    const int64_t nfx = (int64_t)(nx + 1) * ny, nfy = (int64_t)nx * (ny + 1);
    /* x faces: face f in row j lies between cells f-1 and f */
    double *FX = malloc(sizeof(double) * 3 * nfx), *HXL = malloc(sizeof(double) * nfx),
           *HXR = malloc(sizeof(double) * nfx);
    double *FY = malloc(sizeof(double) * 3 * nfy), *HYL = malloc(sizeof(double) * nfy),
           *HYR = malloc(sizeof(double) * nfy);
    double vout = 0.0;

#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; ++j) {
        for (int32_t f = 0; f <= nx; ++f) {
            double hL, qxL, qyL, zL, hR, qxR, qyR, zR;
            int wall = 0;
            if (f == 0) {
                int64_t c = (int64_t)j * nx;
                ghost(S, 0, c, &hL, &qxL, &qyL, &zL, &wall);
                hR = S->h[c]; qxR = S->qx[c]; qyR = S->qy[c]; zR = S->z[c];
            } else if (f == nx) {
                int64_t c = (int64_t)j * nx + nx - 1;
                hL = S->h[c]; qxL = S->qx[c]; qyL = S->qy[c]; zL = S->z[c];
                ghost(S, 1, c, &hR, &qxR, &qyR, &zR, &wall);
            } else {
                int64_t cl = (int64_t)j * nx + f - 1, cr = cl + 1;
                hL = S->h[cl]; qxL = S->qx[cl]; qyL = S->qy[cl]; zL = S->z[cl];
                hR = S->h[cr]; qxR = S->qx[cr]; qyR = S->qy[cr]; zR = S->z[cr];
            }
            int64_t k = (int64_t)j * (nx + 1) + f;
            or_face(P, hL, qxL, qyL, zL, hR, qxR, qyR, zR, wall, &FX[3 * k], &HXL[k], &HXR[k]);
        }
    }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j <= ny; ++j) {
        for (int32_t i = 0; i < nx; ++i) {
            double hL, qxL, qyL, zL, hR, qxR, qyR, zR;
            int wall = 0;
            if (j == 0) {
                int64_t c = i;
                ghost(S, 2, c, &hL, &qxL, &qyL, &zL, &wall);
                hR = S->h[c]; qxR = S->qx[c]; qyR = S->qy[c]; zR = S->z[c];
            } else if (j == ny) {
                int64_t c = (int64_t)(ny - 1) * nx + i;
                hL = S->h[c]; qxL = S->qx[c]; qyL = S->qy[c]; zL = S->z[c];
                ghost(S, 3, c, &hR, &qxR, &qyR, &zR, &wall);
            } else {
                int64_t cl = (int64_t)(j - 1) * nx + i, cr = cl + nx;
                hL = S->h[cl]; qxL = S->qx[cl]; qyL = S->qy[cl]; zL = S->z[cl];
                hR = S->h[cr]; qxR = S->qx[cr]; qyR = S->qy[cr]; zR = S->z[cr];
            }
            int64_t k = (int64_t)j * nx + i;
            /* y is normal: pass (qy, qx) as (normal, tangential) */
            or_face(P, hL, qyL, qxL, zL, hR, qyR, qxR, zR, wall, &FY[3 * k], &HYL[k], &HYR[k]);
        }
    }
    /* outflow through transmissive sides (outward positive) */
    if (P->bc[0] == OR_TRANSMISSIVE)
        for (int32_t j = 0; j < ny; ++j) vout -= FX[3 * ((int64_t)j * (nx + 1))] * P->dy;
    if (P->bc[1] == OR_TRANSMISSIVE)
        for (int32_t j = 0; j < ny; ++j) vout += FX[3 * ((int64_t)j * (nx + 1) + nx)] * P->dy;
    if (P->bc[2] == OR_TRANSMISSIVE)
        for (int32_t i = 0; i < nx; ++i) vout -= FY[3 * (int64_t)i] * P->dx;
    if (P->bc[3] == OR_TRANSMISSIVE)
        for (int32_t i = 0; i < nx; ++i) vout += FY[3 * ((int64_t)ny * nx + i)] * P->dx;
    S->v_out += vout * dt;

    /* inflow depth for this step (R9) */
    double inc = 0.0;
    if (P->inflow_side >= 0) {
        double dn = P->inflow_side <= 1 ? P->dx : P->dy;
        inc = or_hydro_integral(S->nh, S->ht, S->hq, S->t, S->t + dt) / dn;
    }

    const double lx = dt / P->dx, ly = dt / P->dy;
    /* inflow and clipped volumes: one partial per row, added in row order below,
       so any number of threads gives the same sums */
    double *row_in = calloc((size_t)ny, sizeof(double)), *row_clip = calloc((size_t)ny, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; ++j) {
        for (int32_t i = 0; i < nx; ++i) {
            int64_t c = (int64_t)j * nx + i;
            int64_t kW = (int64_t)j * (nx + 1) + i, kE = kW + 1;
            int64_t kS = c, kN = c + nx;
            const double *fW = &FX[3 * kW], *fE = &FX[3 * kE];
            const double *fS = &FY[3 * kS], *fN = &FY[3 * kN];
            /* this cell's own reconstructed depths at its four faces */
            double hsW = HXR[kW], hsE = HXL[kE], hsS = HYR[kS], hsN = HYL[kN];
            double pW = 0.5 * g * hsW * hsW, pE = 0.5 * g * hsE * hsE;
            double pS = 0.5 * g * hsS * hsS, pN = 0.5 * g * hsN * hsN;
            /* Eq. (2): mass */
            double ax_h = lx * (fE[0] - fW[0]);
            double ay_h = ly * (fN[0] - fS[0]);
            double hn = S->h[c] - (ax_h + ay_h);
            /* x momentum: normal on x faces (with bed-slope correction), tangential on y faces */
            double ax_qx = lx * ((fE[1] - pE) - (fW[1] - pW));
            double ay_qx = ly * (fN[2] - fS[2]);
            double qxn = S->qx[c] - (ax_qx + ay_qx);
            /* y momentum */
            double ay_qy = ly * ((fN[1] - pN) - (fS[1] - pS));
            double ax_qy = lx * (fE[2] - fW[2]);
            double qyn = S->qy[c] - (ay_qy + ax_qy);
            /* inflow line source */
            if (P->inflow_side >= 0) {
                int32_t along = -1;
                if (P->inflow_side == 0 && i == 0) along = j;
                if (P->inflow_side == 1 && i == nx - 1) along = j;
                if (P->inflow_side == 2 && j == 0) along = i;
                if (P->inflow_side == 3 && j == ny - 1) along = i;
                if (along >= P->inflow_c0 && along < P->inflow_c1) {
                    hn += inc;
                    row_in[j] += inc * P->dx * P->dy;
                }
            }
            /* cleanup (R21) */
            if (hn < 0.0) {
                row_clip[j] += -hn * P->dx * P->dy;
                hn = 0.0;
            }
            if (!(hn > eps)) {
                qxn = 0.0;
                qyn = 0.0;
            }
            /* friction with the effective roughness (R5, R13) */
            or_friction(P, dt, hn, or_n_eff(P, S->np[c]), &qxn, &qyn);
            /* in place is safe: every face was computed before this loop */
            S->h[c] = hn;
            S->qx[c] = qxn;
            S->qy[c] = qyn;
        }
    }
    for (int32_t j = 0; j < ny; ++j) {
        S->v_in += row_in[j];
        S->v_clip += row_clip[j];
    }
    free(row_in);
    free(row_clip);
    int wet = 0;
    int64_t nc = (int64_t)nx * ny;
    for (int64_t c = 0; c < nc; ++c)
        if (S->h[c] > eps) { wet = 1; break; }
    S->any_wet = wet;
    free(FX); free(HXL); free(HXR);
    free(FY); free(HYL); free(HYR);
}

/* ------------------------------------------------------------------------ */
/* Second-order variant.  The paper took the scheme of Wang et al. (2011) and  */
/* reduced it to first order (sec. 2.2); this variant puts the second order    */
/* back.  Readings (the scheme's equations are not in the paper):              */
/*   M1 MUSCL reconstruction, per direction, of h, eta = h + z, u and v with    */
/*      the minmod limiter; a cell's slope is zero where it or either          */
/*      neighbour in that direction is dry (h <= h_dry), so the scheme is first */
/*      order at wet/dry fronts, and in ghost cells; the face bed is            */
/*      z = eta - h of the reconstructed values.                               */
/*   M2 at each face the hydrostatic reconstruction (R2) of the two             */
/*      reconstructed states, then HLLC or HLL (R1) with the reconstructed      */
/*      velocities (limited between the neighbours' velocities, so a thin face  */
/*      depth cannot make them large; 0 where the face depth <= h_dry).         */
/*   M3 bed slope in the second-order form of Audusse et al. (2004): a cell's  */
/*      normal momentum gets g/2 (h_f^2 - h*_f^2) at each of its faces (h_f its */
/*      reconstructed depth there, h*_f the hydrostatic one) and the centred   */
/*      term -g/2 (h_w + h_e)(z_e - z_w) per direction; a lake at rest stays    */
/*      at rest exactly.                                                        */
/*   M4 time: Heun's two-stage Runge-Kutta, U1 = U + dt L(U), U' = (U + U1 +    */
/*      dt L(U1)) / 2, depth cleanup (R21) after each stage; inflow (R9) and   */
/*      friction (R5) once after both stages; outflow and clipped volumes are  */
/*      the means of the two stages'.                                          */
/* ------------------------------------------------------------------------ */
double or_minmod(double a, double b)
{
    if (!(a * b > 0.0)) return 0.0;
    return fabs(a) <= fabs(b) ? a : b;
}

/* cell (i, j) with one ghost layer: i in [-1, nx], j in [-1, ny] (not both
   outside); v = (h, eta, u, v) with the velocities of R2 (0 where h <= h_dry);
   *ghost set for ghost cells (R8) */
static void cell2(const or_params *P, const double *h, const double *qx, const double *qy, const double *z,
                  int32_t i, int32_t j, double v[4], int *ghost)
{
    int32_t ii = i < 0 ? 0 : (i >= P->nx ? P->nx - 1 : i);
    int32_t jj = j < 0 ? 0 : (j >= P->ny ? P->ny - 1 : j);
    int64_t c = (int64_t)jj * P->nx + ii;
    double hh = h[c], ux = qx[c], uy = qy[c];
    *ghost = i != ii || j != jj;
    if (i < 0 && P->bc[0] == OR_WALL) ux = -ux;
    if (i >= P->nx && P->bc[1] == OR_WALL) ux = -ux;
    if (j < 0 && P->bc[2] == OR_WALL) uy = -uy;
    if (j >= P->ny && P->bc[3] == OR_WALL) uy = -uy;
    v[0] = hh;
    v[1] = hh + z[c];
    v[2] = hh > P->h_dry ? ux / hh : 0.0;
    v[3] = hh > P->h_dry ? uy / hh : 0.0;
}

/* limited slopes of cell (i, j) in direction dir (0: x, 1: y) (M1) */
static void slopes2(const or_params *P, const double *h, const double *qx, const double *qy, const double *z,
                    int32_t i, int32_t j, int dir, double s[4])
{
    double a[4], b[4], c[4];
    int ga, gb, gc;
    cell2(P, h, qx, qy, z, i, j, b, &gb);
    for (int k = 0; k < 4; ++k) s[k] = 0.0;
    if (gb) return;
    if (dir == 0) {
        cell2(P, h, qx, qy, z, i - 1, j, a, &ga);
        cell2(P, h, qx, qy, z, i + 1, j, c, &gc);
    } else {
        cell2(P, h, qx, qy, z, i, j - 1, a, &ga);
        cell2(P, h, qx, qy, z, i, j + 1, c, &gc);
    }
    if (!(a[0] > P->h_dry) || !(b[0] > P->h_dry) || !(c[0] > P->h_dry)) return;
    for (int k = 0; k < 4; ++k) s[k] = or_minmod(c[k] - b[k], b[k] - a[k]);
}

/* reconstructed state of cell (i, j) at its face on side sgn (+1: east /
   north, -1: west / south) in direction dir: (h, eta, u, v) */
static void face_state2(const or_params *P, const double *h, const double *qx, const double *qy,
                        const double *z, int32_t i, int32_t j, int dir, double sgn, double v[4])
{
    double s[4];
    int g;
    cell2(P, h, qx, qy, z, i, j, v, &g);
    slopes2(P, h, qx, qy, z, i, j, dir, s);
    for (int k = 0; k < 4; ++k) v[k] += 0.5 * sgn * s[k];
}

/* one face between the reconstructed states L and R (h, eta, un, ut) in the
   face's normal direction (M2).  hf / hs: each side's reconstructed and
   hydrostatic depths; zf: each side's face bed. */
static void face2(const or_params *P, const double L[4], const double R[4], int wall, double F[3],
                  double hf[2], double hs[2], double zfc[2])
{
    double eps = P->h_dry;
    double zL = L[1] - L[0], zR = R[1] - R[0];
    double zf = fmax(zL, zR);
    double hl = L[0] - (zf - zL), hr = R[0] - (zf - zR);
    if (!(hl > eps)) hl = 0.0;
    if (!(hr > eps)) hr = 0.0;
    double unL = 0.0, utL = 0.0, unR = 0.0, utR = 0.0;
    if (L[0] > eps) { unL = L[2]; utL = L[3]; }
    if (R[0] > eps) { unR = R[2]; utR = R[3]; }
    if (P->flux == OR_FLUX_HLL) or_hll(P->g, hl, unL, utL, hr, unR, utR, F);
    else or_hllc(P->g, hl, unL, utL, hr, unR, utR, F);
    if (wall) {
        F[0] = 0.0;
        F[2] = 0.0;
    }
    hf[0] = L[0];
    hf[1] = R[0];
    hs[0] = hl;
    hs[1] = hr;
    zfc[0] = zL;
    zfc[1] = zR;
}

/* dU = -L(U) dt-free residual times dt/d: rh, rqx, rqy[nc] get the change of
   one forward-Euler stage of length dt; out gets the outflow volume rate */
static void stage2(const or_sim *S, const double *h, const double *qx, const double *qy, double dt,
                   double *dh, double *dqx, double *dqy, double *vout_rate)
{
    const or_params *P = &S->P;
    const int32_t nx = P->nx, ny = P->ny;
    const double g = P->g;
    const int64_t nfx = (int64_t)(nx + 1) * ny, nfy = (int64_t)nx * (ny + 1);
    /* per face: flux, and for each side (0: west/south cell, 1: east/north
       cell) the reconstructed depth, hydrostatic depth and face bed */
    double *FX = malloc(sizeof(double) * 3 * nfx), *AX = malloc(sizeof(double) * 6 * nfx);
    double *FY = malloc(sizeof(double) * 3 * nfy), *AY = malloc(sizeof(double) * 6 * nfy);
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; ++j) {
        for (int32_t f = 0; f <= nx; ++f) {
            double L[4], R[4], hf[2], hs[2], zc[2];
            face_state2(P, h, qx, qy, S->z, f - 1, j, 0, 1.0, L);
            face_state2(P, h, qx, qy, S->z, f, j, 0, -1.0, R);
            int wall = (f == 0 && P->bc[0] == OR_WALL) || (f == nx && P->bc[1] == OR_WALL);
            int64_t k = (int64_t)j * (nx + 1) + f;
            face2(P, L, R, wall, &FX[3 * k], hf, hs, zc);
            for (int q = 0; q < 2; ++q) {
                AX[6 * k + q] = hf[q];
                AX[6 * k + 2 + q] = hs[q];
                AX[6 * k + 4 + q] = zc[q];
            }
        }
    }
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j <= ny; ++j) {
        for (int32_t i = 0; i < nx; ++i) {
            double L[4], R[4], Ly[4], Ry[4], hf[2], hs[2], zc[2];
            face_state2(P, h, qx, qy, S->z, i, j - 1, 1, 1.0, L);
            face_state2(P, h, qx, qy, S->z, i, j, 1, -1.0, R);
            /* y is normal: (h, eta, v, u) */
            Ly[0] = L[0]; Ly[1] = L[1]; Ly[2] = L[3]; Ly[3] = L[2];
            Ry[0] = R[0]; Ry[1] = R[1]; Ry[2] = R[3]; Ry[3] = R[2];
            int wall = (j == 0 && P->bc[2] == OR_WALL) || (j == ny && P->bc[3] == OR_WALL);
            int64_t k = (int64_t)j * nx + i;
            face2(P, Ly, Ry, wall, &FY[3 * k], hf, hs, zc);
            for (int q = 0; q < 2; ++q) {
                AY[6 * k + q] = hf[q];
                AY[6 * k + 2 + q] = hs[q];
                AY[6 * k + 4 + q] = zc[q];
            }
        }
    }
    double vout = 0.0;
    if (P->bc[0] == OR_TRANSMISSIVE)
        for (int32_t j = 0; j < ny; ++j) vout -= FX[3 * ((int64_t)j * (nx + 1))] * P->dy;
    if (P->bc[1] == OR_TRANSMISSIVE)
        for (int32_t j = 0; j < ny; ++j) vout += FX[3 * ((int64_t)j * (nx + 1) + nx)] * P->dy;
    if (P->bc[2] == OR_TRANSMISSIVE)
        for (int32_t i = 0; i < nx; ++i) vout -= FY[3 * (int64_t)i] * P->dx;
    if (P->bc[3] == OR_TRANSMISSIVE)
        for (int32_t i = 0; i < nx; ++i) vout += FY[3 * ((int64_t)ny * nx + i)] * P->dx;
    *vout_rate = vout;
    const double lx = dt / P->dx, ly = dt / P->dy;
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < ny; ++j) {
        for (int32_t i = 0; i < nx; ++i) {
            int64_t c = (int64_t)j * nx + i;
            int64_t kW = (int64_t)j * (nx + 1) + i, kE = kW + 1, kS = c, kN = c + nx;
            const double *fW = &FX[3 * kW], *fE = &FX[3 * kE], *fS = &FY[3 * kS], *fN = &FY[3 * kN];
            /* this cell is side 1 of its west / south face, side 0 of its east / north face */
            double hw = AX[6 * kW + 1], hsw = AX[6 * kW + 3], zw = AX[6 * kW + 5];
            double he = AX[6 * kE + 0], hse = AX[6 * kE + 2], ze = AX[6 * kE + 4];
            double hS = AY[6 * kS + 1], hsS = AY[6 * kS + 3], zS = AY[6 * kS + 5];
            double hN = AY[6 * kN + 0], hsN = AY[6 * kN + 2], zN = AY[6 * kN + 4];
            /* M3: one-sided corrections and the centred bed-slope term */
            double cx = 0.5 * g * (he * he - hse * hse) - 0.5 * g * (hw * hw - hsw * hsw) +
                        0.5 * g * (hw + he) * (ze - zw);
            double cy = 0.5 * g * (hN * hN - hsN * hsN) - 0.5 * g * (hS * hS - hsS * hsS) +
                        0.5 * g * (hS + hN) * (zN - zS);
            dh[c] = -(lx * (fE[0] - fW[0]) + ly * (fN[0] - fS[0]));
            dqx[c] = -(lx * ((fE[1] - fW[1]) + cx) + ly * (fN[2] - fS[2]));
            dqy[c] = -(ly * ((fN[1] - fS[1]) + cy) + lx * (fE[2] - fW[2]));
        }
    }
    free(FX); free(AX); free(FY); free(AY);
}

static void fv_step2(or_sim *S, double dt)
{
    const or_params *P = &S->P;
    const int32_t nx = P->nx, ny = P->ny;
    const int64_t nc = (int64_t)nx * ny;
    const double eps = P->h_dry;
    double *h1 = malloc(sizeof(double) * nc), *qx1 = malloc(sizeof(double) * nc), *qy1 = malloc(sizeof(double) * nc);
    double *dh = malloc(sizeof(double) * nc), *dqx = malloc(sizeof(double) * nc), *dqy = malloc(sizeof(double) * nc);
    double rate0 = 0.0, rate1 = 0.0, clip = 0.0;
    /* stage 1: U1 = U + dt L(U) */
    stage2(S, S->h, S->qx, S->qy, dt, dh, dqx, dqy, &rate0);
    for (int64_t c = 0; c < nc; ++c) {
        double hh = S->h[c] + dh[c], a = S->qx[c] + dqx[c], b = S->qy[c] + dqy[c];
        if (hh < 0.0) { clip += 0.5 * -hh; hh = 0.0; }
        if (!(hh > eps)) { a = 0.0; b = 0.0; }
        h1[c] = hh; qx1[c] = a; qy1[c] = b;
    }
    /* stage 2: U' = (U + U1 + dt L(U1)) / 2 */
    stage2(S, h1, qx1, qy1, dt, dh, dqx, dqy, &rate1);
    double inc = 0.0;
    if (P->inflow_side >= 0) {
        double dn = P->inflow_side <= 1 ? P->dx : P->dy;
        inc = or_hydro_integral(S->nh, S->ht, S->hq, S->t, S->t + dt) / dn;
    }
    double vin = 0.0;
    for (int32_t j = 0; j < ny; ++j) {
        for (int32_t i = 0; i < nx; ++i) {
            int64_t c = (int64_t)j * nx + i;
            double h2 = h1[c] + dh[c], a2 = qx1[c] + dqx[c], b2 = qy1[c] + dqy[c];
            if (h2 < 0.0) { clip += 0.5 * -h2; h2 = 0.0; }
            if (!(h2 > eps)) { a2 = 0.0; b2 = 0.0; }
            double hn = 0.5 * (S->h[c] + h2), qxn = 0.5 * (S->qx[c] + a2), qyn = 0.5 * (S->qy[c] + b2);
            if (P->inflow_side >= 0) {
                int32_t along = -1;
                if (P->inflow_side == 0 && i == 0) along = j;
                if (P->inflow_side == 1 && i == nx - 1) along = j;
                if (P->inflow_side == 2 && j == 0) along = i;
                if (P->inflow_side == 3 && j == ny - 1) along = i;
                if (along >= P->inflow_c0 && along < P->inflow_c1) {
                    hn += inc;
                    vin += inc * P->dx * P->dy;
                }
            }
            if (!(hn > eps)) { qxn = 0.0; qyn = 0.0; }
            or_friction(P, dt, hn, or_n_eff(P, S->np[c]), &qxn, &qyn);
            S->h[c] = hn;
            S->qx[c] = qxn;
            S->qy[c] = qyn;
        }
    }
    S->v_in += vin;
    S->v_out += 0.5 * (rate0 + rate1) * dt;
    S->v_clip += clip * P->dx * P->dy;
    int wet = 0;
    for (int64_t c = 0; c < nc; ++c)
        if (S->h[c] > eps) { wet = 1; break; }
    S->any_wet = wet;
    free(h1); free(qx1); free(qy1); free(dh); free(dqx); free(dqy);
}

/* ------------------------------------------------------------------------ */
/* Pedestrians                                                                */
/* ------------------------------------------------------------------------ */
int32_t or_cell_index(double x, double d, int32_t n)
{
    /* R19: decided in FP32; the result may lie outside [0, n) */
    float q = (float)x / (float)d;
    float f = floorf(q);
    if (f < -1.0f) return -1;
    if (f > (float)n) return n;
    return (int32_t)f;
}

static int32_t clampi(int32_t v, int32_t lo, int32_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

void or_bins_dims(const or_params *P, int32_t *bsx, int32_t *bsy, int32_t *nbx, int32_t *nby)
{
    /* bin side: whole cells, at least r_cut long */
    int32_t bx = (int32_t)ceil(P->r_cut / P->dx - 1e-9), by = (int32_t)ceil(P->r_cut / P->dy - 1e-9);
    if (bx < 1) bx = 1;
    if (by < 1) by = 1;
    *bsx = bx;
    *bsy = by;
    *nbx = (P->nx + bx - 1) / bx;
    *nby = (P->ny + by - 1) / by;
}

/* stable counting sort of the non-exited agents by bin (ascending agent id inside a bin) */
void or_build_bins(const or_params *P, int32_t na, const float *x, const float *y,
                   const uint8_t *state, int32_t *bin_start, int32_t *perm)
{
    int32_t bsx, bsy, nbx, nby;
    or_bins_dims(P, &bsx, &bsy, &nbx, &nby);
    int32_t nb = nbx * nby;
    for (int32_t b = 0; b <= nb; ++b) bin_start[b] = 0;
    int32_t *key = malloc(sizeof(int32_t) * (na > 0 ? na : 1));
    for (int32_t a = 0; a < na; ++a) {
        key[a] = -1;
        if (state[a] == OR_ST_EXITED || state[a] == OR_ST_OUTSIDE) continue;
        int32_t ci = clampi(or_cell_index(x[a], P->dx, P->nx), 0, P->nx - 1);
        int32_t cj = clampi(or_cell_index(y[a], P->dy, P->ny), 0, P->ny - 1);
        key[a] = (cj / bsy) * nbx + ci / bsx;
        bin_start[key[a] + 1] += 1;
    }
    for (int32_t b = 0; b < nb; ++b) bin_start[b + 1] += bin_start[b];
    int32_t *cur = malloc(sizeof(int32_t) * (nb > 0 ? nb : 1));
    for (int32_t b = 0; b < nb; ++b) cur[b] = bin_start[b];
    for (int32_t a = 0; a < na; ++a)      /* ascending id keeps the sort stable */
        if (key[a] >= 0) perm[cur[key[a]]++] = a;
    free(cur);
    free(key);
}

void or_count_evacuees(or_sim *S)
{
    const or_params *P = &S->P;
    int64_t nc = (int64_t)P->nx * P->ny;
    for (int64_t c = 0; c < nc; ++c) S->np[c] = 0;
    for (int32_t a = 0; a < S->na; ++a) {
        if (S->role[a] != OR_ROLE_EVACUEE || S->state[a] != OR_ST_EVAC) continue;
        int32_t ci = clampi(or_cell_index(S->x[a], P->dx, P->nx), 0, P->nx - 1);
        int32_t cj = clampi(or_cell_index(S->y[a], P->dy, P->ny), 0, P->ny - 1);
        S->np[(int64_t)cj * P->nx + ci] += 1;
    }
}

static float dist_at(const or_sim *S, int32_t d, int32_t i, int32_t j)
{
    return S->dist[((int64_t)d * S->P.ny + j) * S->P.nx + i];
}

static int32_t nearest_exit(const or_sim *S, int32_t ci, int32_t cj)
{
    int32_t best = 0;
    for (int32_t e = 1; e < S->n_exit; ++e)
        if (dist_at(S, e, ci, cj) < dist_at(S, best, ci, cj)) best = e;
    return best;
}

/* desired direction (R14) */
static void direction(const or_sim *S, int32_t d, int32_t ci, int32_t cj, double x, double y,
                      double *ex, double *ey)
{
    static const int32_t off[8][2] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1},
                                      {1, 1}, {-1, 1}, {-1, -1}, {1, -1}};
    const or_params *P = &S->P;
    *ex = 0.0;
    *ey = 0.0;
    float here = dist_at(S, d, ci, cj);
    int32_t ti = ci, tj = cj;
    if (!(here == 0.0f)) {
        float best = here;
        int32_t k_best = -1;
        for (int32_t k = 0; k < 8; ++k) {
            int32_t ni = ci + off[k][0], nj = cj + off[k][1];
            if (ni < 0 || nj < 0 || ni >= P->nx || nj >= P->ny) continue;
            float dk = dist_at(S, d, ni, nj);
            if (dk < best) {
                best = dk;
                k_best = k;
            }
        }
        if (k_best < 0) return;
        ti = ci + off[k_best][0];
        tj = cj + off[k_best][1];
    }
    double tx = (ti + 0.5) * P->dx - x, ty = (tj + 0.5) * P->dy - y;
    double len = sqrt(tx * tx + ty * ty);
    if (len > 0.0) {
        *ex = tx / len;
        *ey = ty / len;
    }
}

void or_ped_step(or_sim *S, double dt)
{
    const or_params *P = &S->P;
    const int32_t na = S->na, nx = P->nx, ny = P->ny;
    if (na <= 0) return;
    int32_t bsx, bsy, nbx, nby;
    or_bins_dims(P, &bsx, &bsy, &nbx, &nby);
    /* cell lists of the positions at the start of the step */
    float *xf = malloc(sizeof(float) * na), *yf = malloc(sizeof(float) * na);
    for (int32_t a = 0; a < na; ++a) {
        xf[a] = (float)S->x[a];
        yf[a] = (float)S->y[a];
    }
    or_build_bins(P, na, xf, yf, S->state, S->bin_start, S->perm);
    double *x1 = malloc(sizeof(double) * na), *y1 = malloc(sizeof(double) * na);
    double *vx1 = malloc(sizeof(double) * na), *vy1 = malloc(sizeof(double) * na);
    const int32_t Rx = (int32_t)ceil(P->r_cut / P->dx - 1e-9), Ry = (int32_t)ceil(P->r_cut / P->dy - 1e-9);
    int32_t drops = 0, leaves = 0;

    /* every agent reads the start-of-step state and writes only its own record */
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : drops, leaves)
    for (int32_t a = 0; a < na; ++a) {
        double x = S->x[a], y = S->y[a];
        x1[a] = x; y1[a] = y; vx1[a] = S->vx[a]; vy1[a] = S->vy[a];
        int32_t st = S->state[a];
        if (st == OR_ST_EXITED || st == OR_ST_OUTSIDE) continue;
        int32_t ci = clampi(or_cell_index(x, P->dx, nx), 0, nx - 1);
        int32_t cj = clampi(or_cell_index(y, P->dy, ny), 0, ny - 1);
        int64_t c = (int64_t)cj * nx + ci;
        /* hazard from the containing cell (Table 1) */
        int32_t cls = or_hr_class(P, S->h[c], S->qx[c], S->qy[c], NULL);
        double v0 = cls == OR_CLS_DRY ? S->vbase[a] : P->v_class[cls];
        /* the stability rule overrides Table 1 where a person cannot stand (S4) */
        if (P->stability && cls != OR_CLS_DRY) {
            double hb = S->body_h ? S->body_h[a] : P->body_h0, mb = S->body_m ? S->body_m[a] : P->body_m0;
            if (or_unstable(P, S->h[c], S->qx[c], S->qy[c], hb, mb, NULL)) {
                cls = OR_CLS_UNSTABLE;
                v0 = 0.0;
            }
        }
        /* the wading rule caps the speed of a person standing in water (W3) */
        if (P->wading && cls != OR_CLS_DRY && cls != OR_CLS_UNSTABLE) {
            double hb = S->body_h ? S->body_h[a] : P->body_h0, mb = S->body_m ? S->body_m[a] : P->body_m0;
            double vw = or_wade_speed(P, S->h[c], hb, mb);
            if (vw < v0) v0 = vw;
        }
        S->cls[a] = (uint8_t)cls;
        /* destinations */
        if (S->dest[a] < 0) {
            if (S->role[a] == OR_ROLE_EVACUEE) {
                S->dest[a] = nearest_exit(S, ci, cj);
                st = OR_ST_EVAC;
            } else {
                S->dest[a] = S->storage_dest;
                st = OR_ST_TO_STORAGE;
            }
        }
        if (S->role[a] == OR_ROLE_RESPONDER && S->done && st != OR_ST_EVAC) {
            st = OR_ST_EVAC;
            S->dest[a] = nearest_exit(S, ci, cj);
        }
        /* water on the site: walkers of the door flow become evacuees (D4) */
        if (st == OR_ST_SHOPPING && S->any_wet) {
            st = OR_ST_EVAC;
            S->dest[a] = nearest_exit(S, ci, cj);
        }
        /* responder waits (sec. 2.4) */
        if (st == OR_ST_PICKING || st == OR_ST_DROPPING) {
            S->timer[a] -= dt;
            if (S->timer[a] > 0.0) {
                vx1[a] = 0.0; vy1[a] = 0.0;
                S->state[a] = (uint8_t)st;
                continue;
            }
            if (st == OR_ST_PICKING) {
                st = OR_ST_TO_BARRIER;
                S->dest[a] = S->barrier_dest;
            } else {
                drops += 1;
                st = OR_ST_TO_STORAGE;
                S->dest[a] = S->storage_dest;
            }
        }
        /* evacuation trigger (R17); an agent without a destination stands */
        if ((S->role[a] == OR_ROLE_EVACUEE && st == OR_ST_EVAC && !S->any_wet) || S->dest[a] < 0 ||
            S->dest[a] >= S->n_dest) {
            vx1[a] = 0.0; vy1[a] = 0.0;
            S->state[a] = (uint8_t)st;
            continue;
        }
        /* social force (R15) */
        double ex, ey;
        direction(S, S->dest[a], ci, cj, x, y, &ex, &ey);
        double k = exp(-dt / P->tau);
        double vx = v0 * ex + (S->vx[a] - v0 * ex) * k;
        double vy = v0 * ey + (S->vy[a] - v0 * ey) * k;
        double fx = 0.0, fy = 0.0;
        int32_t bi = ci / bsx, bj = cj / bsy;
        for (int32_t qj = bj - 1; qj <= bj + 1; ++qj) {
            if (qj < 0 || qj >= nby) continue;
            for (int32_t qi = bi - 1; qi <= bi + 1; ++qi) {
                if (qi < 0 || qi >= nbx) continue;
                int32_t b = qj * nbx + qi;
                for (int32_t s = S->bin_start[b]; s < S->bin_start[b + 1]; ++s) {
                    int32_t o = S->perm[s];
                    if (o == a) continue;
                    double rx = x - S->x[o], ry = y - S->y[o];
                    double d = sqrt(rx * rx + ry * ry);
                    if (!(d > 0.0) || !(d < P->r_cut)) continue;
                    double w = P->a_over_m * exp((2.0 * P->radius - d) / P->b_range);
                    fx += w * rx / d;
                    fy += w * ry / d;
                }
            }
        }
        for (int32_t dj = -Ry; dj <= Ry; ++dj) {
            int32_t wj = cj + dj;
            if (wj < 0 || wj >= ny) continue;
            for (int32_t di = -Rx; di <= Rx; ++di) {
                int32_t wi = ci + di;
                if (wi < 0 || wi >= nx) continue;
                if (S->walk[(int64_t)wj * nx + wi]) continue;
                double px = fmin(fmax(x, wi * P->dx), (wi + 1) * P->dx);
                double py = fmin(fmax(y, wj * P->dy), (wj + 1) * P->dy);
                double rx = x - px, ry = y - py;
                double d = sqrt(rx * rx + ry * ry);
                if (!(d > 0.0) || !(d < P->r_cut)) continue;
                double w = P->a_over_m * exp((P->radius - d) / P->b_range);
                fx += w * rx / d;
                fy += w * ry / d;
            }
        }
        vx += dt * fx;
        vy += dt * fy;
        double sp = sqrt(vx * vx + vy * vy);
        if (sp > v0) {
            if (v0 > 0.0) {
                vx *= v0 / sp;
                vy *= v0 / sp;
            } else {
                vx = 0.0;
                vy = 0.0;
            }
        }
        /* move with axis-wise rejection (R15) */
        double xn = x + dt * vx;
        int32_t ni = or_cell_index(xn, P->dx, nx);
        if (ni < 0 || ni >= nx || !S->walk[(int64_t)cj * nx + ni]) {
            xn = x;
            vx = 0.0;
            ni = ci;
        }
        double yn = y + dt * vy;
        int32_t nj = or_cell_index(yn, P->dy, ny);
        if (nj < 0 || nj >= ny || !S->walk[(int64_t)nj * nx + ni]) {
            yn = y;
            vy = 0.0;
            nj = cj;
        }
        /* arrival (R16) */
        if (dist_at(S, S->dest[a], ni, nj) <= (float)P->r_arrive) {
            if (st == OR_ST_EVAC) {
                st = OR_ST_EXITED;
            } else if (st == OR_ST_TO_STORAGE) {
                st = OR_ST_PICKING;
                S->timer[a] = P->pick_s;
                vx = 0.0; vy = 0.0;
            } else if (st == OR_ST_TO_BARRIER) {
                st = OR_ST_DROPPING;
                S->timer[a] = P->drop_s;
                vx = 0.0; vy = 0.0;
            } else if (st == OR_ST_SHOPPING) {
                st = OR_ST_OUTSIDE;      /* left by its door (D3) */
                leaves += 1;
            }
        }
        x1[a] = xn; y1[a] = yn; vx1[a] = vx; vy1[a] = vy;
        S->state[a] = (uint8_t)st;
    }
    for (int32_t a = 0; a < na; ++a) {
        S->x[a] = x1[a]; S->y[a] = y1[a]; S->vx[a] = vx1[a]; S->vy[a] = vy1[a];
    }
    S->door_out += leaves;
    or_doors(S);
    /* barrier fill (R18) */
    S->drops_total += drops;
    if (!S->done && S->nline > 0) {
        S->bags += drops;
        while (!S->done && S->bags >= S->bags_per) {
            S->bags -= S->bags_per;
            double th = S->layers_done == S->n_layers - 1 ? S->t_last : S->t_bag;
            S->z[S->line[S->active]] += th;
            S->active += 1;
            if (S->active == S->nline) {
                S->active = 0;
                S->layers_done += 1;
                if (S->layers_done >= S->n_layers) S->done = 1;
            }
        }
    }
    free(xf); free(yf); free(x1); free(y1); free(vx1); free(vy1);
}

/* ------------------------------------------------------------------------ */
/* Pre-flood door flow (sec. 3, sec. 3.2; D1-D6)                              */
/* ------------------------------------------------------------------------ */
uint64_t or_splitmix64(uint64_t seed, uint64_t c)
{
    /* the generator's state after c + 1 steps of the golden-ratio gamma, then
       its output mix (D6) */
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static uint64_t door_draw(const or_sim *S, int32_t a, int32_t k)
{
    uint64_t c = ((uint64_t)S->step << 26) | ((uint64_t)a << 2) | (uint64_t)k;
    return or_splitmix64(S->door_seed, c);
}

static int32_t choice_of(uint64_t u, int32_t m) { return (int32_t)(((u >> 32) * (uint64_t)m) >> 32); }

static float offset_of(uint64_t u) { return 0.25f + 0.5f * ((float)(u >> 40) * (1.0f / 16777216.0f)); }

void or_doors(or_sim *S)
{
    const or_params *P = &S->P;
    if (S->n_door <= 0 || S->doors_closed) return;
    if (S->any_wet) {
        S->doors_closed = 1;
        return;
    }
    int32_t taken[OR_MAX_DOOR] = {0};
    for (int32_t a = 0; a < S->na; ++a) {
        if (S->state[a] != OR_ST_OUTSIDE) continue;
        int32_t d = choice_of(door_draw(S, a, 0), S->n_door);
        if (taken[d] >= S->door_rate) continue;
        taken[d] += 1;
        int32_t j = choice_of(door_draw(S, a, 1), S->n_door - 1);
        int32_t leave = j < d ? j : j + 1;
        int32_t ci = S->door_cell[d] % P->nx, cj = S->door_cell[d] / P->nx;
        float xf = ((float)ci + offset_of(door_draw(S, a, 2))) * (float)P->dx;
        float yf = ((float)cj + offset_of(door_draw(S, a, 3))) * (float)P->dy;
        S->x[a] = xf;
        S->y[a] = yf;
        S->vx[a] = 0.0;
        S->vy[a] = 0.0;
        S->timer[a] = 0.0;
        S->state[a] = OR_ST_SHOPPING;
        S->cls[a] = OR_CLS_DRY;
        S->dest[a] = S->door_dest[leave];
        S->door_in += 1;
    }
}

double or_coupled_step(or_sim *S, double dt)
{
    if (!(dt > 0.0)) dt = or_compute_dt(S);
    or_fv_step(S, dt);
    or_ped_step(S, dt);
    or_count_evacuees(S);
    S->t += dt;
    S->step += 1;
    return dt;
}

void or_run(or_sim *S, int32_t n, const double *dts, double *dt_used, int32_t with_peds)
{
    for (int32_t k = 0; k < n; ++k) {
        double dt = dts ? dts[k] : or_compute_dt(S);
        if (dt_used) dt_used[k] = dt;
        or_fv_step(S, dt);
        if (with_peds) {
            or_ped_step(S, dt);
            or_count_evacuees(S);
        }
        S->t += dt;
        S->step += 1;
    }
}
