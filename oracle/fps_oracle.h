/*
 * fps_oracle.h -- plain FP64 CPU oracle of the coupled flood-pedestrian step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library under paper_1908_05232_amd/.
 *
 * Every array is owned by the caller (the Python binding keeps numpy arrays
 * alive and stores their addresses here).  Layout of every grid array is
 * row-major [ny][nx], index j*nx + i, x east with i, y north with j, cell
 * centre ((i+1/2)dx, (j+1/2)dy).
 */
#ifndef FPS_ORACLE_H
#define FPS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* boundary kinds per side (order W, E, S, N) */
#define OR_WALL 0
#define OR_TRANSMISSIVE 1

/* pedestrian roles, states and hazard classes */
#define OR_ROLE_EVACUEE 0
#define OR_ROLE_RESPONDER 1
#define OR_ST_EVAC 0       /* heading for (or waiting to head for) an exit */
#define OR_ST_EXITED 1
#define OR_ST_TO_STORAGE 2
#define OR_ST_PICKING 3
#define OR_ST_TO_BARRIER 4
#define OR_ST_DROPPING 5
#define OR_ST_SHOPPING 6   /* before the flood: walking to the door it leaves by (D3) */
#define OR_ST_OUTSIDE 7    /* outside the building: a free slot (D1) */
#define OR_MAX_DOOR 16
#define OR_CLS_DRY 0
#define OR_CLS_LOW 1
#define OR_CLS_MEDIUM 2
#define OR_CLS_HIGH 3
#define OR_CLS_HIGHEST 4
#define OR_CLS_UNSTABLE 5  /* the stability rule (S1-S4): swept off the feet, speed 0 */
#define OR_FLUX_HLLC 0
#define OR_FLUX_HLL 1

typedef struct {
    int32_t nx, ny;
    double dx, dy;
    double g, cfl, h_dry, dt_max;
    int32_t bc[4];                       /* W, E, S, N */
    int32_t inflow_side;                 /* 0..3 or -1 for none */
    int32_t inflow_c0, inflow_c1;        /* cell range [c0, c1) along that side */
    double n_base;                       /* Manning n of the bare cell */
    int32_t np_cap;                      /* evacuee count cap in the roughness rule */
    /* pedestrian constants */
    double tau, a_over_m, b_range, radius, r_cut, r_arrive;
    double v_class[5];                   /* index by class; [0] unused (dry uses v_base) */
    double hr_t[3];                      /* class thresholds 0.75, 1.5, 2.5 */
    double pick_s, drop_s;
    int32_t flux;                        /* OR_FLUX_HLLC (R1) or OR_FLUX_HLL (variant) */
    int32_t order;                       /* 1: the paper's first-order scheme; 2: the MUSCL variant */
    /* stability rule of a person standing in flowing water (S1-S4); 0 = Table 1 only */
    int32_t stability;
    double c_drag, mu_f, rho_w, rho_body; /* drag coefficient, foot friction, water and body densities */
    double body_h0, body_m0;             /* the body of people without one of their own (m, kg) */
    /* wading rule: walking speed capped by the drag of wading (W1-W3); 0 = Table 1 only */
    int32_t wading;
    double wade_k;                       /* sustained push as a fraction of the weight less buoyancy */
} or_params;

typedef struct {
    or_params P;
    /* flood state (FP64) */
    double *h, *qx, *qy, *z;
    int32_t *np;                         /* active evacuees per cell */
    double t;
    int64_t step;
    /* hydrograph, piecewise linear in (t_k, q_k), q in m^2/s */
    int32_t nh;
    const double *ht, *hq;
    /* accumulated volumes, m^3 */
    double v_in, v_out, v_clip;
    int32_t any_wet;
    /* navigation */
    int32_t n_dest, n_exit;
    const float *dist;                   /* [n_dest][ny][nx], metres, +inf = unreachable */
    const uint8_t *walk;                 /* [ny][nx], 1 walkable */
    /* agents */
    int32_t na;
    double *x, *y, *vx, *vy, *vbase, *timer;
    uint8_t *role, *state, *cls;
    int32_t *dest;
    /* sandbag barrier */
    int32_t nline;
    const int32_t *line;
    int32_t storage_dest, barrier_dest, n_layers, bags_per;
    double t_bag, t_last;
    int32_t active, layers_done, bags, done;
    int32_t drops_total;
    /* scratch for the cell lists, sized by the caller: bin_start[nbins+1], perm[na] */
    int32_t *bin_start, *perm;
    /* pre-flood door flow (sec. 3, sec. 3.2; D1-D6): n_door = 0 switches it off */
    int32_t n_door, door_rate;
    const int32_t *door_cell, *door_dest;  /* [n_door]: cell j*nx+i, destination index */
    uint64_t door_seed;
    int32_t doors_closed;
    int64_t door_in, door_out;
    /* bodies of the people (S1): height (m), mass (kg) per agent, or NULL */
    const double *body_h, *body_m;
} or_sim;

/* ---- single operations (exposed for the pins) ---- */
void or_hllc(double g, double hL, double uL, double vL, double hR, double uR, double vR,
             double F[3]);
void or_hll(double g, double hL, double uL, double vL, double hR, double uR, double vR,
            double F[3]);
void or_face(const or_params *P, double hL, double qnL, double qtL, double zL,
             double hR, double qnR, double qtR, double zR, int wall, double F[3],
             double *hsL, double *hsR);
double or_hydro_integral(int32_t nh, const double *ht, const double *hq, double a, double b);
int32_t or_hr_class(const or_params *P, double h, double qx, double qy, double *hr_out);
/* 1 if a person of the given height and mass cannot stand in the cell (S2, S3);
   *margin (may be NULL): the smaller relative excess of holding over pushing */
int32_t or_unstable(const or_params *P, double h, double qx, double qy, double height, double mass,
                    double *margin);
/* the wading speed cap of a person of that body in still water of depth h (W1, W2) */
double or_wade_speed(const or_params *P, double h, double height, double mass);
double or_n_eff(const or_params *P, int32_t np);
void or_friction(const or_params *P, double dt, double h, double n, double *qx, double *qy);
int32_t or_cell_index(double x, double d, int32_t n);
void or_bins_dims(const or_params *P, int32_t *bsx, int32_t *bsy, int32_t *nbx, int32_t *nby);
void or_build_bins(const or_params *P, int32_t na, const float *x, const float *y,
                   const uint8_t *state, int32_t *bin_start, int32_t *perm);

/* ---- the step ---- */
double or_compute_dt(const or_sim *S);
void or_fv_step(or_sim *S, double dt);            /* flood update, no time advance */
double or_minmod(double a, double b);             /* slope limiter of the second-order variant */
void or_count_evacuees(or_sim *S);                /* recompute np from the agents */
void or_ped_step(or_sim *S, double dt);           /* agents + barrier fill + door entries */
uint64_t or_splitmix64(uint64_t seed, uint64_t c); /* output c + 1 of SplitMix64 from seed (D6) */
void or_doors(or_sim *S);                         /* the entries of one step (D2, D4) */
/* one coupled step; dt <= 0 means "compute it", returns the dt used */
double or_coupled_step(or_sim *S, double dt);
/* n coupled steps; dts (may be NULL) replays a dt per step; dt_used (may be NULL) records */
void or_run(or_sim *S, int32_t n, const double *dts, double *dt_used, int32_t with_peds);
double or_mass(const or_sim *S);

#ifdef __cplusplus
}
#endif
#endif
