/*
 * fps.h -- C-ABI of libfps.so, the MI355X (gfx950) hot path of the coupled
 * flood-pedestrian simulator of Shirvani, Kesserwani & Richmond,
 * "Agent-based simulator of dynamic flood-people interactions" (arXiv 1908.05232).
 *
 * The calls follow the paper's problem statement: a grid of flood cells and an
 * aligned grid of navigation cells of the same size (sec. 2.1), initial
 * topography/water and boundary inflow hydrograph (sec. 3.1), pedestrian agents
 * whose roles are assigned at input (sec. 2.4), stepping, and read-out of the
 * flood fields and agent states (sec. 3.2 records coordinates, depth,
 * velocity and HR of the flood cells, coordinates and HR state of pedestrians).
 *
 * Conventions
 *  - Grids are row-major [ny][nx], index j*nx + i; x runs east with i, y north
 *    with j; the centre of cell (i, j) is ((i + 1/2) dx, (j + 1/2) dy).
 *  - The flood state is the conserved vector U = [h, hu, hv] of Eq. (1): depth
 *    h (m) and unit discharges hu, hv (m^2/s), FP32.  z is bed elevation (m).
 *  - Pointers documented "device" are HIP device pointers owned by the caller;
 *    they must stay valid until rebinding or fps_destroy.  The library never
 *    allocates or frees device memory: all scratch lives in the caller's
 *    workspace (fps_workspace_bytes).  "host" pointers are read during the
 *    call only.
 *  - Every call returns an fps_status.  An invalid argument returns
 *    FPS_E_INVALID and changes nothing.  No C++ exception crosses this ABI.
 *  - Stepping is asynchronous on the stream given to fps_create; numeric faults
 *    detected on the device are latched and reported by the next synchronising
 *    call (fps_get_diag) as FPS_E_NUMERIC, after which fps_step returns
 *    FPS_E_STATE until fields are bound again.  Reads stay available.
 *  - Handles are not thread-safe; distinct handles are independent.
 */
#ifndef FPS_H
#define FPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FPS_OK = 0,
    FPS_E_INVALID = -1,   /* bad argument: nothing changed */
    FPS_E_DEVICE = -2,    /* a HIP call failed */
    FPS_E_STATE = -3,     /* call out of order (e.g. step before binding fields) */
    FPS_E_CAPACITY = -4,  /* workspace or a fixed capacity too small */
    FPS_E_NUMERIC = -5    /* latched non-finite state or time step */
} fps_status;

/* boundary kinds, sides */
enum { FPS_BC_WALL = 0, FPS_BC_TRANSMISSIVE = 1 };
enum { FPS_SIDE_W = 0, FPS_SIDE_E = 1, FPS_SIDE_S = 2, FPS_SIDE_N = 3 };
/* face flux of the finite-volume update (sec. 2.2 defers the Riemann solver
   to Wang et al. 2011): HLLC (the default) or HLL for all three components */
enum { FPS_FLUX_HLLC = 0, FPS_FLUX_HLL = 1 };
/* agent roles (sec. 2.4), states, hazard classes (Table 1, plus DRY) */
enum { FPS_ROLE_EVACUEE = 0, FPS_ROLE_RESPONDER = 1 };
enum {
    FPS_ST_EVAC = 0,        /* heading for an exit (evacuees wait until any cell is wet) */
    FPS_ST_EXITED = 1,
    FPS_ST_TO_STORAGE = 2,  /* responder walking to the sandbag storage */
    FPS_ST_PICKING = 3,     /* responder picking up a bag (timer running) */
    FPS_ST_TO_BARRIER = 4,  /* responder carrying a bag to the barrier */
    FPS_ST_DROPPING = 5,    /* responder dropping the bag (timer running) */
    FPS_ST_SHOPPING = 6,    /* before the flood: walking to the door it will leave by (fps_set_doors) */
    FPS_ST_OUTSIDE = 7      /* outside the building: a free slot a new pedestrian may enter by (fps_set_doors) */
};
enum { FPS_CLS_DRY = 0, FPS_CLS_LOW = 1, FPS_CLS_MEDIUM = 2, FPS_CLS_HIGH = 3, FPS_CLS_HIGHEST = 4,
       FPS_CLS_UNSTABLE = 5 /* the stability rule: cannot stand in the flow (speed 0) */ };

/* Grid and flood constants.  Eq. (1)-(2), sec. 2.2; time step rule, sec. 3. */
typedef struct {
    int32_t nx, ny;          /* cells, >= 1 each, nx * ny <= 2^30 (32-bit byte offsets) */
    double dx, dy;           /* cell size (m), > 0 */
    double g;                /* gravity (m/s^2), e.g. 9.81 */
    double cfl;              /* Courant number in (0, 1], e.g. 0.5 */
    double h_dry;            /* dry threshold (m), e.g. 1e-5 */
    double dt_max;           /* step cap and the dry-domain step (s): 1.0 in the paper */
    int32_t bc[4];           /* W, E, S, N: FPS_BC_WALL or FPS_BC_TRANSMISSIVE */
    int32_t inflow_side;     /* side carrying the hydrograph, or -1 for none */
    int32_t inflow_c0, inflow_c1;  /* cells [c0, c1) along that side */
    double n_base;           /* Manning n of a cell with no evacuees, e.g. 0.01 */
    int32_t np_cap;          /* evacuees counted per cell, at most (20 in sec. 2.4) */
} fps_grid_desc;

/* Pedestrian constants (sec. 2.3-2.4, Table 1).  fps_ped_params_default fills
   the values used throughout: Table 1 speeds and thresholds, 30 s waits, and
   social-force constants tau 0.5 s, A/m 25 m/s^2, B 0.08 m, radius 0.25 m,
   interaction cut-off 1 m, arrival radius 1 m. */
typedef struct {
    double tau, a_over_m, b_range, radius, r_cut, r_arrive;
    double v_class[5];       /* walking speed per class; [0] unused (dry: agent's base speed) */
    double hr_t[3];          /* class thresholds (0.75, 1.5, 2.5) */
    double pick_s, drop_s;   /* responder waits (s) */
    /* Stability rule (the paper names richer walking-speed and stability rules
       and variable bodies as further work, sec. 2.4 note 1 and sec. 4; this is
       a mechanics reading of them).  stability = 0 (the default): Table 1
       alone.  stability = 1: a person in a wet cell is an upright cylinder of
       its height H and its volume M / rho_body (cross-section A = M /
       (rho_body H), diameter b = 2 sqrt(A / pi)); the water of depth h takes
       rho_w g A h of its weight W = M g by buoyancy and pushes it with the
       drag D = 1/2 rho_w c_drag b h u^2 of the flow speed u = |(hu, hv)| / h
       at the cell, acting at h / 2.  It cannot stand (class FPS_CLS_UNSTABLE,
       speed 0) when D > mu_f (W - buoyancy) (sliding), when D h / 2 > (W -
       buoyancy) b / 2 (toppling about the cylinder's edge), or when h >= H.
       Defaults 1.1, 0.45, 1000, 1000 kg/m^3; bodies from fps_set_bodies, else
       body_h0 = 1.71 m and body_m0 = 70 kg for everyone.  Evaluated in FP32. */
    int32_t stability;
    double c_drag, mu_f, rho_w, rho_body, body_h0, body_m0;
    /* Wading rule (the walking-speed half of the same further work; a
       mechanics reading).  wading = 0 (the default): Table 1's speeds.
       wading = 1: in a wet cell where the person stands, the walking speed is
       the smaller of Table 1's and v_w = sqrt(2 wade_k W' / (rho_w c_drag b
       h)), the speed at which the drag of wading through still water of depth
       h on the body's frontal width b (the cylinder above) equals the push
       wade_k W' its feet keep up, W' = g M - rho_w g A h the weight less
       buoyancy; v_w = 0 where W' <= 0.  The class stays Table 1's.  Default
       wade_k 0.1 (an adult of 1.71 m and 70 kg wades at 1.55, 0.88 and
       0.48 m/s in 0.2, 0.5 and 1 m of water).  Evaluated in FP32. */
    int32_t wading;
    double wade_k;
} fps_ped_params;

typedef struct {
    double t;                /* simulated time (s) */
    int64_t step;            /* steps taken */
    int64_t ped_steps;       /* agent-steps taken by non-exited agents */
    double dt_last;          /* step length of the last step (s) */
    double dt_next;          /* step length the next step will use (s) */
    double mass;             /* sum of h dx dy after the last step (m^3), FP64 on device */
    double v_in, v_out, v_clip;  /* accumulated inflow, transmissive outflow, clipped volume (m^3) */
    int32_t any_wet;         /* some cell has h > h_dry */
    int32_t n_agents;
    int32_t class_count[6];  /* agents inside per hazard class (FPS_CLS_*) */
    int32_t state_count[8];  /* agents per state */
    int32_t barrier_layers_done, barrier_active_cell, barrier_bags, barrier_done;
    int32_t drops_total;     /* sandbags delivered */
    int32_t status;          /* FPS_OK or the latched fault */
    int32_t active;          /* 0 once the end time (fps_set_end_time) is reached */
    int32_t flood_steps;     /* steps whose flood update ran; the others were dry and skipped */
    int32_t doors_closed;    /* the pre-flood door flow has stopped (fps_set_doors) */
    int64_t door_entries;    /* pedestrians that entered by a door */
    int64_t door_leaves;     /* pedestrians that left by a door before the flood */
} fps_diag;

typedef struct fps_sim fps_sim;
typedef struct fps_ens fps_ens;

/* Default pedestrian constants (see fps_ped_params). */
void fps_ped_params_default(fps_ped_params* out);

/* Bytes of device workspace one simulation of this grid with up to max_agents
   agents needs.  0 on invalid input. */
size_t fps_workspace_bytes(const fps_grid_desc* desc, int32_t max_agents);

/* Create a simulation.  ws: device workspace of ws_bytes (>= fps_workspace_bytes),
   256-byte aligned, caller-owned.  stream: hipStream_t all work is queued on
   (NULL = default stream).  ped may be NULL (defaults).  The handle is written
   to *out.  FPS_E_CAPACITY if ws_bytes is too small. */
int fps_create(const fps_grid_desc* desc, const fps_ped_params* ped, int32_t max_agents,
               void* ws, size_t ws_bytes, void* stream, fps_sim** out);
void fps_destroy(fps_sim* sim);

/* Bind the flood state and bed (device, float32 [ny][nx] each).  h >= 0.  The
   state is read and written in place by fps_step; z is read by every step and
   raised at barrier cells by the sandbag write-back (sec. 2.4).  Computes the
   first time step from the bound state.  Clears a latched numeric fault. */
int fps_bind_fields(fps_sim* sim, float* h, float* hu, float* hv, float* z);

/* Inflow hydrograph (sec. 3.1): piecewise-linear unit discharge q_k (m^2/s)
   at times t_k (s, increasing), constant beyond the ends; host arrays, copied;
   at most 64 points.  The inflow enters the cells along the inflow segment
   as a depth source of (1/dn) * integral of q over each step. */
int fps_set_hydrograph(fps_sim* sim, const double* t, const double* q, int32_t npts);

/* Navigation map (sec. 2.1): n_dest distance fields (device, float32
   [n_dest][ny][nx], metres to the nearest cell of that destination, +inf where
   unreachable); destinations [0, n_exit) are exits.  walkable: device uint8
   [ny][nx], 1 where pedestrians may stand.  Caller-owned, read-only.  The
   per-cell decisions the step takes from them are derived here, once: the
   heading of each cell for the first 16 destinations (the neighbour of
   steepest descent) and whether it lies within the arrival radius, by the
   same FP32 comparisons the step would make (further destinations are read
   from the fields at every step), and the obstacles around each cell; call
   again after changing the contents. */
int fps_set_navigation(fps_sim* sim, int32_t n_dest, int32_t n_exit, const float* dist,
                       const uint8_t* walkable);

/* Agents (sec. 2.1, 2.4): structure of arrays of length n <= max_agents, all
   device, caller-owned, updated in place by fps_step.  Positions in metres
   inside the domain on walkable cells; role FPS_ROLE_*; state FPS_ST_*;
   dest: destination index, or -1 to let the first step choose (evacuee:
   nearest exit, responder: storage); timer: seconds left of a wait.
   Recomputes the per-cell evacuee counts and the neighbour bins.
   FPS_E_INVALID if an agent lies outside the domain. */
int fps_bind_agents(fps_sim* sim, int32_t n, float* x, float* y, float* vx, float* vy,
                    float* v_base, uint8_t* role, uint8_t* state, uint8_t* hr_class,
                    int32_t* dest, float* timer);

/* Bodies of the agents for the stability and wading rules (fps_ped_params.stability, .wading):
   height (m) and mass (kg), device float32 [n_agents] each, caller-owned,
   read at every step; both NULL: the default body for everyone.  Call after
   fps_bind_agents (the arrays follow its agent count); FPS_E_INVALID for one
   array without the other. */
int fps_set_bodies(fps_sim* sim, const float* height, const float* mass);

/* Sandbag barrier (sec. 2.4, sec. 3.3): cells (host, copied) in fill order
   starting at the first barrier cell; responders shuttle between destination
   storage_dest and destination barrier_dest; a cell takes bags_per bags per
   layer; layers 1..n_layers-1 raise z by layer_thickness, the last by
   last_thickness.  At most 2 (nx + ny) cells. */
int fps_set_barrier(fps_sim* sim, const int32_t* cells, int32_t ncells, int32_t storage_dest,
                    int32_t barrier_dest, int32_t n_layers, float layer_thickness,
                    float last_thickness, int32_t bags_per);

/* Pre-flood pedestrian flow (sec. 3 and sec. 3.2: people enter and leave the
   open area by n_doors entrance doors, each with probability 1/n_doors, at a
   constant rate per door, and no one enters once the flood has reached the
   site).  Agents in state FPS_ST_OUTSIDE are free slots; each step, every
   free slot draws a door with probability 1/n_doors, and at each door the
   first per_step slots (in slot order) that drew it enter: placed at a
   uniform point in the central half of the door's cell, standing, state
   FPS_ST_SHOPPING, heading for a leaving door drawn uniformly from the other
   doors (so each door is the leaving door with probability 1/n_doors).  A
   walker that reaches its leaving door (within the arrival radius) goes back
   to FPS_ST_OUTSIDE and its slot may enter again.  On the first step after
   whose flood update some cell is wet, the doors close for good: no more
   entries, and every walker inside becomes an evacuee heading for the
   nearest exit (the doors are not exits).  The draws come from SplitMix64
   (Steele, Lea & Flood 2014) seeded with seed: draw k of slot a in step n is
   output ((n << 26) | (a << 2) | k) + 1 of the generator; a door index is
   ((u >> 32) * m) >> 32 for m choices and an offset in the cell 0.25 + 0.5 *
   (u >> 40) / 2^24.  Both the per-door rate and the slot count (the
   agents bound, 1000 in the paper) bound the population inside.  The
   walkers do not add roughness (only evacuees do, sec. 2.4).
   cells: host int32 [n_doors], the door cells (j * nx + i, walkable);
   dests: host int32 [n_doors], the distance field of each door, in
   [n_exit, n_dest) of the navigation map; copied.  n_doors in [2, 16],
   per_step >= 0.  n_doors = 0 switches the flow off.  Needs the navigation
   map; at most 2^24 agents.  Opens the doors (a previous closing is
   forgotten).  Synchronises. */
int fps_set_doors(fps_sim* sim, int32_t n_doors, const int32_t* cells, const int32_t* dests,
                  int32_t per_step, uint64_t seed);

/* Set the simulated time and step counter (resume). */
int fps_set_time(fps_sim* sim, double t, int64_t step);

/* Advance n_steps coupled steps (sec. 2.4 order: flood update Eq. (2), then
   pedestrians read the new flood state and move, then roughness and bed
   write-back).  Asynchronous; no host synchronisation inside.  A step in
   which nothing is wet and no inflow enters uses the 1 s dry step of sec. 3
   and skips the flood update (it would leave the state unchanged).  Steps
   are replayed from a captured HIP graph in chunks (fps_set_graph).
   FPS_E_STATE for a member of an ensemble (step the ensemble instead). */
int fps_step(fps_sim* sim, int32_t n_steps);

/* Stop advancing this scenario once its time reaches t_end (<= 0: never);
   further steps leave it unchanged.  Synchronises. */
int fps_set_end_time(fps_sim* sim, double t_end);

/* Depth the inflow adds to each inflow cell over [t0, t1]: the exact
   integral of the piecewise-linear hydrograph divided by the cell width
   normal to the inflow side (sec. 3.1); 0 without an inflow.  Host result. */
int fps_inflow_depth(fps_sim* sim, double t0, double t1, double* depth);

/* Judge region (used to check a learned flood update against the finite-
   volume method on part of the grid): while mask is set, a flood update
   writes only the cells of waves that meet a set block of the mask, a
   device uint8 [ceil(ny/block)][ceil(nx/block)] array of block x block cell
   blocks (caller-owned, read at every step, so its contents may change
   between calls), and every step has length dt_max (no CFL limit).  Cells
   outside the region keep stale values; a region of k steps is exact at
   cells more than k cells inside its border.  mask NULL restores the
   normal update.  block in [1, 4096].  First-order update only
   (FPS_E_STATE with the second-order variant). */
int fps_set_judge_region(fps_sim* sim, const uint8_t* mask, int32_t block);

/* Hold the flood (frozen = 1): the following steps have the fixed length
   dt_max, leave the flood state, its time step and volumes untouched, add no
   inflow, and advance only the pedestrians (hazard, movement, counts,
   sandbags), who read the state as it is, e.g. one written into the bound
   fields from outside (a learned update; rebind after writing).  frozen = 0
   resumes the coupled step with the CFL step of the current state.  Binding
   fields also resumes it.  Synchronises.  FPS_E_STATE before fields are
   bound. */
int fps_set_flood_frozen(fps_sim* sim, int32_t frozen);

/* Per-cell evacuee counts that raise the Manning coefficient (sec. 2.3) for
   a simulation with no agents bound: device int32 [ny][nx], copied
   (asynchronously) and kept until the next call; NULL clears them.
   FPS_E_STATE when agents are bound (their counts are used). */
int fps_set_occupancy(fps_sim* sim, const int32_t* counts);

/* Steps per captured HIP graph for fps_step (0 = launch every step
   eagerly); calls with fewer steps run eagerly.  Results are identical. */
int fps_set_graph(fps_sim* sim, int32_t steps_per_graph);

/* Face flux of the flood update (sec. 2.2, Eq. 2): FPS_FLUX_HLLC (default;
   the tangential momentum flux taken from the side of the contact wave) or
   FPS_FLUX_HLL (the tangential momentum averaged between the two outer waves
   like mass and normal momentum; those two are identical in both).  Same
   reconstruction, wave speeds, bed-slope terms and wall treatment.  Applies
   from the next step.  FPS_E_INVALID for another value; FPS_E_STATE for an
   ensemble member (the whole ensemble shares one flux: fps_ens_set_flux). */
int fps_set_flux(fps_sim* sim, int32_t flux);

/* Order of the flood update (sec. 2.2: the paper reduced the second-order
   scheme of Wang et al. 2011 to first order).  1 (the default): the
   first-order update.  2: the second-order variant: MUSCL reconstruction of
   (h, h + z, u, v) per direction with the minmod limiter (zero slope where
   the cell or a neighbour in that direction is dry, so first order at
   wet/dry fronts, and in ghost cells), the same hydrostatic reconstruction,
   face flux and walls on the reconstructed states, the second-order
   bed-slope form of Audusse et al. (2004) (still water stays still), and
   Heun's two-stage Runge-Kutta step with the depth cleanup after each stage;
   inflow and friction once per step.  Same time step rule.  Applies from the
   next step.  FPS_E_INVALID for another value; FPS_E_STATE for an ensemble
   member (fps_ens_set_order) or while a judge region is set (first order
   only). */
int fps_set_order(fps_sim* sim, int32_t order);

/* Synchronise the stream and report diagnostics (sec. 3.2 statistics). */
int fps_get_diag(fps_sim* sim, fps_diag* out);

/* Simulated time and the length of the next step only (host outputs): the
   part of fps_get_diag that needs no pass over the agents.  Synchronises. */
int fps_get_time(fps_sim* sim, double* t, double* dt_next);

/* Hazard rate HR = (max(|u|,|v|) + 0.5) h per cell (sec. 2.4), 0 where dry;
   device float32 [ny][nx] output, caller-owned.  Asynchronous. */
int fps_hazard_field(fps_sim* sim, float* hr_out);

/* Copies of internal state for verification, asynchronous, device outputs:
   counts: int32 [ny][nx] active evacuees per cell (the N_p of sec. 2.4);
   bin_start: int32 [nbins + 1]; perm: int32 [n_agents] agent ids sorted by
   (bin, id) for non-exited agents (bin_start[nbins] entries used). */
int fps_get_counts(fps_sim* sim, int32_t* counts);
int fps_get_bins(fps_sim* sim, int32_t* bin_start, int32_t* perm, int32_t* nbins_out);

/* Run n_steps with HIP events around every launch and return mean device
   milliseconds per launch of each kernel kind, in the order
   {flood update, pedestrian step, end-of-step finalize (reductions, barrier, bin scan), bin place, bin sort}; ms_out[5]
   (host).  Synchronises. */
int fps_step_profiled(fps_sim* sim, int32_t n_steps, double* ms_out);

/* Average duration of one flood-update launch of this simulation in its
   current tile shape: reps back-to-back launches on the current state between
   two HIP events on the library's stream (the state is left unchanged).
   Synchronises. */
int fps_time_flood(fps_sim* sim, int32_t reps, double* ms_per_launch);

/* Tile shape of the flood update: rows each wave marches through (a power of
   two in [1, 64]); every choice gives the same flood state, only the FP64
   mass diagnostic's summation order changes.  Synchronises. */
int fps_set_rows_per_wave(fps_sim* sim, int32_t rows);

/* Current tile shape of the flood update (rows per wave) into *rows (host). */
int fps_get_rows_per_wave(fps_sim* sim, int32_t* rows);

/* Pick the rows per wave for this grid by timing the flood update on the
   bound state (outputs to scratch; the simulation state is not advanced):
   every H in three interleaved passes, each H keeping its fastest pass.
   cache_path (host string, may be NULL): a text file of lines
   "<gfx arch> <nx> <ny> <rows> <ms>"; a matching line is used instead of
   timing, a new result is appended.  rows_out / ms_out may be NULL. */
int fps_autotune(fps_sim* sim, const char* cache_path, int32_t* rows_out, double* ms_out);

/* ---- Ensembles: S scenarios of uneven grids stepped by one set of launches
   per step (one flood launch over the tiles of every scenario, one
   pedestrian launch over every agent, one end-of-step launch with a block per
   scenario), each scenario with its own time, time step and end time.  The
   sweep structure follows sec. 3.3 (responder counts x barrier heights). ---- */

/* Workspace bytes for S scenarios (descs[S], max_agents[S] may be NULL = 0). */
size_t fps_ens_workspace_bytes(int32_t S, const fps_grid_desc* descs, const int32_t* max_agents);

/* Create an ensemble over one caller workspace; peds may be NULL (defaults)
   or point to S records.  Scenario s is configured through the member handle
   fps_ens_member(ens, s) with the same calls as a single simulation (bind
   fields, hydrograph, navigation, agents, barrier, end time, diagnostics). */
int fps_ens_create(int32_t S, const fps_grid_desc* descs, const fps_ped_params* peds,
                   const int32_t* max_agents, void* ws, size_t ws_bytes, void* stream,
                   fps_ens** out);
void fps_ens_destroy(fps_ens* ens);
/* Member handle of scenario s (owned by the ensemble; NULL if out of range). */
fps_sim* fps_ens_member(fps_ens* ens, int32_t s);
/* Advance every active scenario by n_steps of its own time step; asynchronous. */
int fps_ens_step(fps_ens* ens, int32_t n_steps);
/* As fps_step_profiled, for the whole ensemble. */
int fps_ens_step_profiled(fps_ens* ens, int32_t n_steps, double* ms_out);
/* Steps per captured HIP graph (0 = eager). */
int fps_ens_set_graph(fps_ens* ens, int32_t steps_per_graph);
/* Face flux of every scenario (see fps_set_flux). */
int fps_ens_set_flux(fps_ens* ens, int32_t flux);
/* Order of the flood update of every scenario (see fps_set_order). */
int fps_ens_set_order(fps_ens* ens, int32_t order);
/* Rows per wave of every scenario (see fps_set_rows_per_wave), tuned for the
   duration of the ensemble's whole flood launch on the bound states: one value
   for all scenarios, then each distinct grid size moved by factors of two
   while the launch gets shorter.  The states are not advanced; results do not
   depend on the choice.  cache_path (may be NULL): a text file of tuning
   results shared with fps_autotune; a line for this device's architecture
   and this mix of grids (the members' sizes in member order) is used instead
   of timing, and a new result is appended.  Synchronises. */
int fps_ens_autotune(fps_ens* ens, const char* cache_path);
/* Average duration of the ensemble's flood-update launch (one launch over
   the tiles of every member) in the current tile shapes: reps back-to-back
   launches on the current states between two HIP events on the ensemble's
   stream; the states are left unchanged.  Synchronises. */
int fps_ens_time_flood(fps_ens* ens, int32_t reps, double* ms_per_launch);
/* Number of scenarios that have not reached their end time.  Synchronises. */
int fps_ens_active(fps_ens* ens, int32_t* n_active);
const char* fps_ens_last_error(const fps_ens* ens);

/* ---- Convolutional surrogate (not part of the paper): five 3x3 convolutions,
   16 -> 64 -> 64 -> 64 -> 64 -> 3 channels, ReLU between, BF16 weights and
   activations with FP32 accumulation on the matrix cores, FP32 master
   weights and Adam.  It maps the scaled state (h, hu, hv, z, occupancy) to
   the scaled change of (h, hu, hv) over k finite-volume steps.  Tensors are
   channels last: x bf16 [n][H][W][16] (channels 5..15 zero), outputs and
   targets fp32 [n][H][W][4] (channel 3 zero).  H a multiple of 16, W of 32. ---- */
typedef struct fps_sur fps_sur;

/* Number of packed FP32 parameters: per layer W[cout][3][3][cin] then b[cout],
   with the padded channel counts (16 inputs, 16 outputs in the last layer). */
int32_t fps_sur_param_count(void);
size_t fps_sur_workspace_bytes(int32_t max_batch, int32_t H, int32_t W);
/* Caps on the blocks the convolution and weight-gradient kernels launch
   (0 = the defaults: one block per compute unit for both).  Both kernels walk their tiles with a stride of
   the grid, so a cap makes every block take several tiles at any size (used to
   test that path on small images); the forward pass and input gradients are
   unchanged bit for bit, the weight gradients change only in the grouping of
   their FP32 partial sums.  FPS_E_INVALID for a negative cap. */
int fps_sur_set_blocks(fps_sur* sur, int32_t conv_blocks, int32_t wgrad_blocks);
int fps_sur_create(int32_t max_batch, int32_t H, int32_t W, void* ws, size_t ws_bytes, void* stream,
                   fps_sur** out);
void fps_sur_destroy(fps_sur* sur);
/* Copy packed FP32 parameters (device) into the master weights; clears Adam. */
int fps_sur_set_params(fps_sur* sur, const float* params);
int fps_sur_get_params(fps_sur* sur, float* params);
/* y = net(x) for n <= max_batch images (device pointers). */
int fps_sur_forward(fps_sur* sur, int32_t n, const void* x_bf16, float* y);
/* Allocation-free forward pass, for callers that cannot allocate device
   memory or bring a workspace (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): y = net(x) for n images of H x W
   with the packed FP32 parameters params (device, caller-owned, the layout of
   fps_sur_param_count; read only), x bf16 [n][H][W][16] and y fp32
   [n][H][W][4] (device, caller-owned), on stream (NULL = default).  Same
   kernels and same result, bit for bit, as fps_sur_forward with these
   parameters.  The BF16 weights and the activations live in a static device
   array of the library, one per GPU, set up on the first call on that GPU and
   held until the process ends: about 33 MB, for n * H * W <= 131,072 pixels
   (two 256 x 256 patches).  Calls that overlap on one GPU race on that array
   (run them on one stream, or one after another).  Allocates nothing and
   does not synchronise.  FPS_E_INVALID for NULL pointers or H, W not positive
   multiples of 16, 32; FPS_E_CAPACITY, before any device work, for more
   pixels; FPS_E_DEVICE if the array's address cannot be found (message in
   fps_sur_last_error(NULL)). */
int fps_sur_forward_noalloc(const float* params, int32_t n, int32_t H, int32_t W, const void* x_bf16, float* y,
                            void* stream);
/* Mean squared error against target and its gradients (packed like the
   parameters; grads may be NULL); loss: one device float. */
int fps_sur_gradients(fps_sur* sur, int32_t n, const void* x_bf16, const float* target, float* grads,
                      float* loss);
/* One Adam step with the last gradients (beta 0.9 / 0.999, eps 1e-8). */
int fps_sur_adam(fps_sur* sur, float lr);
/* fps_sur_gradients then fps_sur_adam. */
int fps_sur_train_step(fps_sur* sur, int32_t n, const void* x_bf16, const float* target, float lr,
                       float* loss);
/* Network input from a flood state into x bf16 [ny][nx][16], channels h, hu,
   hv, z / 3, occupancy / 4 and, on the cells of the inflow segment (the
   boundary cells of side inflow_side, -1 = none, from c0 to c1 - 1), the depth
   the inflow adds over the block (fps_inflow_depth); the rest zero.  h, hu,
   hv, z: device float32 [ny][nx]; occupancy: evacuee counts per cell, device
   int32 [ny][nx] or NULL.  Async. */
int fps_sur_pack(int32_t nx, int32_t ny, const float* h, const float* hu, const float* hv, const float* z,
                 const int32_t* occupancy, int32_t inflow_side, int32_t inflow_c0, int32_t inflow_c1,
                 double inflow_depth, void* x_bf16, void* stream);
/* Training target: the scaled change (U1 - U0) / scale into fp32 [H][W][4]; async. */
int fps_sur_make_target(int64_t npix, const float* h0, const float* hu0, const float* hv0,
                        const float* h1, const float* hu1, const float* hv1, float* target, void* stream);
/* Apply a network output to a flood state in place: U += scale * y, h >= 0;
   a cell that was dry (h <= h_dry) stays dry unless the update puts at least
   h_snap metres on it; no discharge where h <= h_dry.  Async.  (Rebind the
   fields of a simulation afterwards so its next time step is recomputed.) */
int fps_sur_apply(int64_t npix, const float* y, float* h, float* hu, float* hv, float h_dry, float h_snap,
                  void* stream);
/* Judge of a surrogate state (a) against a finite-volume state (b) at the
   cells of the judged agents of the device SoA (x, y, state) of length na,
   those that have not exited: every stride-th agent and, when a selection
   state (hs, qxs, qys; device float32 [ny][nx], may be NULL) is given, also
   every agent whose cell there is within h_margin (m) of the dry threshold
   h_dry or has a hazard rate within hr_margin of one of the three Table 1
   thresholds hr_thresholds[3] (host): the people whose class a small depth
   error could change.  out3 (device int32[3]): [0] judged agents whose depth
   differs by more than tol (m) or whose hazard class (Table 1, DRY where
   h <= h_dry) differs, [1] the largest depth difference as float bits, [2]
   the number of judged agents.  Cells: floor(x / dx) in FP32, clamped to the
   grid.  Async.  FPS_E_INVALID, before any device call, for bad sizes, a NULL
   array (the agent and flood arrays may be NULL only when na = 0) or a
   negative margin. */
int fps_sur_judge(int32_t na, int32_t stride, const float* x, const float* y, const uint8_t* state,
                  int32_t nx, int32_t ny, double dx, double dy, const float* ha, const float* qxa,
                  const float* qya, const float* hb, const float* qxb, const float* qyb, double tol,
                  double h_dry, const double* hr_thresholds, const float* hs, const float* qxs, const float* qys,
                  double hr_margin, double h_margin, int32_t* out3, void* stream);
/* Judge region for fps_set_judge_region: clears mask (device uint8
   [ceil(ny/block)][ceil(nx/block)]) and marks every block within halo cells of
   the cell of a judged agent (the same people as fps_sur_judge with the same
   selection arguments; hr_thresholds may be NULL when hs is); async.
   FPS_E_INVALID for bad sizes, a NULL mask, NULL agent arrays with na > 0,
   or a negative margin. */
int fps_sur_judge_mask(int32_t na, int32_t stride, const float* x, const float* y, const uint8_t* state,
                       int32_t nx, int32_t ny, double dx, double dy, const float* hs, const float* qxs,
                       const float* qys, double h_dry, const double* hr_thresholds, double hr_margin,
                       double h_margin, int32_t halo, int32_t block, uint8_t* mask, void* stream);
/* Per-cell counts of evacuees still evacuating (role evacuee, state EVAC),
   the counts that raise the Manning coefficient (sec. 2.3), into device int32
   [ny][nx]; async.  FPS_E_INVALID for bad sizes, NULL counts, or NULL agent
   arrays with na > 0. */
int fps_sur_occupancy(int32_t na, const float* x, const float* y, const uint8_t* role,
                      const uint8_t* state, int32_t nx, int32_t ny, double dx, double dy,
                      int32_t* counts, void* stream);
/* Device copy of a flood state (h, hu, hv) of npix cells; async. */
int fps_sur_copy_state(int64_t npix, const float* h, const float* hu, const float* hv, float* h_out,
                       float* hu_out, float* hv_out, void* stream);
const char* fps_sur_last_error(const fps_sur* sur);

/* Streaming probe, the practical bandwidth ceiling the flood update's roofline
   is read against: buf (device, caller-owned, 16-byte aligned) holds n_in
   input arrays followed by n_out output arrays of n floats each, array k at
   buf + k * stride (stride >= n floats); a pass reads every input element once
   and writes every output element once with 16-byte accesses (out_k = sum of
   the inputs + k).  (n_in, n_out) is (1, 1) (a copy), (4, 3) or (5, 3) (the
   flood update's SoA streams: h, hu, hv, z and the evacuee counts in; h, hu,
   hv out).  reps passes between two HIP events on stream; *ms_per_pass gets
   the mean.  n and stride positive multiples of 4.  Synchronises. */
int fps_stream_probe(float* buf, int64_t n, int64_t stride, int32_t n_in, int32_t n_out, int32_t reps, void* stream,
                     double* ms_per_pass);

const char* fps_status_string(int status);
/* Last error message of this handle (or of the last failed fps_create when sim is NULL). */
const char* fps_last_error(const fps_sim* sim);

#ifdef __cplusplus
}
#endif
#endif /* FPS_H */
