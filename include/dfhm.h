/*
 * dfhm.h -- C ABI of the MI355X Dufort-Frankel hygrothermal wall / room solver.
 *
 * The library advances batches of 1-D porous walls under the coupled heat and
 * vapour-pressure balance of Gasparin, Berger, Dutykh & Mendes (arXiv
 * 1703.10119), Sec. 2 eq. (2.2), with Robin surface exchange eq. (2.3),
 * uniform initial state eq. (2.4), the nonlinear Dufort-Frankel update of
 * Sec. 3.1 (eqs. DF_NL, DF_NL_RHS) applied to the weakly coupled pair as in
 * App. A (moisture first, then heat with the new vapour pressure, eq.
 * DF_eq2b), the DF-averaged surface value in the Robin term (eq. bc_v), and
 * optionally a lumped room-air balance per zone (Sec. 5.1, eq. LAV_equation
 * with the exchange terms of eq. LAV_couplage) coupled explicitly as in
 * Sec. 5.3 (eq. wbse_tn_exp).  All time stepping runs in HIP kernels on one
 * gfx950 device.
 *
 * Conventions
 *   - Units are SI: K, Pa, m, s, W, kg.
 *   - Side 0 of a wall is x = 0, side 1 is x = L.  Surface fluxes are
 *     positive INTO the wall on both sides: heat in W/m2, vapour in kg/(m2 s).
 *   - Every call returns a dfhm_status; nothing aborts across the ABI.  On an
 *     error the context is unchanged, the message is kept for
 *     dfhm_last_error(), and a non-finite state latches DFHM_E_STATE until
 *     fields are set again.
 *   - Host descriptors are copied at the call; the caller may free them
 *     afterwards.  Host output buffers are caller-owned.
 *   - One context must not be used by two threads at once.  Contexts are
 *     independent of each other.
 *   - Work is queued on the stream given in dfhm_config (NULL = the default
 *     stream).  Calls that return host data synchronise that stream.
 */
#ifndef DFHM_H
#define DFHM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dfhm_ctx dfhm_ctx;

typedef enum {
    DFHM_OK = 0,
    DFHM_E_INVAL = 1,     /* bad argument or descriptor */
    DFHM_E_NOMEM = 2,     /* device allocation failed or arena too small */
    DFHM_E_DEVICE = 3,    /* a HIP call failed */
    DFHM_E_NONFINITE = 4, /* a step produced a non-finite value */
    DFHM_E_STATE = 5,     /* call not allowed in the current state */
    DFHM_E_UNSTABLE = 6   /* explicit room step would be unstable at dt */
} dfhm_status;

enum { DFHM_FP64 = 0, DFHM_FP32 = 1 };
/* Start of the three-level scheme (the paper leaves it open):
 *   FTCS   -- the first step is m forward-Euler sub-steps of dt/m, with m =
 *             ceil(2 dt / b), b the explicit stability bound of the wall at
 *             its initial state (dimensional form of eqs. cfl_heat_Eq and
 *             cfl_moisture_Eq, surface exchange included);
 *   REPEAT -- level n-1 := level 0 and the first step is a DF step. */
enum { DFHM_START_FTCS = 0, DFHM_START_REPEAT = 1 };
/* Kernel schedule: STREAM = one launch per step over HBM-resident levels;
 * RESIDENT = one persistent launch per chunk of steps, each workgroup keeping
 * its walls' levels on chip; AUTO = chosen by the autotuner. */
enum { DFHM_SCHED_AUTO = 0, DFHM_SCHED_STREAM = 1, DFHM_SCHED_RESIDENT = 2 };
/* Material law of a context (dfhm_config.law): SHAPE = the per-layer law
 * of dfhm_layer below; TABLE1 = the load-bearing material of Sec. 6
 * (Table 1), see dfhm_layer. */
enum { DFHM_LAW_SHAPE = 0, DFHM_LAW_TABLE1 = 1 };

/* x(t) = mean + amp * sin(2 pi t / period_s + phase) */
typedef struct { double mean, amp, period_s, phase; } dfhm_sine;

/* One material layer.  With phi = Pv / Ps(T), theta = T - 273.15 and
 * Ps(T) = 610.94 exp(17.625 theta / (theta + 243.04)) Pa (Magnus form):
 *   k_TT = k0  (1 + a_T phi)        W/(m K)
 *   k_M  = kM0 (1 + a_M phi^2)      s
 *   k_TM = b_TM k_M                 m2/s      (k_TM = Lv delta_v, Sec. 2)
 *   c_TT = c0  (1 + c_T phi)        J/(m3 K)
 *   c_M  = cM0 (1 + c_M phi)        s2/m2
 *   c_TM = (e_TM + f_TM theta) c_M  (c_TM = c_w T f'/Ps, Sec. 2)
 * All-zero shape coefficients (a_T, a_M, c_T, c_M, f_TM) give the
 * constant-coefficient walls of Sec. 6.1 (Table 2).
 *
 * Under DFHM_LAW_TABLE1 (Table 1, with s = -R_v T ln phi the suction in
 * J/kg, R_v = 461.5, T in K; s = 0 for phi >= 1):
 *   f    = 47.1 [1 + (1.25e-5 s)^1.65]^-(1-1/1.65) + 109.9 [1 + (1.8e-5 s)^6]^-(5/6)  kg/m3
 *   k_TT = k0 (0.2 + 0.0045 f)
 *   k_M  = kM0 (1.97e-10 10^(1.44 - 0.07 log10(2 phi)) + 1.77e-7 exp(-8 (2 phi - 2)^2))
 *   k_TM = kM0 Lv delta_v,  delta_v = 1.88e-6/T (1 - f/157) / (0.503 (1 - f/157)^2 + 0.497)
 *   c_TT = c0 790 x 870 + cw f,  c_M = cM0 (df/dphi) / Ps,  c_TM = cw theta c_M
 * so that k0 = kM0 = c0 = cM0 = 1 is the paper's material; the other fields
 * are ignored. */
typedef struct {
    double thickness_m;
    double k0, a_T, kM0, a_M, b_TM, c0, c_T, cM0, c_M, e_TM, f_TM;
} dfhm_layer;

/* One wall: nx uniform nodes over L = sum of layer thicknesses (dx =
 * L/(nx-1); both surfaces are nodes).  Node j belongs to the first layer
 * whose right end is >= j dx; a face between nodes of different layers takes
 * the harmonic mean of the two layers' conductivities at the face state
 * (zero when both are zero).  T_amb / RH_amb give the outdoor air of each
 * side (ignored on a side coupled to a room).  T0 / RH0 give the uniform
 * initial state (Pv0 = RH0 Ps(T0)).  area_m2 is used by the room balance.
 *
 * Radiation (Sec. 2, the heat source q_inf of the boundary condition eq.
 * (2.3)): the heat source of side s at t^n is
 *     q_inf[s] + max(0, q_sun[s](t^n))
 *       + (side coupled to a zone)  s_z eps[s] sigma sum_w (T_w^4 - T^4),
 * the last term being the long-wave exchange with the zone-side surfaces of
 * all walls of the zone (T_w, T: level-n zone-side surface temperatures in K,
 * sigma = 5.670374419e-8 W/(m2 K4), s_z the zone's view_factor, eps the
 * emissivity of the receiving surface).  All three enter the surface node
 * explicitly and are part of the reported heat flux.  The start-up step
 * holds the long-wave term at level 0 and evaluates q_sun at each sub-step. */
typedef struct {
    int32_t nx, n_layers;           /* 3 <= nx <= 2048, 1 <= n_layers <= 3 */
    dfhm_layer layer[3];
    double h_T[2], h_M[2];          /* W/(m2 K), s/m;  >= 0 */
    double q_inf[2], g_inf[2];      /* extra heat / liquid flux into the wall */
    dfhm_sine T_amb[2], RH_amb[2];
    double T0, RH0, area_m2;
    double emissivity[2];           /* in [0, 1]; used on a zone side only */
    dfhm_sine q_sun[2];             /* incident radiation, W/m2, clipped at 0
                                       (period_s > 0 even when unused) */
} dfhm_wall;

/* One perfectly mixed zone (Sec. 5.1): w ~ Pv / Pv_ref, ventilation flow
 * g_v = ach * rho_a V / 3600 kg/s from outdoor air (T_out, RH_out), moisture
 * source g_o (latent heat Lv g_o to the air) and heat source Q_h, both
 * piecewise constant over n_sched slots of sched_dt_s, repeated
 * periodically. */
typedef struct {
    double volume_m3, ach_per_h, T0, RH0;
    dfhm_sine T_out, RH_out;
    int32_t n_sched;                /* >= 1 */
    double sched_dt_s;              /* > 0 */
    const double *g_o_kg_s;         /* [n_sched] host */
    const double *Q_h_W;            /* [n_sched] host */
    double view_factor;             /* s between two surfaces of the zone, in
                                       [0, 1]; 0 = no long-wave exchange */
} dfhm_room;

typedef struct {
    int32_t precision;      /* DFHM_FP64 | DFHM_FP32 (FP32 fields stored as
                               deviations from each wall's initial state; the
                               outdoor phase, flux integrals and room air stay
                               FP64) */
    int32_t startup;        /* DFHM_START_* */
    int32_t schedule;       /* DFHM_SCHED_* */
    int32_t chunk_steps;    /* steps per resident launch / captured graph; 0 = auto */
    double dt_s;            /* > 0 */
    double Lv, cw;          /* 0 -> 2.5e6 J/kg, 4180 J/(kg K) */
    double rho_a, c_pa, c_pv, Pv_ref;   /* 0 -> 1.2, 1006, 1860, 1.61e5 */
    void *stream;           /* hipStream_t or NULL */
    int32_t block_threads;  /* resident: threads per workgroup; 0 = autotune */
    int32_t nodes_per_thread; /* resident: nodes per thread; 0 = autotune */
    int32_t use_graph;      /* stream schedule: replay captured chunks (1) */
    int32_t law;            /* DFHM_LAW_* */
} dfhm_config;

/* Device bytes the wall state of a batch needs: the two stored time levels of
 * T and Pv of the three-level scheme (eq. dufort, Sec. 3.1: level n+1 is
 * written over level n-1), node layer ids, descriptors, flux state and tile
 * tables.  Pass at least this much as the arena of dfhm_create to keep all
 * wall state in caller-owned memory.  Zone state is not part of the arena
 * (so this takes no zone count): zones are coupled after dfhm_create, by
 * dfhm_room_couple, which allocates their few bytes per zone itself.
 * Returns 0 when cfg or walls is NULL or n_walls < 1. */
size_t dfhm_arena_bytes(const dfhm_config *cfg, const dfhm_wall *walls, int64_t n_walls);

/* Create a batch of n_walls >= 1 walls at their initial state (step index 0).
 * arena: caller-owned device memory of arena_bytes (e.g. a torch tensor) that
 * must outlive the context and is never freed by the library; NULL = the
 * library allocates and frees its own.  Errors: DFHM_E_INVAL on a bad
 * descriptor (nx, n_layers, thickness <= 0, negative coefficients, dt <= 0),
 * DFHM_E_NOMEM, DFHM_E_DEVICE.  *out is set only on success. */
dfhm_status dfhm_create(const dfhm_config *cfg, const dfhm_wall *walls, int64_t n_walls,
                        void *arena, size_t arena_bytes, dfhm_ctx **out);

/* Couple walls to n_rooms zones (Sec. 5.1-5.3): wall_room[w] = zone index or
 * -1, room_side[w] = 0 | 1 the side facing that zone; every zone needs at
 * least one wall (DFHM_E_INVAL otherwise).  Each step the walls
 * see the zone air of level n on that side and the zone is advanced by
 * forward Euler with the level-n surface values (eq. wbse_tn_exp).  Allowed
 * only at step index 0, once.  DFHM_E_UNSTABLE if a zone's explicit step
 * fails a_T dt < 1 or a_M dt < 1, with a_T = (sum A h_T + g_v c_ma) /
 * (rho_a V c_ma) and a_M = (sum A h_M + g_v / Pv_ref) Pv_ref / (rho_a V). */
dfhm_status dfhm_room_couple(dfhm_ctx *ctx, const dfhm_room *rooms, int64_t n_rooms,
                             const int64_t *wall_room, const int8_t *room_side);

/* Airflow between two zones (Sec. 5.1, the inter-zone sources of eq.
 * LAV_equation): g_kg_s of dry air moves from zone_a to zone_b and the same
 * back.  Zone i gains the heat g (c_j theta_j - c_i theta_i) + L_v g (w_j - w_i)
 * and the vapour g (w_j - w_i) from its partner j, with theta = T - 273.15
 * (degC: the moist-air enthalpy c_pa theta + w (L_v + c_pv theta) of the
 * two zones), c = c_pa + c_pv w and w = Pv / Pv_ref, all at level n. */
typedef struct {
    int32_t zone_a, zone_b;         /* distinct zone indices */
    double g_kg_s;                  /* >= 0 */
} dfhm_zone_link;

/* Link zones (host array of n_links >= 1 links, copied).  Allowed once, after
 * dfhm_room_couple, at step index 0.  The zone stability test of
 * dfhm_room_couple is repeated with the link flows added to both zones'
 * g_v (DFHM_E_UNSTABLE).  The resident schedule keeps linked zones, with all
 * their walls, in one workgroup: a connected set of zones must fit one
 * (at most 16 zones, 64 walls, the launch shape's node capacity and 8 links
 * per zone), else stepping on that schedule fails with DFHM_E_INVAL and the
 * streaming schedule is the one to use.  Errors: DFHM_E_INVAL (zone index out
 * of range, zone_a == zone_b, g < 0 or not finite, no zones coupled),
 * DFHM_E_STATE (not at step 0, or links set before). */
dfhm_status dfhm_zone_links(dfhm_ctx *ctx, const dfhm_zone_link *links, int64_t n_links);

/* Queue n_steps >= 0 time steps (asynchronous on the context stream).  One
 * step is the nonlinear Dufort-Frankel update of Sec. 3.1 (eqs. DF_NL,
 * DF_NL_RHS; coefficients at level n, faces at the face-averaged state),
 * moisture first and heat with the new vapour pressure (App. A, eqs. DF_eq1,
 * DF_eq2b), the surface nodes with the DF-averaged surface value (eq. bc_v),
 * the outdoor air at t^n, and the zones advanced explicitly from level-n
 * surfaces (Sec. 5.3, eq. wbse_tn_exp).  The first step from step index 0
 * is the start-up step of dfhm_config.startup.  Errors: DFHM_E_INVAL for
 * n_steps < 0 or a resident group beyond the launch shape's limits,
 * DFHM_E_STATE while a non-finite state is latched, DFHM_E_DEVICE. */
dfhm_status dfhm_step_n(dfhm_ctx *ctx, int64_t n_steps);

/* Wait for queued work; DFHM_E_NONFINITE if a finished step produced a
 * non-finite value (the context then latches DFHM_E_STATE). */
dfhm_status dfhm_sync(dfhm_ctx *ctx);

/* Surface fluxes of the boundary condition eq. (2.3) (HAM_BC) as the scheme
 * applies them (eq. bc_v), host arrays [n_walls][2 sides][2 fields (heat,
 * vapour)]:
 * now = the flux applied by the most recent step (DF-averaged surface value,
 * ambient at t^n; for the forward-Euler start-up step the mean over its
 * sub-steps); integral = dt * sum over completed steps, Neumaier-compensated
 * in FP64 (J/m2, kg/m2).  Either pointer may be NULL.  Synchronises. */
dfhm_status dfhm_fluxes(dfhm_ctx *ctx, double *now, double *integral);

/* Fields of one wall at level 0 (= t^n) or 1 (= t^{n-1}) of the three-level
 * scheme (eq. dufort) as FP64 host arrays of nx values (absolute K and Pa,
 * also on the FP32 path).  Synchronises.  DFHM_E_INVAL for a wall or level
 * out of range or a NULL array. */
dfhm_status dfhm_get_fields(dfhm_ctx *ctx, int64_t wall, int level, double *T, double *Pv);
/* All walls concatenated in wall order (sum of nx values each). */
dfhm_status dfhm_get_all_fields(dfhm_ctx *ctx, int level, double *T, double *Pv);
/* Overwrite one wall's level (0 or 1); clears a latched non-finite state. */
dfhm_status dfhm_set_fields(dfhm_ctx *ctx, int64_t wall, int level, const double *T,
                            const double *Pv);
/* Set the step index (with dfhm_set_fields: restart from two given levels;
 * n >= 1 makes the next step a DF step). */
dfhm_status dfhm_set_step_index(dfhm_ctx *ctx, int64_t n);

/* Zone air at level n (the state of eq. LAV_equation, Sec. 5.1): Ta [K],
 * Pva [Pa], host arrays of n_rooms.  Synchronises; DFHM_E_STATE without
 * zones. */
dfhm_status dfhm_get_rooms(dfhm_ctx *ctx, double *Ta, double *Pva);

/* Resolved launch configuration (after autotuning). */
typedef struct {
    int32_t schedule, precision, block_threads, nodes_per_thread;
    int32_t chunk_steps, n_blocks, max_walls_per_block, use_graph;
    int64_t n_walls, n_rooms, total_nodes, step_index;
    double pack_efficiency;   /* useful nodes / node slots of the resident packing */
    int32_t max_rooms_per_block, reserved;
    int64_t n_links;          /* inter-zone links */
} dfhm_info;
dfhm_status dfhm_get_info(const dfhm_ctx *ctx, dfhm_info *info);

/* Choose the schedule and resident launch shape by timing candidate kernels
 * on a copy of the batch for `probe_steps` steps each (state unchanged).  The
 * result is cached per (device, precision, schedule candidates, size
 * bucket) in the file named by the DFHM_AUTOTUNE_CACHE environment variable
 * when it is set.  Allowed only at step index 0 or after a completed step. */
dfhm_status dfhm_autotune(dfhm_ctx *ctx, int32_t probe_steps);

/* ---------------------------------------------------------------------
 * Implicit comparator (Sec. 5.2 and Algorithm 1): the theta-scheme in time
 * (theta = 1 Euler implicit, 1/2 Crank-Nicolson) on the same grid and law as
 * the DF scheme, with fixed-point sub-iterations on the coefficients
 * (evaluated at the theta-weighted state between level n and the current
 * iterate, faces at the face-averaged state) and one tridiagonal solve per
 * field and sub-iteration, moisture first, heat with the new vapour
 * pressure.  A sub-iteration loop stops when the largest change of T and of
 * Pv is at most eta times the largest |T| and |Pv|, or after max_iters.  FP64,
 * either material law (dfhm_implicit_config.law),
 * walls with the outdoor air on both sides (zones are not coupled), from the
 * walls' uniform initial state; no start-up step (two-level scheme).  For
 * measuring what the explicit DF scheme saves against it.
 * ------------------------------------------------------------------- */
typedef struct dfhm_implicit dfhm_implicit;
typedef struct {
    double dt_s;           /* > 0 */
    double theta;          /* in [0.5, 1] */
    double eta;            /* > 0, relative fixed-point tolerance */
    int32_t max_iters;     /* >= 1 sub-iterations per step */
    int32_t law;           /* DFHM_LAW_SHAPE or DFHM_LAW_TABLE1 (the material
                              of Sec. 6 and Table 3) */
    double Lv;             /* 0 -> 2.5e6 J/kg */
    void *stream;          /* hipStream_t or NULL */
    double cw;             /* 0 -> 4180 J/(kg K) (c_TM of the Table 1 law) */
} dfhm_implicit_config;
/* Walls as for dfhm_create (side 1 uses T_amb[1] / RH_amb[1]).  Allocates
 * 7 doubles per node (walls grouped by 64, each group padded to its longest
 * wall).  DFHM_E_INVAL on a bad descriptor or configuration. */
dfhm_status dfhm_implicit_create(const dfhm_implicit_config *cfg, const dfhm_wall *walls,
                                 int64_t n_walls, dfhm_implicit **out);
/* Queue n_steps steps on the stream (asynchronous). */
dfhm_status dfhm_implicit_step_n(dfhm_implicit *ic, int64_t n_steps);
/* T and Pv (host, nx values each) of one wall at the current step; synchronises. */
dfhm_status dfhm_implicit_get_fields(dfhm_implicit *ic, int64_t wall, double *T, double *Pv);
/* Mean sub-iterations per wall and step so far; synchronises. */
dfhm_status dfhm_implicit_iterations(dfhm_implicit *ic, double *mean_per_step);
int64_t dfhm_implicit_step_index(const dfhm_implicit *ic);
void dfhm_implicit_destroy(dfhm_implicit *ic);

/* ---------------------------------------------------------------------
 * Surface-flux surrogate (not part of the paper): an MLP mapping a wall's
 * recent outdoor history and parameters to the next interval's mean interior
 * surface fluxes, with BF16 weights / activations and FP32 accumulation on
 * the MFMA units, trained on histories the DF solver produces; the DF solve
 * is its fallback.  Layers: n_in -> width (GELU) x depth -> n_out.  All
 * device pointers are caller-owned; BF16 is stored as uint16 (round to
 * nearest even).  Work is queued on cfg->stream.
 * ------------------------------------------------------------------- */
typedef struct dfhm_mlp dfhm_mlp;
typedef struct {
    int32_t n_in;          /* input features, multiple of 8 */
    int32_t width;         /* hidden width, multiple of 8 */
    int32_t depth;         /* hidden layers, 1..16 */
    int32_t n_out;         /* outputs, 1..32 (training needs an even count) */
    int32_t max_batch;     /* largest batch of one call, <= 4,194,304 */
    uint64_t seed;         /* weight initialisation (normal, std sqrt(2/fan_in)) */
    float beta1, beta2, eps, weight_decay;   /* AdamW */
    void *stream;          /* hipStream_t or NULL */
} dfhm_mlp_config;

dfhm_status dfhm_mlp_create(const dfhm_mlp_config *cfg, dfhm_mlp **out);
int64_t dfhm_mlp_param_count(const dfhm_mlp *m);
/* Parameters in logical order: for each layer W[n_out_l][n_in_l] row-major
 * then b[n_out_l]; FP32 host arrays of dfhm_mlp_param_count values. */
dfhm_status dfhm_mlp_get_params(dfhm_mlp *m, float *host);
dfhm_status dfhm_mlp_set_params(dfhm_mlp *m, const float *host);
/* y_dev[batch][n_out] (FP32) = network(x_dev[batch][n_in] BF16).  Keeps
 * every hidden activation and pre-activation in the network's buffers. */
dfhm_status dfhm_mlp_forward(dfhm_mlp *m, const uint16_t *x_dev, int64_t batch, float *y_dev);

/* Stored intermediates of the last forward / gradients pass, for checking
 * them layer by layer: kind ACT = the BF16 GELU output of hidden layer
 * `layer` (0 <= layer < depth), PRE = its BF16 pre-activation, DZ = the BF16
 * loss gradient with respect to the pre-activation of layer `layer` (0 <=
 * layer <= depth; the output layer's rows are padded to 32 columns), after a
 * gradients or training pass.  Copies rows x columns values to host
 * (row-major); synchronises.  DFHM_E_INVAL for a bad kind, layer or rows. */
enum { DFHM_MLP_ACT = 0, DFHM_MLP_PRE = 1, DFHM_MLP_DZ = 2 };
dfhm_status dfhm_mlp_get_intermediate(dfhm_mlp *m, int32_t kind, int32_t layer, int64_t rows,
                                      uint16_t *host);
/* Training loss for n_out = 2F outputs (means mu_f, then log variances s_f,
 * f < F) and targets y_dev[batch][F] (FP32):
 * L = mean_b sum_f [ r^2 + sg(r^2) exp(-s_f) + s_f ], r = y_f - mu_f,
 * sg = no gradient (the means learn the targets, s_f learns the log of the
 * expected squared residual; the s_f train the output layer only, the
 * hidden layers learn from the means alone).  DFHM_E_STATE if n_out is odd.  gradients:
 * FP32 host array in logical order; loss (host) may be NULL. */
dfhm_status dfhm_mlp_gradients(dfhm_mlp *m, const uint16_t *x_dev, const float *y_dev,
                               int64_t batch, float *grad_host, float *loss);
/* One AdamW step with learning rate lr on the loss above. */
dfhm_status dfhm_mlp_train_step(dfhm_mlp *m, const uint16_t *x_dev, const float *y_dev,
                                int64_t batch, float lr, float *loss);
const char *dfhm_mlp_last_error(const dfhm_mlp *m);
void dfhm_mlp_destroy(dfhm_mlp *m);

/* Feature rows for the surrogate: for sample s of wall wall_dev[s] at time
 * t_dev[s] (s): n_hist samples every dt_hist of the side-0 outdoor T and RH
 * ending at t (oldest first), then 5 wall parameters params_dev[w][5] and 3
 * time features (t / 1 day, sin and cos of the time of day), each z-scored
 * with the given means / scales, zero-padded to stride (BF16).  sines_dev[w]
 * = (T mean, amp, period, phase, RH mean, amp, period, phase). */
typedef struct {
    int32_t n_hist, stride;
    float dt_hist, T_mean, T_scale, RH_mean, RH_scale;
    float p_mean[8], p_scale[8];
} dfhm_feature_desc;
dfhm_status dfhm_mlp_features(const int32_t *wall_dev, const double *t_dev, const double *sines_dev,
                              const float *params_dev, int64_t nsamp, const dfhm_feature_desc *fd,
                              uint16_t *x_dev, void *stream);
/* Decode the flux head (n_out = 8): per field f (heat, vapour) the network
 * predicts u_f = flux / RMS flux of the wall over the prediction windows and
 * l_f = log(RMS flux), normalised as value = mean + std * output with host
 * scale[8] = {mean, std} of u_q, u_g, l_q, l_g; outputs y_dev[b] = (u_q, u_g,
 * l_q, l_g, then their log variances).  flux_dev[b][f] = u_f exp(l_f) (heat
 * W/m2, vapour kg/(m2 s)); fallback_dev[b] = 1 when the predicted error
 * relative to the RMS flux, sd(u_f) + |u_f| sd(l_f), exceeds tau for either
 * field: those samples go back to the DF solver.  DFHM_E_INVAL on a
 * non-positive std or tau. */
dfhm_status dfhm_mlp_decode(const float *y_dev, int64_t batch, const float *scale, float tau,
                            float *flux_dev, uint8_t *fallback_dev, void *stream);
/* Decode an ensemble of n_nets networks trained on the same targets
 * (1 <= n_nets <= 4): y_dev is a host array of n_nets device output arrays,
 * each laid out as for dfhm_mlp_decode.  flux_dev[b][f] is the mean of the
 * members' u_f exp(l_f); the predicted error adds, in quadrature, the mean
 * of their sd(u_f) + |u_f| sd(l_f) and their disagreement (the population
 * standard deviation of the members' fluxes over exp of their mean l_f),
 * and is compared with tau as there; n_nets = 1 gives dfhm_mlp_decode's
 * results.  DFHM_E_INVAL as there, and for a null y_dev or
 * member or n_nets outside [1, 4]. */
dfhm_status dfhm_mlp_decode_ensemble(const float *const *y_dev, int32_t n_nets, int64_t batch,
                                     const float *scale, float tau, float *flux_dev,
                                     uint8_t *fallback_dev, void *stream);

/* Inference of the flux head (n_out = 8, see dfhm_mlp_decode) in one call:
 * the network on x_dev[batch][n_in] (BF16), then per sample the fluxes
 * flux_dev[b][2] (heat W/m2, vapour kg/(m2 s)) and the predicted error of
 * the sample relative to the wall's RMS flux, err_est_dev[b] = max over the
 * two fields of sd(u_f) + |u_f| sd(l_f): a sample whose estimate exceeds the
 * caller's threshold goes back to the DF solver.  scale as for
 * dfhm_mlp_decode.  Device pointers, queued on the network's stream.
 * DFHM_E_INVAL for a null pointer, a bad scale or batch outside
 * [1, max_batch]; DFHM_E_STATE when n_out != 8. */
dfhm_status dfhm_mlp_infer(dfhm_mlp *m, const uint16_t *x_dev, int64_t batch, const float *scale,
                           float *flux_dev, float *err_est_dev);

/* dfhm_mlp_infer over an ensemble of 1 to 4 networks with the same inputs
 * (n_in), stream and device: every member's forward pass on x_dev, then the
 * ensemble decode (as dfhm_mlp_decode_ensemble): flux_dev[b][f] the mean of
 * the members' fluxes, err_est_dev[b] the maximum over the two fields of the
 * ensemble's error estimate defined there.  Device pointers, queued on the members'
 * stream.  DFHM_E_INVAL for a null member, members that differ, n_nets
 * outside [1, 4], and as dfhm_mlp_infer for each member; the message goes
 * to the first member's dfhm_mlp_last_error. */
dfhm_status dfhm_mlp_infer_ensemble(dfhm_mlp *const *nets, int32_t n_nets, const uint16_t *x_dev,
                                    int64_t batch, const float *scale, float *flux_dev,
                                    float *err_est_dev);

/* dfhm_mlp_infer for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops): the same results, with the raw
 * outputs (and, for a network the one-launch inference kernel does not
 * cover, the hidden activations) in one statically allocated 64 MiB device
 * array per GPU instead of the network's buffers; it calls no allocator.
 * batch may not exceed dfhm_mlp_noalloc_max_batch(m) (DFHM_E_INVAL above it):
 * 524,280 rows at width 256 or 512, (64 MiB - 1 KiB) / (4 width + 128) at
 * other widths.  Calls on one GPU share that array: two calls
 * whose work overlaps on one GPU (different streams, or threads) race, and
 * the caller must order them.  Errors as dfhm_mlp_infer, and DFHM_E_DEVICE
 * if the array's address could not be resolved when the network was
 * created. */
dfhm_status dfhm_mlp_infer_noalloc(dfhm_mlp *m, const uint16_t *x_dev, int64_t batch,
                                   const float *scale, float *flux_dev, float *err_est_dev);
int64_t dfhm_mlp_noalloc_max_batch(const dfhm_mlp *m);

/* Checkpoint / restart.  dfhm_save writes the evolving state of a context —
 * its step index, both levels of every wall in the storage format (FP64
 * values, or the FP32 deviations), the flux state (applied fluxes, Neumaier
 * sums and compensations) and the zone air — into a host buffer after a
 * header (magic, version, precision, wall / node / zone counts and a digest of
 * everything else the run's future depends on: the run constants -- dt above
 * all, since levels n and n-1 are one dt apart in the recurrence -- the
 * material law and start-up mode, every input field of the wall descriptors,
 * the zone descriptors with their schedules and the zone links).  With buf ==
 * NULL it only stores the
 * required size in *bytes; otherwise *bytes must hold at least that size
 * (DFHM_E_INVAL) and receives the size written.  dfhm_load restores such a
 * buffer into a context created from the same configuration, walls, zones
 * and links (DFHM_E_INVAL otherwise, state unchanged), which then continues exactly as
 * the saving context would have: the DF recurrence only needs levels n and
 * n-1 (eq. dufort), and the ambient and zone schedules are functions of the
 * step index.  Both synchronise the context's stream; the caller owns buf. */
dfhm_status dfhm_save(dfhm_ctx *ctx, void *buf, size_t *bytes);
dfhm_status dfhm_load(dfhm_ctx *ctx, const void *buf, size_t bytes);

int64_t dfhm_step_index(const dfhm_ctx *ctx);
const char *dfhm_last_error(const dfhm_ctx *ctx);
const char *dfhm_status_string(dfhm_status s);
void dfhm_destroy(dfhm_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DFHM_H */
