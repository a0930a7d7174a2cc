/*
 * dfhm_ref.c -- plain FP64 CPU oracle for the Dufort-Frankel hygrothermal
 * wall / room method of Gasparin, Berger, Dutykh & Mendes, "An improved
 * explicit scheme for whole-building hygrothermal simulation" (arXiv
 * 1703.10119).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; both sides only receive the
 * same seeded input arrays.
 *
 * Everything is written to be read against the paper, not to be fast:
 *   - model: coupled moisture / energy balance in vapour-pressure form,
 *     Sec. 2, eq. (2.2) (label HAM_equation2), Robin surface exchange eq.
 *     (2.3) (HAM_BC), uniform initial state eq. (2.4) (HAM_ic);
 *   - nonlinear Dufort-Frankel update, Sec. 3.1, eqs. (3.2)-(3.5) (dufort,
 *     DF_NL, DF_NL_RHS) with face properties at the face-averaged state;
 *   - weakly coupled pair: moisture first, then heat with the new vapour
 *     pressure, App. A eqs. (A.3)-(A.5) (DF_eq1, DF_eq2b);
 *   - surface node: DF-averaged surface value in the Robin term, App. A eq.
 *     (A.6) (bc_v), written as a conservative half cell (equal to the ghost
 *     node of eqs. (A.7)-(A.8) for constant coefficients);
 *   - room air: lumped zone balance eq. (5.1) (LAV_equation) with the wall
 *     exchange terms eq. (5.2) (LAV_couplage), stepped by forward Euler with
 *     level-n surface values as in the explicit coupling of Sec. 5.3 eq.
 *     (5.6) (wbse_tn_exp);
 *   - implicit comparators (Euler implicit / Crank-Nicolson with fixed-point
 *     sub-iterations, Sec. 5.2 and Algorithm 1) used as fine-grid references.
 *
 * Readings where the paper is silent or garbled (all shared with the GPU
 * library by statement, not by code):
 *   - saturation pressure: Magnus form with the Alduchov-Eskridge (1996)
 *     constants 610.94 Pa, 17.625, 243.04 degC;
 *   - material law per layer, with phi = Pv / Ps(T) and theta = T - 273.15:
 *       k_TT = k0 (1 + aT phi),     k_M  = kM0 (1 + aM phi^2),
 *       k_TM = bTM k_M,             c_TT = c0 (1 + cT phi),
 *       c_M  = cM0 (1 + aC phi),    c_TM = (eTM + fTM theta) c_M;
 *     aT = aM = cT = aC = fTM = 0 gives the constant-coefficient walls of
 *     Sec. 6.1 (Table 2);
 *   - grid: x_j = j dx, dx = L/(Nx-1), both surfaces are nodes; node j
 *     belongs to the first layer whose right end is >= x_j; a face between
 *     nodes of different layers takes the harmonic mean of the two layers'
 *     laws evaluated at the face state;
 *   - side 0 is x = 0, side 1 is x = L; the boundary law is written with the
 *     outward normal, so fluxes are positive into the wall on both sides;
 *   - start of the three-level scheme: either m forward-Euler sub-steps of
 *     dt/m for the first step (m from the explicit stability bound at the
 *     initial state, with a safety factor 2), or u^{-1} := u^0;
 *   - radiation in the surface heat source q_inf of eq. (2.3) (Sec. 2): on
 *     every side, a constant part plus an incident flux max(0, sinusoid of
 *     t) (the paper's outside radiation is only shown in a figure); on a
 *     zone side, in addition, the long-wave exchange with the other surfaces
 *     of the zone, s eps sigma sum_w (T_w^4 - T^4), with s the zone's view
 *     factor, eps the emissivity of the receiving surface and T_w the
 *     zone-side surface temperatures of all walls of the zone.  Both are
 *     taken at t^n and level n, explicitly like the zone air; the start-up
 *     step holds the long-wave part at level 0 and re-evaluates the
 *     incident flux at every sub-step like the outdoor air;
 *   - inter-zone airflow (Sec. 5.1): a link exchanges g kg/s of dry air each
 *     way; zone i gains g (c_j theta_j - c_i theta_i) + L_v g (w_j - w_i) of
 *     heat and g (w_j - w_i) of vapour, with theta in degC (the enthalpy
 *     reference at which L_v is the latent heat) and c = c_pa + c_pv w the
 *     moist-air capacity of each zone, all at level n.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_MAXL 3
#define REF_PI 3.14159265358979323846

typedef struct {
    double thick;
    double k0, aT, kM0, aM, bTM, c0, cT, cM0, aC, eTM, fTM;
} ref_layer;

typedef struct { double mean, amp, period, phase; } ref_sine;

typedef struct {
    int32_t nx, n_layers;
    ref_layer layer[REF_MAXL];
    double hT[2], hM[2], qinf[2], ginf[2];
    ref_sine Tamb[2], RHamb[2];
    double T0, RH0, area;
    double emis[2];       /* emissivity of each surface (zone side only) */
    ref_sine qsun[2];     /* incident radiation, clipped at zero */
    int32_t law, pad_law; /* material law (set from the run's configuration) */
    double Lv, cw;        /* latent heat and water heat capacity (likewise) */
} ref_wall;

typedef struct {
    double volume, ach, T0, RH0;
    ref_sine Tout, RHout;
    int32_t n_sched;
    double sched_dt;
    const double *g_o;  /* kg/s, piecewise constant, periodic */
    const double *Q_h;  /* W */
    double view;        /* view factor s between two surfaces of the zone */
} ref_room;

typedef struct {
    double dt, Lv, cw, rho_a, c_pa, c_pv, Pv_ref;
    int32_t startup; /* 0 = forward-Euler sub-steps, 1 = repeat initial level */
    int32_t law;     /* 0 = shape law (scales x shape factors), 1 = Table 1 */
} ref_cfg;

/* ------------------------------------------------------------------ laws */

/* Saturation vapour pressure (Pa) of temperature T (K), Magnus form. */
double ref_psat(double T)
{
    double th = T - 273.15;
    return 610.94 * exp(17.625 * th / (th + 243.04));
}

typedef struct { double kTT, kM, kTM; } ref_kcoef;
typedef struct { double cTT, cM, cTM; } ref_ccoef;

/*
 * Table 1 (Sec. 6, the load-bearing material), read as follows:
 *   suction s = -P_c = -R_v T ln(phi) in J/kg (Kelvin's law with rho_l
 *   dropped, natural log: the printed c_M formula omits rho_l and carries
 *   the same c_1, c_2); s = 0 for phi >= 1;
 *   moisture content f = sum_i w_i [1 + (c_i s)^n_i]^(-m_i), (w, c, n) =
 *   (47.1, 1.25e-5, 1.65) and (109.9, 1.8e-5, 6), m_i = 1 - 1/n_i (the
 *   printed 0.39 and 0.83, and the printed c_M prefactors 30.62 = 47.1 m_1
 *   n_1 and 549.5 = 109.9 m_2 n_2);
 *   c_M = (df/dphi) / P_s (Sec. 2), the derivative taken exactly;
 *   c_TT = rho_0 c_0 + c_w f, rho_0 c_0 = 790 x 870; c_TM = c_w theta c_M;
 *   k_TT = lambda = 0.2 + 0.0045 f;
 *   delta_v = 1.88e-6 / T (1 - f/157) / (0.503 (1 - f/157)^2 + 0.497);
 *   k_TM = L_v delta_v;
 *   k_M = 1.97e-10 10^(1.44 - 0.07 log10(2 phi)) + 1.77e-7 exp(-8 (2 phi - 2)^2):
 *   the table's moisture transfer coefficient with its first exponential
 *   read in base 10 (its argument is a log10) and the square of the second
 *   inside the exponent.
 * Evaluated at 20 degC this reproduces every coefficient of Table 2 within
 * 1.5 % for the north and east/west walls (15 % and 50 % relative
 * humidity) and for the south wall at 75 %.
 * A layer's k0, kM0, c0 and cM0 multiply lambda, (k_M, k_TM), rho_0 c_0 and
 * (c_M, c_TM); 1 gives the paper's material.
 */
#define T1_RV 461.5
#define T1_RHO0C0 (790.0 * 870.0)

static double t1_suction(double T, double phi)
{
    double s = -T1_RV * T * log(phi);
    return s > 0.0 ? s : 0.0;
}

/* moisture content f (kg/m3) and df/dphi at (T, phi) */
static void t1_isotherm(double T, double phi, double *f, double *dfdphi)
{
    static const double w[2] = {47.1, 109.9}, c[2] = {1.25e-5, 1.8e-5}, n[2] = {1.65, 6.0};
    double s = t1_suction(T, phi);
    double F = 0.0, G = 0.0;      /* G = -df/ds */
    for (int i = 0; i < 2; ++i) {
        double m = 1.0 - 1.0 / n[i];
        double x = c[i] * s;
        double xn = pow(x, n[i]);
        F += w[i] * pow(1.0 + xn, -m);
        G += w[i] * m * n[i] * c[i] * pow(x, n[i] - 1.0) * pow(1.0 + xn, -m - 1.0);
    }
    *f = F;
    *dfdphi = G * T1_RV * T / phi;    /* ds/dphi = -R_v T / phi */
}

static double t1_delta_v(double T, double f)
{
    double u = 1.0 - f / 157.0;
    return 1.88e-6 / T * u / (0.503 * u * u + 0.497);
}

static double t1_moisture_k(double phi)
{
    double a = 2.0 * phi;
    return 1.97e-10 * pow(10.0, 1.44 - 0.07 * log10(a)) + 1.77e-7 * exp(-8.0 * (a - 2.0) * (a - 2.0));
}

static ref_kcoef law_k(const ref_wall *w, const ref_layer *m, double T, double P)
{
    ref_kcoef k;
    double phi = P / ref_psat(T);
    if (w->law == 1) {
        double f, df;
        t1_isotherm(T, phi, &f, &df);
        double dv = t1_delta_v(T, f);
        k.kTT = m->k0 * (0.2 + 0.0045 * f);
        k.kM = m->kM0 * t1_moisture_k(phi);
        k.kTM = m->kM0 * w->Lv * dv;
        return k;
    }
    k.kTT = m->k0 * (1.0 + m->aT * phi);
    k.kM = m->kM0 * (1.0 + m->aM * phi * phi);
    k.kTM = m->bTM * k.kM;
    return k;
}

static ref_ccoef law_c(const ref_wall *w, const ref_layer *m, double T, double P)
{
    ref_ccoef c;
    double phi = P / ref_psat(T);
    double th = T - 273.15;
    if (w->law == 1) {
        double f, df;
        t1_isotherm(T, phi, &f, &df);
        c.cTT = m->c0 * T1_RHO0C0 + w->cw * f;
        c.cM = m->cM0 * df / ref_psat(T);
        c.cTM = w->cw * th * c.cM;
        return c;
    }
    c.cTT = m->c0 * (1.0 + m->cT * phi);
    c.cM = m->cM0 * (1.0 + m->aC * phi);
    c.cTM = (m->eTM + m->fTM * th) * c.cM;
    return c;
}

/* Harmonic mean of two conductivities; zero when both are zero (a layer pair
 * without cross transport). */
static double harm(double a, double b)
{
    double s = a + b;
    return s > 0.0 ? 2.0 * a * b / s : 0.0;
}

/* Face coefficients between nodes j and j+1 (Sec. 3.1: properties at the
 * face-averaged state; harmonic mean across a layer interface). */
static ref_kcoef face_k(const ref_wall *w, const int *lay, const double *T,
                        const double *P, int j)
{
    double Tf = 0.5 * (T[j] + T[j + 1]);
    double Pf = 0.5 * (P[j] + P[j + 1]);
    ref_kcoef a = law_k(w, &w->layer[lay[j]], Tf, Pf);
    if (lay[j] == lay[j + 1]) return a;
    ref_kcoef b = law_k(w, &w->layer[lay[j + 1]], Tf, Pf);
    ref_kcoef k;
    k.kTT = harm(a.kTT, b.kTT);
    k.kM = harm(a.kM, b.kM);
    k.kTM = harm(a.kTM, b.kTM);
    return k;
}

static double sine_at(const ref_sine *s, double t)
{
    return s->mean + s->amp * sin(2.0 * REF_PI * t / s->period + s->phase);
}

/* Incident radiation (W/m2) on one side at time t: the sinusoid clipped at
 * zero (no negative absorbed flux). */
static double incident(const ref_wall *w, int side, double t)
{
    double q = sine_at(&w->qsun[side], t);
    return q > 0.0 ? q : 0.0;
}

#define REF_SIGMA 5.670374419e-8   /* Stefan-Boltzmann constant, W/(m2 K4) */

/* -------------------------------------------------------------- geometry */

static double wall_length(const ref_wall *w)
{
    double L = 0.0;
    for (int l = 0; l < w->n_layers; ++l) L += w->layer[l].thick;
    return L;
}

static void wall_layers(const ref_wall *w, int *lay)
{
    double L = wall_length(w);
    double dx = L / (double)(w->nx - 1);
    double right[REF_MAXL];
    double acc = 0.0;
    for (int l = 0; l < w->n_layers; ++l) { acc += w->layer[l].thick; right[l] = acc; }
    for (int j = 0; j < w->nx; ++j) {
        double x = (double)j * dx;
        int l = 0;
        while (l < w->n_layers - 1 && x > right[l]) ++l;
        lay[j] = l;
    }
}

/* ----------------------------------------------------- compensated sums */

/* Neumaier (1974) compensated accumulation: s + c carries the sum. */
static void neumaier_add(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
    else *c += (x - t) + *s;
    *s = t;
}

/* ------------------------------------------------------------ simulation */

typedef struct {
    ref_cfg cfg;
    int64_t nw, nr;
    ref_wall *walls;
    ref_room *rooms;
    double *sched;            /* copies of the room schedules */
    int64_t *wall_room;       /* -1 = none */
    int8_t *room_side;
    int64_t *off;             /* node offset of each wall */
    int *lay;                 /* layer of each node */
    double *Tp, *Tc, *Pp, *Pc;/* levels n-1 and n */
    double *fnow;             /* [w][side][field] applied flux of last step */
    double *fsum, *fcmp;      /* Neumaier pairs of the flux integrals */
    double *Ta, *Pa;          /* room air at level n */
    int64_t nl;               /* inter-zone links: zones la[l], lb[l], flow lg[l] */
    int32_t *la, *lb;
    double *lg;
    int64_t n;
} ref_sim;

void ref_destroy(ref_sim *s)
{
    if (!s) return;
    free(s->walls); free(s->rooms); free(s->sched); free(s->wall_room);
    free(s->room_side); free(s->off); free(s->lay);
    free(s->Tp); free(s->Tc); free(s->Pp); free(s->Pc);
    free(s->fnow); free(s->fsum); free(s->fcmp); free(s->Ta); free(s->Pa);
    free(s->la); free(s->lb); free(s->lg);
    free(s);
}

/* Air exchanged between zones (Sec. 5.1, the inter-zone sources): link l
 * moves lg[l] kg/s of dry air from zone la[l] to zone lb[l] and the same back.
 * Replaces any previous links. */
int ref_set_links(ref_sim *s, const int32_t *a, const int32_t *b, const double *g, int64_t n)
{
    free(s->la); free(s->lb); free(s->lg);
    s->nl = n;
    s->la = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    s->lb = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    s->lg = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t l = 0; l < n; ++l) { s->la[l] = a[l]; s->lb[l] = b[l]; s->lg[l] = g[l]; }
    return 0;
}

ref_sim *ref_create(const ref_cfg *cfg, const ref_wall *walls, int64_t nw,
                    const ref_room *rooms, int64_t nr, const int64_t *wall_room,
                    const int8_t *room_side)
{
    ref_sim *s = (ref_sim *)calloc(1, sizeof(ref_sim));
    if (!s) return NULL;
    s->cfg = *cfg;
    s->nw = nw;
    s->nr = nr;
    s->walls = (ref_wall *)malloc(sizeof(ref_wall) * (size_t)(nw > 0 ? nw : 1));
    memcpy(s->walls, walls, sizeof(ref_wall) * (size_t)nw);
    for (int64_t w = 0; w < nw; ++w) {
        s->walls[w].law = cfg->law;
        s->walls[w].Lv = cfg->Lv;
        s->walls[w].cw = cfg->cw;
    }
    s->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nw + 1));
    s->off[0] = 0;
    for (int64_t w = 0; w < nw; ++w) s->off[w + 1] = s->off[w] + walls[w].nx;
    int64_t N = s->off[nw];
    size_t nb = sizeof(double) * (size_t)(N > 0 ? N : 1);
    s->lay = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    s->Tp = (double *)malloc(nb); s->Tc = (double *)malloc(nb);
    s->Pp = (double *)malloc(nb); s->Pc = (double *)malloc(nb);
    size_t nf = sizeof(double) * (size_t)(4 * (nw > 0 ? nw : 1));
    s->fnow = (double *)calloc(1, nf);
    s->fsum = (double *)calloc(1, nf);
    s->fcmp = (double *)calloc(1, nf);
    s->wall_room = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nw > 0 ? nw : 1));
    s->room_side = (int8_t *)malloc((size_t)(nw > 0 ? nw : 1));
    for (int64_t w = 0; w < nw; ++w) {
        s->wall_room[w] = wall_room ? wall_room[w] : -1;
        s->room_side[w] = room_side ? room_side[w] : 1;
    }
    for (int64_t w = 0; w < nw; ++w) {
        const ref_wall *wl = &walls[w];
        int64_t o = s->off[w];
        wall_layers(wl, s->lay + o);
        double P0 = wl->RH0 * ref_psat(wl->T0);
        for (int j = 0; j < wl->nx; ++j) {
            s->Tc[o + j] = wl->T0; s->Pc[o + j] = P0;
            s->Tp[o + j] = wl->T0; s->Pp[o + j] = P0;
        }
    }
    /* rooms: copy schedules */
    int64_t tot = 0;
    for (int64_t r = 0; r < nr; ++r) tot += rooms[r].n_sched;
    s->rooms = (ref_room *)malloc(sizeof(ref_room) * (size_t)(nr > 0 ? nr : 1));
    s->sched = (double *)malloc(sizeof(double) * (size_t)(2 * tot + 1));
    s->Ta = (double *)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
    s->Pa = (double *)malloc(sizeof(double) * (size_t)(nr > 0 ? nr : 1));
    int64_t k = 0;
    for (int64_t r = 0; r < nr; ++r) {
        s->rooms[r] = rooms[r];
        int ns = rooms[r].n_sched;
        memcpy(s->sched + k, rooms[r].g_o, sizeof(double) * (size_t)ns);
        memcpy(s->sched + k + ns, rooms[r].Q_h, sizeof(double) * (size_t)ns);
        s->rooms[r].g_o = s->sched + k;
        s->rooms[r].Q_h = s->sched + k + ns;
        k += 2 * ns;
        s->Ta[r] = rooms[r].T0;
        s->Pa[r] = rooms[r].RH0 * ref_psat(rooms[r].T0);
    }
    s->n = 0;
    return s;
}

/* Ambient (T_inf, P_inf) seen by one side of wall w at time t: the outdoor
 * sinusoids of that side, or the room air of level n on a room side. */
static void ambient(const ref_sim *s, int64_t w, int side, double t,
                    const double *Ta, const double *Pa, double *Tinf, double *Pinf)
{
    const ref_wall *wl = &s->walls[w];
    int64_t r = s->wall_room[w];
    if (r >= 0 && s->room_side[w] == side) {
        *Tinf = Ta[r];
        *Pinf = Pa[r];
    } else {
        double T = sine_at(&wl->Tamb[side], t);
        double RH = sine_at(&wl->RHamb[side], t);
        *Tinf = T;
        *Pinf = RH * ref_psat(T);
    }
}

/*
 * One Dufort-Frankel step n -> n+1 of one wall.
 * Inputs: levels n-1 (Tp, Pp) and n (Tc, Pc); ambient at t^n.
 * Output: level n+1 in (Tn, Pn) and the applied surface fluxes.
 *
 * With r = dt/dx^2, s = dt/dx, K = k(j-1/2) + k(j+1/2):
 *  interior moisture (eq. DF_NL with u_j^n -> (u^{n+1}+u^{n-1})/2):
 *    (c_M + r K_M) P+ = (c_M - r K_M) P- + 2 r (k_M+ P_{j+1} + k_M- P_{j-1})
 *  interior heat, after moisture (App. A, eq. DF_eq2b with variable
 *  coefficients):
 *    (c_TT + r K_T) T+ = (c_TT - r K_T) T- + 2 r (k_TT+ T_{j+1} + k_TT- T_{j-1})
 *        + (c_TM - r K_TM) P- - (c_TM + r K_TM) P+ + 2 r (k_TM+ P_{j+1} + k_TM- P_{j-1})
 *  surface node (half cell of width dx/2; DF-averaged surface value in the
 *  Robin term, eq. bc_v; k = the single inner face, P_nb the inner node):
 *    (c_M + 2rk + 2s h_M) P+ = (c_M - 2rk - 2s h_M) P- + 4rk P_nb + 4s (h_M P_inf + g_inf)
 *    (c_TT + 2rk_TT + 2s h_T) T+ = (c_TT - 2rk_TT - 2s h_T) T- + 4rk_TT T_nb + 4s h_T T_inf
 *        + (c_TM - 2rk_TM - 2s Lv h_M) P- - (c_TM + 2rk_TM + 2s Lv h_M) P+
 *        + 4rk_TM P_nb + 4s Lv h_M P_inf + 4s q_inf
 *  where q_inf = the wall's constant source + qx (radiation at t^n, level n).
 */
static void df_wall_step(const ref_wall *w, const int *lay, double dt, double Lv,
                         const double *Tp, const double *Tc, const double *Pp,
                         const double *Pc, double *Tn, double *Pn,
                         const double Tinf[2], const double Pinf[2], const double qx[2],
                         double flux[2][2], ref_kcoef *kf /* scratch nx-1 */)
{
    int nx = w->nx;
    double dx = wall_length(w) / (double)(nx - 1);
    double r = dt / (dx * dx);
    double sd = dt / dx;
    for (int j = 0; j < nx - 1; ++j) kf[j] = face_k(w, lay, Tc, Pc, j);

    /* moisture first */
    for (int j = 0; j < nx; ++j) {
        ref_ccoef c = law_c(w, &w->layer[lay[j]], Tc[j], Pc[j]);
        if (j > 0 && j < nx - 1) {
            double KM = kf[j - 1].kM + kf[j].kM;
            Pn[j] = ((c.cM - r * KM) * Pp[j]
                     + 2.0 * r * (kf[j].kM * Pc[j + 1] + kf[j - 1].kM * Pc[j - 1]))
                    / (c.cM + r * KM);
        } else {
            int side = (j == 0) ? 0 : 1;
            int jf = (j == 0) ? 0 : nx - 2;     /* inner face */
            int jn = (j == 0) ? 1 : nx - 2;     /* inner neighbour */
            double k = kf[jf].kM, h = w->hM[side];
            Pn[j] = ((c.cM - 2.0 * r * k - 2.0 * sd * h) * Pp[j]
                     + 4.0 * r * k * Pc[jn]
                     + 4.0 * sd * (h * Pinf[side] + w->ginf[side]))
                    / (c.cM + 2.0 * r * k + 2.0 * sd * h);
        }
    }
    /* then heat, using the new vapour pressure */
    for (int j = 0; j < nx; ++j) {
        ref_ccoef c = law_c(w, &w->layer[lay[j]], Tc[j], Pc[j]);
        if (j > 0 && j < nx - 1) {
            double KT = kf[j - 1].kTT + kf[j].kTT;
            double KX = kf[j - 1].kTM + kf[j].kTM;
            double rhs = (c.cTT - r * KT) * Tp[j]
                       + 2.0 * r * (kf[j].kTT * Tc[j + 1] + kf[j - 1].kTT * Tc[j - 1])
                       + (c.cTM - r * KX) * Pp[j]
                       - (c.cTM + r * KX) * Pn[j]
                       + 2.0 * r * (kf[j].kTM * Pc[j + 1] + kf[j - 1].kTM * Pc[j - 1]);
            Tn[j] = rhs / (c.cTT + r * KT);
        } else {
            int side = (j == 0) ? 0 : 1;
            int jf = (j == 0) ? 0 : nx - 2;
            int jn = (j == 0) ? 1 : nx - 2;
            double kT = kf[jf].kTT, kX = kf[jf].kTM;
            double hT = w->hT[side], hL = Lv * w->hM[side];
            double rhs = (c.cTT - 2.0 * r * kT - 2.0 * sd * hT) * Tp[j]
                       + 4.0 * r * kT * Tc[jn] + 4.0 * sd * hT * Tinf[side]
                       + (c.cTM - 2.0 * r * kX - 2.0 * sd * hL) * Pp[j]
                       - (c.cTM + 2.0 * r * kX + 2.0 * sd * hL) * Pn[j]
                       + 4.0 * r * kX * Pc[jn] + 4.0 * sd * hL * Pinf[side]
                       + 4.0 * sd * (w->qinf[side] + qx[side]);
            Tn[j] = rhs / (c.cTT + 2.0 * r * kT + 2.0 * sd * hT);
        }
    }
    /* applied surface fluxes (positive into the wall), eq. HAM_BC with the
     * DF-averaged surface values */
    for (int side = 0; side < 2; ++side) {
        int j = side == 0 ? 0 : nx - 1;
        double Ts = 0.5 * (Tn[j] + Tp[j]);
        double Ps = 0.5 * (Pn[j] + Pp[j]);
        double g = w->hM[side] * (Pinf[side] - Ps) + w->ginf[side];
        double q = w->hT[side] * (Tinf[side] - Ts)
                 + Lv * w->hM[side] * (Pinf[side] - Ps) + (w->qinf[side] + qx[side]);
        flux[side][0] = q;
        flux[side][1] = g;
    }
}

/* Explicit stability bound (s) of forward Euler for one wall at its current
 * level n: min over nodes of capacity / conductance for both fields, the
 * dimensional counterpart of eqs. (4.1)-(4.2) (cfl_heat_Eq, cfl_moisture_Eq),
 * with the surface exchange included in the surface conductance. */
static double ftcs_bound(const ref_wall *w, const int *lay, const double *T,
                         const double *P, ref_kcoef *kf)
{
    int nx = w->nx;
    double dx = wall_length(w) / (double)(nx - 1);
    for (int j = 0; j < nx - 1; ++j) kf[j] = face_k(w, lay, T, P, j);
    double best = INFINITY;
    for (int j = 0; j < nx; ++j) {
        ref_ccoef c = law_c(w, &w->layer[lay[j]], T[j], P[j]);
        double width = (j == 0 || j == nx - 1) ? 0.5 * dx : dx;
        double gT = 0.0, gM = 0.0;
        if (j > 0) { gT += kf[j - 1].kTT / dx; gM += kf[j - 1].kM / dx; }
        if (j < nx - 1) { gT += kf[j].kTT / dx; gM += kf[j].kM / dx; }
        if (j == 0) { gT += w->hT[0]; gM += w->hM[0]; }
        if (j == nx - 1) { gT += w->hT[1]; gM += w->hM[1]; }
        double bT = c.cTT * width / gT;
        double bM = c.cM * width / gM;
        if (bT < best) best = bT;
        if (bM < best) best = bM;
    }
    return best;
}

/* Number of forward-Euler sub-steps for the start-up step: ceil(2 dt / b),
 * at least 1 and at most 2^20 (a zero or non-finite bound gives 1 or the cap). */
#define REF_MAX_SUBSTEPS ((int64_t)1 << 20)
static int64_t ftcs_substeps(double dt, double bound)
{
    double m = ceil(2.0 * dt / bound);
    if (!(m >= 1.0)) return 1;
    if (m > (double)REF_MAX_SUBSTEPS) return REF_MAX_SUBSTEPS;
    return (int64_t)m;
}

/*
 * Start-up step 0 -> 1 by m forward-Euler sub-steps of dt/m (same half-cell
 * balance as the DF step with the time derivative taken forward and every
 * value at the sub-step start).  Coefficients and the outdoor ambient are
 * re-evaluated at every sub-step; a room side sees the level-0 room air.
 */
static void ftcs_startup(const ref_sim *s, int64_t w, const int *lay, double *T,
                         double *P, double *Tw, double *Pw, ref_kcoef *kf,
                         const double qlw[2], double flux_now[2][2], double *fsum,
                         double *fcmp)
{
    const ref_wall *wl = &s->walls[w];
    int nx = wl->nx;
    double dt = s->cfg.dt, Lv = s->cfg.Lv;
    double dx = wall_length(wl) / (double)(nx - 1);
    int64_t m = ftcs_substeps(dt, ftcs_bound(wl, lay, T, P, kf));
    double dts = dt / (double)m;
    double acc[2][2] = {{0, 0}, {0, 0}};
    for (int64_t k = 0; k < m; ++k) {
        double t = (double)k * dt / (double)m;
        double Tinf[2], Pinf[2], qs[2];
        for (int side = 0; side < 2; ++side) {
            ambient(s, w, side, t, s->Ta, s->Pa, &Tinf[side], &Pinf[side]);
            qs[side] = wl->qinf[side] + (incident(wl, side, t) + qlw[side]);
        }
        for (int j = 0; j < nx - 1; ++j) kf[j] = face_k(wl, lay, T, P, j);
        /* fluxes applied during this sub-step (surface value at its start) */
        for (int side = 0; side < 2; ++side) {
            int j = side == 0 ? 0 : nx - 1;
            double g = wl->hM[side] * (Pinf[side] - P[j]) + wl->ginf[side];
            double q = wl->hT[side] * (Tinf[side] - T[j])
                     + Lv * wl->hM[side] * (Pinf[side] - P[j]) + qs[side];
            neumaier_add(&fsum[side * 2 + 0], &fcmp[side * 2 + 0], dts * q);
            neumaier_add(&fsum[side * 2 + 1], &fcmp[side * 2 + 1], dts * g);
            acc[side][0] += q;
            acc[side][1] += g;
        }
        for (int j = 0; j < nx; ++j) {
            ref_ccoef c = law_c(wl, &wl->layer[lay[j]], T[j], P[j]);
            double width = (j == 0 || j == nx - 1) ? 0.5 * dx : dx;
            double dM = 0.0, dT = 0.0;
            if (j > 0) {
                dM += kf[j - 1].kM * (P[j - 1] - P[j]) / dx;
                dT += kf[j - 1].kTT * (T[j - 1] - T[j]) / dx
                    + kf[j - 1].kTM * (P[j - 1] - P[j]) / dx;
            }
            if (j < nx - 1) {
                dM += kf[j].kM * (P[j + 1] - P[j]) / dx;
                dT += kf[j].kTT * (T[j + 1] - T[j]) / dx
                    + kf[j].kTM * (P[j + 1] - P[j]) / dx;
            }
            if (j == 0 || j == nx - 1) {
                int side = j == 0 ? 0 : 1;
                dM += wl->hM[side] * (Pinf[side] - P[j]) + wl->ginf[side];
                dT += wl->hT[side] * (Tinf[side] - T[j])
                    + Lv * wl->hM[side] * (Pinf[side] - P[j]) + qs[side];
            }
            double Pnew = P[j] + dts * dM / (c.cM * width);
            /* c_TT dT/dt + c_TM dP/dt = (heat flux divergence) */
            double Tnew = T[j] + (dts * dT / width - c.cTM * (Pnew - P[j])) / c.cTT;
            Pw[j] = Pnew;
            Tw[j] = Tnew;
        }
        memcpy(T, Tw, sizeof(double) * (size_t)nx);
        memcpy(P, Pw, sizeof(double) * (size_t)nx);
    }
    for (int side = 0; side < 2; ++side)
        for (int f = 0; f < 2; ++f) flux_now[side][f] = acc[side][f] / (double)m;
}

/* Long-wave exchange (W/m2, into the wall) received by the zone-side surface
 * of wall w from the zone-side surfaces of all walls of its zone (Sec. 2,
 * boundary conditions), at the level-n surface temperatures; 0 on a wall
 * without a zone. */
static double longwave(const ref_sim *s, int64_t w)
{
    int64_t r = s->wall_room[w];
    if (r < 0) return 0.0;
    const ref_wall *wl = &s->walls[w];
    int side = s->room_side[w];
    double T = s->Tc[s->off[w] + (side == 0 ? 0 : wl->nx - 1)];
    double sum = 0.0;
    for (int64_t v = 0; v < s->nw; ++v) {
        if (s->wall_room[v] != r) continue;
        const ref_wall *vl = &s->walls[v];
        double Tv = s->Tc[s->off[v] + (s->room_side[v] == 0 ? 0 : vl->nx - 1)];
        sum += Tv * Tv * Tv * Tv - T * T * T * T;
    }
    return s->rooms[r].view * wl->emis[side] * REF_SIGMA * sum;
}

/* Room air at step n -> n+1 by forward Euler (eq. LAV_equation with
 * w ~ Pv / Pv_ref, exchange terms eq. LAV_couplage at the level-n wall
 * surface values, inter-zone airflow at the level-n air of the linked
 * zones, sources at t^n). */
static void room_step(const ref_sim *s, int64_t r, double t, double *Ta_new,
                      double *Pa_new)
{
    const ref_room *rm = &s->rooms[r];
    const ref_cfg *c = &s->cfg;
    double Ta = s->Ta[r], Pa = s->Pa[r];
    double mass = c->rho_a * rm->volume;                /* kg of air */
    double gv = rm->ach * mass / 3600.0;                /* kg/s */
    double cma = c->c_pa + c->c_pv * Pa / c->Pv_ref;    /* J/(kg K) */
    int64_t slot = (int64_t)floor(t / rm->sched_dt) % rm->n_sched;
    double go = rm->g_o[slot], Qh = rm->Q_h[slot];
    double Tout = sine_at(&rm->Tout, t);
    double Pout = sine_at(&rm->RHout, t) * ref_psat(Tout);
    double G = go + gv * (Pout - Pa) / c->Pv_ref;
    double Q = Qh + c->Lv * go + gv * cma * (Tout - Ta)
             + c->Lv * gv * (Pout - Pa) / c->Pv_ref;
    for (int64_t w = 0; w < s->nw; ++w) {
        if (s->wall_room[w] != r) continue;
        const ref_wall *wl = &s->walls[w];
        int side = s->room_side[w];
        int64_t j = s->off[w] + (side == 0 ? 0 : wl->nx - 1);
        double Ts = s->Tc[j], Ps = s->Pc[j];
        G += wl->area * wl->hM[side] * (Ps - Pa);
        Q += wl->area * (wl->hT[side] * (Ts - Ta) + c->Lv * wl->hM[side] * (Ps - Pa));
    }
    /* inter-zone airflow from each linked zone j (level n): the moist-air
     * enthalpy c_j theta_j - c_i theta_i (theta in degC, c = c_pa + c_pv w) and
     * the latent part L_v (w_j - w_i) */
    for (int64_t l = 0; l < s->nl; ++l) {
        int64_t j;
        if (s->la[l] == r) j = s->lb[l];
        else if (s->lb[l] == r) j = s->la[l];
        else continue;
        double g = s->lg[l];
        double Tj = s->Ta[j], Pj = s->Pa[j];
        double cj = c->c_pa + c->c_pv * Pj / c->Pv_ref;
        G += g * (Pj - Pa) / c->Pv_ref;
        Q += g * (cj * (Tj - 273.15) - cma * (Ta - 273.15)) + c->Lv * g * (Pj - Pa) / c->Pv_ref;
    }
    *Pa_new = Pa + c->dt * G / (mass / c->Pv_ref);
    *Ta_new = Ta + c->dt * Q / (mass * cma);
}

/* Advance the whole simulation by nsteps steps. */
int ref_step(ref_sim *s, int64_t nsteps, int nthreads)
{
    int64_t maxnx = 1;
    for (int64_t w = 0; w < s->nw; ++w)
        if (s->walls[w].nx > maxnx) maxnx = s->walls[w].nx;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
    double *Ta_new = (double *)malloc(sizeof(double) * (size_t)(s->nr > 0 ? s->nr : 1));
    double *Pa_new = (double *)malloc(sizeof(double) * (size_t)(s->nr > 0 ? s->nr : 1));
    double *qlw = (double *)malloc(sizeof(double) * (size_t)(s->nw > 0 ? s->nw : 1));
    for (int64_t it = 0; it < nsteps; ++it) {
        double t = (double)s->n * s->cfg.dt;
        for (int64_t r = 0; r < s->nr; ++r) room_step(s, r, t, &Ta_new[r], &Pa_new[r]);
        for (int64_t w = 0; w < s->nw; ++w) qlw[w] = longwave(s, w);
#pragma omp parallel
        {
            ref_kcoef *kf = (ref_kcoef *)malloc(sizeof(ref_kcoef) * (size_t)maxnx);
            double *Tw = (double *)malloc(sizeof(double) * (size_t)maxnx);
            double *Pw = (double *)malloc(sizeof(double) * (size_t)maxnx);
            double *Tx = (double *)malloc(sizeof(double) * (size_t)maxnx);
            double *Px = (double *)malloc(sizeof(double) * (size_t)maxnx);
#pragma omp for schedule(dynamic, 16)
            for (int64_t w = 0; w < s->nw; ++w) {
                const ref_wall *wl = &s->walls[w];
                int64_t o = s->off[w];
                int nx = wl->nx;
                double *fs = s->fsum + 4 * w, *fc = s->fcmp + 4 * w;
                double fl[2][2];
                /* long-wave part on the zone side only (level n) */
                double ql[2] = {0.0, 0.0};
                if (s->wall_room[w] >= 0) ql[s->room_side[w]] = qlw[w];
                if (s->n == 0 && s->cfg.startup == 0) {
                    memcpy(Tx, s->Tc + o, sizeof(double) * (size_t)nx);
                    memcpy(Px, s->Pc + o, sizeof(double) * (size_t)nx);
                    ftcs_startup(s, w, s->lay + o, Tx, Px, Tw, Pw, kf, ql, fl, fs, fc);
                    memcpy(s->Tp + o, s->Tc + o, sizeof(double) * (size_t)nx);
                    memcpy(s->Pp + o, s->Pc + o, sizeof(double) * (size_t)nx);
                    memcpy(s->Tc + o, Tx, sizeof(double) * (size_t)nx);
                    memcpy(s->Pc + o, Px, sizeof(double) * (size_t)nx);
                } else {
                    if (s->n == 0) { /* repeat start: u^{-1} := u^0 */
                        memcpy(s->Tp + o, s->Tc + o, sizeof(double) * (size_t)nx);
                        memcpy(s->Pp + o, s->Pc + o, sizeof(double) * (size_t)nx);
                    }
                    double Tinf[2], Pinf[2], qx[2];
                    for (int side = 0; side < 2; ++side) {
                        ambient(s, w, side, t, s->Ta, s->Pa, &Tinf[side], &Pinf[side]);
                        qx[side] = incident(wl, side, t) + ql[side];
                    }
                    df_wall_step(wl, s->lay + o, s->cfg.dt, s->cfg.Lv,
                                 s->Tp + o, s->Tc + o, s->Pp + o, s->Pc + o,
                                 Tw, Pw, Tinf, Pinf, qx, fl, kf);
                    /* rotate: n -> n-1, n+1 -> n */
                    memcpy(s->Tp + o, s->Tc + o, sizeof(double) * (size_t)nx);
                    memcpy(s->Pp + o, s->Pc + o, sizeof(double) * (size_t)nx);
                    memcpy(s->Tc + o, Tw, sizeof(double) * (size_t)nx);
                    memcpy(s->Pc + o, Pw, sizeof(double) * (size_t)nx);
                    for (int side = 0; side < 2; ++side)
                        for (int f = 0; f < 2; ++f)
                            neumaier_add(&fs[side * 2 + f], &fc[side * 2 + f],
                                         s->cfg.dt * fl[side][f]);
                }
                for (int side = 0; side < 2; ++side)
                    for (int f = 0; f < 2; ++f) s->fnow[4 * w + side * 2 + f] = fl[side][f];
            }
            free(kf); free(Tw); free(Pw); free(Tx); free(Px);
        }
        for (int64_t r = 0; r < s->nr; ++r) { s->Ta[r] = Ta_new[r]; s->Pa[r] = Pa_new[r]; }
        s->n += 1;
    }
    free(Ta_new);
    free(Pa_new);
    free(qlw);
    return 0;
}

/* ------------------------------------------------------------- accessors */

int64_t ref_step_index(const ref_sim *s) { return s->n; }
/* Set the step index (so that a run can start from two given levels). */
void ref_set_step_index(ref_sim *s, int64_t n) { s->n = n; }
int64_t ref_total_nodes(const ref_sim *s) { return s->off[s->nw]; }

int ref_get_fields(const ref_sim *s, int64_t w, int level, double *T, double *P)
{
    if (w < 0 || w >= s->nw) return 1;
    int64_t o = s->off[w];
    int nx = s->walls[w].nx;
    const double *Ts = level == 0 ? s->Tc : s->Tp;
    const double *Ps = level == 0 ? s->Pc : s->Pp;
    memcpy(T, Ts + o, sizeof(double) * (size_t)nx);
    memcpy(P, Ps + o, sizeof(double) * (size_t)nx);
    return 0;
}

int ref_set_fields(ref_sim *s, int64_t w, int level, const double *T, const double *P)
{
    if (w < 0 || w >= s->nw) return 1;
    int64_t o = s->off[w];
    int nx = s->walls[w].nx;
    double *Ts = level == 0 ? s->Tc : s->Tp;
    double *Ps = level == 0 ? s->Pc : s->Pp;
    memcpy(Ts + o, T, sizeof(double) * (size_t)nx);
    memcpy(Ps + o, P, sizeof(double) * (size_t)nx);
    return 0;
}

/* now / integral: [n_walls][2 sides][2 fields (heat W/m2, vapour kg/m2 s)] */
void ref_get_fluxes(const ref_sim *s, double *now, double *integral)
{
    for (int64_t i = 0; i < 4 * s->nw; ++i) {
        if (now) now[i] = s->fnow[i];
        if (integral) integral[i] = s->fsum[i] + s->fcmp[i];
    }
}

void ref_get_rooms(const ref_sim *s, double *Ta, double *Pa)
{
    for (int64_t r = 0; r < s->nr; ++r) { Ta[r] = s->Ta[r]; Pa[r] = s->Pa[r]; }
}

void ref_get_layers(const ref_sim *s, int64_t w, int32_t *lay)
{
    int64_t o = s->off[w];
    for (int j = 0; j < s->walls[w].nx; ++j) lay[j] = s->lay[o + j];
}

/* Coefficients used by the next step of wall w (state at level n):
 * node[nx][3] = (c_TT, c_M, c_TM), face[nx-1][3] = (k_TT, k_M, k_TM). */
void ref_get_coeffs(const ref_sim *s, int64_t w, double *node, double *face)
{
    const ref_wall *wl = &s->walls[w];
    int64_t o = s->off[w];
    const int *lay = s->lay + o;
    for (int j = 0; j < wl->nx; ++j) {
        ref_ccoef c = law_c(wl, &wl->layer[lay[j]], s->Tc[o + j], s->Pc[o + j]);
        node[3 * j] = c.cTT; node[3 * j + 1] = c.cM; node[3 * j + 2] = c.cTM;
    }
    for (int j = 0; j < wl->nx - 1; ++j) {
        ref_kcoef k = face_k(wl, lay, s->Tc + o, s->Pc + o, j);
        face[3 * j] = k.kTT; face[3 * j + 1] = k.kM; face[3 * j + 2] = k.kTM;
    }
}

/* Start-up sub-step count the first step of wall w would use. */
int64_t ref_startup_substeps(const ref_sim *s, int64_t w)
{
    const ref_wall *wl = &s->walls[w];
    int64_t o = s->off[w];
    ref_kcoef *kf = (ref_kcoef *)malloc(sizeof(ref_kcoef) * (size_t)wl->nx);
    double b = ftcs_bound(wl, s->lay + o, s->Tc + o, s->Pc + o, kf);
    free(kf);
    return ftcs_substeps(s->cfg.dt, b);
}

/* ==================================================================== */
/* Implicit comparator: theta-scheme (1 = Euler implicit, 1/2 = Crank-   */
/* Nicolson) with fixed-point sub-iterations on the coefficients, one    */
/* wall with outdoor ambient on both sides (Sec. 5.2, Algorithm 1; the   */
/* fixed point stops when the max change of both fields, relative to the */
/* field scale, drops below eta).                                        */
/* ==================================================================== */

static void thomas(int n, double *a, double *b, double *c, double *d, double *x)
{
    /* a: sub, b: diag, c: super; overwrites b, d */
    for (int i = 1; i < n; ++i) {
        double m = a[i] / b[i - 1];
        b[i] -= m * c[i - 1];
        d[i] -= m * d[i - 1];
    }
    x[n - 1] = d[n - 1] / b[n - 1];
    for (int i = n - 2; i >= 0; --i) x[i] = (d[i] - c[i] * x[i + 1]) / b[i];
}

/*
 * Run nsteps of the theta-scheme from the wall's uniform initial state.
 * Fields at the end go to T, P (length nx).  Returns the mean number of
 * fixed-point iterations per step.  Coefficients are evaluated at the
 * theta-weighted state between level n and the current iterate.
 */
double ref_implicit_run(const ref_wall *w, double dt, double Lv, int64_t nsteps,
                        double theta, double eta, double *T, double *P)
{
    int nx = w->nx;
    double dx = wall_length(w) / (double)(nx - 1);
    int *lay = (int *)malloc(sizeof(int) * (size_t)nx);
    wall_layers(w, lay);
    double *To = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Po = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Tk = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Pk = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Ts = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Ps = (double *)malloc(sizeof(double) * (size_t)nx);
    double *a = (double *)malloc(sizeof(double) * (size_t)nx);
    double *b = (double *)malloc(sizeof(double) * (size_t)nx);
    double *c = (double *)malloc(sizeof(double) * (size_t)nx);
    double *d = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Pn = (double *)malloc(sizeof(double) * (size_t)nx);
    double *Tn = (double *)malloc(sizeof(double) * (size_t)nx);
    ref_kcoef *kf = (ref_kcoef *)malloc(sizeof(ref_kcoef) * (size_t)nx);
    ref_ccoef *cn = (ref_ccoef *)malloc(sizeof(ref_ccoef) * (size_t)nx);
    double P0 = w->RH0 * ref_psat(w->T0);
    for (int j = 0; j < nx; ++j) { T[j] = w->T0; P[j] = P0; }
    double iters = 0.0;
    for (int64_t n = 0; n < nsteps; ++n) {
        double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
        double Ti0[2], Pi0[2], Ti1[2], Pi1[2];
        for (int side = 0; side < 2; ++side) {
            Ti0[side] = sine_at(&w->Tamb[side], t0);
            Pi0[side] = sine_at(&w->RHamb[side], t0) * ref_psat(Ti0[side]);
            Ti1[side] = sine_at(&w->Tamb[side], t1);
            Pi1[side] = sine_at(&w->RHamb[side], t1) * ref_psat(Ti1[side]);
        }
        memcpy(To, T, sizeof(double) * (size_t)nx);
        memcpy(Po, P, sizeof(double) * (size_t)nx);
        memcpy(Tk, T, sizeof(double) * (size_t)nx);
        memcpy(Pk, P, sizeof(double) * (size_t)nx);
        int it = 0;
        for (;;) {
            ++it;
            for (int j = 0; j < nx; ++j) {
                Ts[j] = theta * Tk[j] + (1.0 - theta) * To[j];
                Ps[j] = theta * Pk[j] + (1.0 - theta) * Po[j];
            }
            for (int j = 0; j < nx - 1; ++j) kf[j] = face_k(w, lay, Ts, Ps, j);
            for (int j = 0; j < nx; ++j) cn[j] = law_c(w, &w->layer[lay[j]], Ts[j], Ps[j]);
            /* moisture: width c (P1 - P0)/dt = theta F(P1) + (1-theta) F(P0) */
            for (int j = 0; j < nx; ++j) {
                double width = (j == 0 || j == nx - 1) ? 0.5 * dx : dx;
                double diag = width * cn[j].cM / dt, rhs = diag * Po[j];
                a[j] = 0.0; c[j] = 0.0;
                if (j > 0) {
                    double g = kf[j - 1].kM / dx;
                    diag += theta * g; a[j] = -theta * g;
                    rhs += (1.0 - theta) * g * (Po[j - 1] - Po[j]);
                }
                if (j < nx - 1) {
                    double g = kf[j].kM / dx;
                    diag += theta * g; c[j] = -theta * g;
                    rhs += (1.0 - theta) * g * (Po[j + 1] - Po[j]);
                }
                if (j == 0 || j == nx - 1) {
                    int side = j == 0 ? 0 : 1;
                    double h = w->hM[side];
                    diag += theta * h;
                    rhs += theta * (h * Pi1[side] + w->ginf[side])
                         + (1.0 - theta) * (h * (Pi0[side] - Po[j]) + w->ginf[side]);
                }
                b[j] = diag; d[j] = rhs;
            }
            thomas(nx, a, b, c, d, Pn);
            /* heat, with the new vapour pressure */
            for (int j = 0; j < nx; ++j) {
                double width = (j == 0 || j == nx - 1) ? 0.5 * dx : dx;
                double diag = width * cn[j].cTT / dt;
                double rhs = diag * To[j] - width * cn[j].cTM * (Pn[j] - Po[j]) / dt;
                a[j] = 0.0; c[j] = 0.0;
                if (j > 0) {
                    double gT = kf[j - 1].kTT / dx, gX = kf[j - 1].kTM / dx;
                    diag += theta * gT; a[j] = -theta * gT;
                    rhs += (1.0 - theta) * gT * (To[j - 1] - To[j])
                         + gX * (theta * (Pn[j - 1] - Pn[j]) + (1.0 - theta) * (Po[j - 1] - Po[j]));
                }
                if (j < nx - 1) {
                    double gT = kf[j].kTT / dx, gX = kf[j].kTM / dx;
                    diag += theta * gT; c[j] = -theta * gT;
                    rhs += (1.0 - theta) * gT * (To[j + 1] - To[j])
                         + gX * (theta * (Pn[j + 1] - Pn[j]) + (1.0 - theta) * (Po[j + 1] - Po[j]));
                }
                if (j == 0 || j == nx - 1) {
                    int side = j == 0 ? 0 : 1;
                    double hT = w->hT[side], hL = Lv * w->hM[side];
                    diag += theta * hT;
                    double q1 = w->qinf[side] + incident(w, side, t1);
                    double q0 = w->qinf[side] + incident(w, side, t0);
                    rhs += theta * (hT * Ti1[side] + hL * (Pi1[side] - Pn[j]) + q1)
                         + (1.0 - theta) * (hT * (Ti0[side] - To[j])
                                            + hL * (Pi0[side] - Po[j]) + q0);
                }
                b[j] = diag; d[j] = rhs;
            }
            thomas(nx, a, b, c, d, Tn);
            double dT = 0.0, dP = 0.0, sT = 0.0, sP = 0.0;
            for (int j = 0; j < nx; ++j) {
                double e = fabs(Tn[j] - Tk[j]); if (e > dT) dT = e;
                e = fabs(Pn[j] - Pk[j]); if (e > dP) dP = e;
                if (fabs(Tn[j]) > sT) sT = fabs(Tn[j]);
                if (fabs(Pn[j]) > sP) sP = fabs(Pn[j]);
            }
            memcpy(Tk, Tn, sizeof(double) * (size_t)nx);
            memcpy(Pk, Pn, sizeof(double) * (size_t)nx);
            if ((dT <= eta * sT && dP <= eta * sP) || it >= 200) break;
        }
        iters += it;
        memcpy(T, Tk, sizeof(double) * (size_t)nx);
        memcpy(P, Pk, sizeof(double) * (size_t)nx);
    }
    free(lay); free(To); free(Po); free(Tk); free(Pk); free(Ts); free(Ps);
    free(a); free(b); free(c); free(d); free(Pn); free(Tn); free(kf); free(cn);
    return nsteps > 0 ? iters / (double)nsteps : 0.0;
}
