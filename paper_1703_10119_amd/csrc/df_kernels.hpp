// df_kernels.hpp -- set-up, start-up, streaming DF step and room kernels.
//
// Streaming step (one launch per time step, levels in HBM):
//   workgroup = one tile of 255 consecutive nodes of one wall plus one halo
//   lane on its left; lane i owns node j = j0 - 1 + i.  Each lane evaluates
//   the face j+1/2 at the face-averaged state of level n (Sec. 3.1); the
//   faces and the nodes' level-n state are exchanged through LDS, so every
//   face is evaluated once and every level is read once, all reads issued
//   before the face arithmetic.  Lane 0 only contributes its face.  Moisture is updated first and heat uses the
//   new vapour pressure (App. A, eq. DF_eq2b).  Surface lanes evaluate the
//   outdoor air at t^n in FP64 (or read the zone air of level n), apply the
//   DF-averaged Robin half cell (eq. bc_v) and update the wall's applied flux
//   and its Neumaier-compensated integral in FP64.
#pragma once
#include "dfhm_device.hpp"

namespace dfhm {

constexpr int kStreamBlock = 256;
constexpr int kStreamTile = kStreamBlock - 1;   // nodes per tile

// ---------------------------------------------------------------- set-up

// Per wall: grid constants and initial vapour pressure.
__global__ void k_init_walls(WallDev *walls, int nw, double dt)
{
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nw) return;
    WallDev &W = walls[w];
    double L = 0.0;
    for (int l = 0; l < W.n_layers; ++l) L += W.lay[l][L_THICK];
    double dx = L / (double)(W.nx - 1);
    W.dx = dx;
    W.r = dt / (dx * dx);
    W.s = dt / dx;
    W.th0 = W.T0 - 273.15;
    W.P0 = W.RH0 * psat_th(W.T0 - 273.15);
}

// Per node: layer id (first layer whose right end is >= x_j) and the
// uniform initial state in the storage format.
template <typename R>
__global__ void k_init_nodes(const WallDev *__restrict__ walls, const int2 *__restrict__ tiles,
                             uint8_t *lay, R *T0b, R *T1b, R *P0b, R *P1b)
{
    const int2 tile = tiles[blockIdx.x];
    const WallDev &W = walls[tile.x];
    const int j = tile.y + (int)threadIdx.x - 1;
    if (threadIdx.x == 0 || j >= W.nx) return;
    double right[kMaxLayers];
    double acc = 0.0;
    for (int l = 0; l < W.n_layers; ++l) { acc += W.lay[l][L_THICK]; right[l] = acc; }
    double x = (double)j * W.dx;
    int l = 0;
    while (l < W.n_layers - 1 && x > right[l]) ++l;
    const int64_t g = (int64_t)W.off + j;
    lay[g] = (uint8_t)l;
    R Tv = (R)(W.T0 - Store<R>::tref(W));
    R Pv = (R)(W.P0 - (double)Store<R>::pref(W));
    T0b[g] = Tv; T1b[g] = Tv;
    P0b[g] = Pv; P1b[g] = Pv;
}

// Per zone: initial vapour pressure from the initial relative humidity
// (the host stores RH0 in roomP before this runs).
__global__ void k_init_rooms(const RoomDev *__restrict__ rooms, double *roomP, int nr)
{
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    roomP[r] = rooms[r].RH0 * psat_th(rooms[r].T0 - 273.15);
}

// ---------------------------------------------------------------- ambient

// Ambient (T_inf, P_inf) of one side at time t: outdoor sinusoids, or the
// zone air of level n on a zone side.
__device__ __forceinline__ void ambient(const WallDev &W, int side, double t,
                                        const double *__restrict__ roomT,
                                        const double *__restrict__ roomP,
                                        double &Tinf, double &Pinf)
{
    if (W.room >= 0 && W.room_side == side) {
        Tinf = roomT[W.room];
        Pinf = roomP[W.room];
    } else {
        double T = sine_at(W.Tamb[side], t);
        double RH = sine_at(W.RHamb[side], t);
        Tinf = T;
        Pinf = RH * psat_th(T - 273.15);
    }
}

// Long-wave exchange received by the zone-side surface of W (Sec. 2,
// boundary conditions): s eps sigma (S4 - m T^4) with S4 the sum of T_w^4 over
// the zone-side surfaces of the m walls of the zone, all read from the level
// buffer Tg (whole batch) and Ts the surface temperature of W itself (K).
template <typename R>
__device__ __forceinline__ double longwave(const WallDev &W, const WallDev *__restrict__ walls,
                                           const RoomDev *__restrict__ rooms,
                                           const int32_t *__restrict__ room_walls, const R *Tg,
                                           double Ts)
{
    const RoomDev &Rm = rooms[W.room];
    double S4 = 0.0;
    for (int q = Rm.w_begin; q < Rm.w_end; ++q) {
        const WallDev &V = walls[room_walls[q]];
        const int64_t g = (int64_t)V.off + (V.room_side == 0 ? 0 : V.nx - 1);
        S4 += pow4(Store<R>::tref(V) + (double)Tg[g]);
    }
    return W.esig * (S4 - (double)W.room_walls * pow4(Ts));
}

// ----------------------------------------------------------- DF node math

// Interior node update; returns (T+, P+).  r = dt/dx^2.
template <typename R>
__device__ __forceinline__ void df_interior(R r, const CCoef<R> &c, const KCoef<R> &kl,
                                            const KCoef<R> &kr, R Tm, R Pm, R Tl, R Pl,
                                            R Tr, R Pr, R &Tn, R &Pn)
{
    R KM = kl.kM + kr.kM;
    Pn = ((c.cM - r * KM) * Pm + (R)2 * r * (kr.kM * Pr + kl.kM * Pl)) / (c.cM + r * KM);
    R KT = kl.kT + kr.kT;
    R KX = kl.kX + kr.kX;
    R rhs = (c.cT - r * KT) * Tm + (R)2 * r * (kr.kT * Tr + kl.kT * Tl)
          + (c.cX - r * KX) * Pm - (c.cX + r * KX) * Pn
          + (R)2 * r * (kr.kX * Pr + kl.kX * Pl);
    Tn = rhs / (c.cT + r * KT);
}

// Surface node (half cell, DF-averaged surface value in the Robin term).
template <typename R>
__device__ __forceinline__ void df_surface(R r, R s, R hT, R hM, R hL, R qinf, R ginf,
                                           const CCoef<R> &c, const KCoef<R> &k, R Tm, R Pm,
                                           R Tnb, R Pnb, R Tid, R Pid, R &Tn, R &Pn)
{
    Pn = ((c.cM - (R)2 * r * k.kM - (R)2 * s * hM) * Pm + (R)4 * r * k.kM * Pnb
          + (R)4 * s * (hM * Pid + ginf))
       / (c.cM + (R)2 * r * k.kM + (R)2 * s * hM);
    R rhs = (c.cT - (R)2 * r * k.kT - (R)2 * s * hT) * Tm + (R)4 * r * k.kT * Tnb
          + (R)4 * s * hT * Tid
          + (c.cX - (R)2 * r * k.kX - (R)2 * s * hL) * Pm
          - (c.cX + (R)2 * r * k.kX + (R)2 * s * hL) * Pn
          + (R)4 * r * k.kX * Pnb + (R)4 * s * hL * Pid + (R)4 * s * qinf;
    Tn = rhs / (c.cT + (R)2 * r * k.kT + (R)2 * s * hT);
}

// Applied fluxes of one side and their compensated integral (FP64).
template <typename R>
__device__ __forceinline__ void surface_flux(const WallDev &W, int side, double Tinf,
                                             double Pinf, double qx, R Tn, R Tm, R Pn, R Pm,
                                             double Lv, double dt, double *__restrict__ fw)
{
    const double tref = Store<R>::tref(W);
    const double pref = (double)Store<R>::pref(W);
    double Ts = 0.5 * ((double)Tn + (double)Tm);
    double Ps = 0.5 * ((double)Pn + (double)Pm);
    double hM = W.hM[side];
    double g = hM * ((Pinf - pref) - Ps) + W.ginf[side];
    double q = W.hT[side] * ((Tinf - tref) - Ts) + Lv * hM * ((Pinf - pref) - Ps)
             + (W.qinf[side] + qx);
    fw[side * 2 + 0] = q;
    fw[side * 2 + 1] = g;
    double s0 = fw[4 + side * 2], c0 = fw[8 + side * 2];
    neumaier_add(s0, c0, dt * q);
    fw[4 + side * 2] = s0;
    fw[8 + side * 2] = c0;
    double s1 = fw[5 + side * 2], c1 = fw[9 + side * 2];
    neumaier_add(s1, c1, dt * g);
    fw[5 + side * 2] = s1;
    fw[9 + side * 2] = c1;
}

// ------------------------------------------------------ streaming DF step

// EXT: radiative sources present in the batch (incident flux or long-wave
// exchange); without them the surface lanes skip that code entirely.
// LAW: 0 = shape law, 1 = the Table 1 law.
template <typename R, bool EXT, int LAW>
__global__ void __launch_bounds__(kStreamBlock)
k_df_stream(const WallDev *__restrict__ walls, const int2 *__restrict__ tiles,
            R *T0b, R *T1b, R *P0b, R *P1b, const uint8_t *__restrict__ lay,
            const double *__restrict__ roomT, const double *__restrict__ roomP,
            const RoomDev *__restrict__ rooms, const int32_t *__restrict__ room_walls,
            double *__restrict__ flux, int *__restrict__ bad,
            const int64_t *__restrict__ step_base, int step_off, RunConst rc)
{
    __shared__ R s_kT[kStreamBlock], s_kM[kStreamBlock], s_kX[kStreamBlock];
    __shared__ R s_T[kStreamBlock], s_P[kStreamBlock];
    __shared__ double s_lay[kMaxLayers][L_COUNT];

    const int2 tile = tiles[blockIdx.x];
    const WallDev &W = walls[tile.x];
    const int nx = W.nx;
    const int i = threadIdx.x;
    const int j = tile.y - 1 + i;
    const int64_t n = *step_base + step_off;
    const int cb = (int)(n & 1);
    const R *Tc = (cb ? T1b : T0b) + W.off;
    const R *Pc = (cb ? P1b : P0b) + W.off;
    R *To = (cb ? T0b : T1b) + W.off;
    R *Po = (cb ? P0b : P1b) + W.off;
    const R *Tp = (n == 0) ? Tc : To;      // repeat start: level -1 := level 0
    const R *Pp = (n == 0) ? Pc : Po;
    const uint8_t *ly = lay + W.off;

    const bool layered = W.n_layers > 1;
    if (layered) {
        for (int q = i; q < kMaxLayers * L_COUNT; q += kStreamBlock)
            s_lay[q / L_COUNT][q % L_COUNT] = W.lay[q / L_COUNT][q % L_COUNT];
        __syncthreads();
    }
    const R thr = Store<R>::thref(W);
    const R pr = Store<R>::pref(W);

    // every level read is issued here, before the face arithmetic: the left
    // neighbour comes from the lane on the left through LDS
    R Tj = 0, Pj = 0, Tr = 0, Pr = 0, Tm = 0, Pm = 0;
    const bool in_wall = j >= 0 && j < nx;
    if (in_wall) { Tj = Tc[j]; Pj = Pc[j]; }
    if (in_wall && i > 0) { Tm = Tp[j]; Pm = Pp[j]; }
    KCoef<R> kr = {0, 0, 0};
    if (j >= 0 && j < nx - 1) {
        Tr = Tc[j + 1];
        Pr = Pc[j + 1];
        R thf = thr + (R)0.5 * (Tj + Tr);
        R Pf = pr + (R)0.5 * (Pj + Pr);
        if constexpr (LAW == 1) {
            const int la = layered ? ly[j] : 0, lb = layered ? ly[j + 1] : 0;
            kr = t1_face_k<R>(W, la, lb, thf, Pf, (R)rc.Lv);
        } else if (!layered) kr = face_k<R>(W, 0, 0, thf, Pf);
        else {
            int la = ly[j], lb = ly[j + 1];
            R phi = Pf / psat_th(thf);
            KCoef<R> a = law_k<R>(s_lay[la], phi);
            if (la == lb) kr = a;
            else {
                KCoef<R> b = law_k<R>(s_lay[lb], phi);
                kr.kT = harm(a.kT, b.kT);
                kr.kM = harm(a.kM, b.kM);
                kr.kX = harm(a.kX, b.kX);
            }
        }
    }
    s_kT[i] = kr.kT;
    s_kM[i] = kr.kM;
    s_kX[i] = kr.kX;
    s_T[i] = Tj;
    s_P[i] = Pj;
    __syncthreads();
    if (i == 0 || !in_wall) return;

    KCoef<R> kl = {s_kT[i - 1], s_kM[i - 1], s_kX[i - 1]};
    const double *m = layered ? s_lay[ly[j]] : W.lay[0];
    const R th = thr + Tj;
    const R P = pr + Pj;
    CCoef<R> c;
    if constexpr (LAW == 1) c = t1_law_c<R>(m, th, P, (R)rc.cw);
    else c = law_c<R>(m, P / psat_th(th), th);
    const R r = (R)W.r;
    R Tn, Pn;
    if (j > 0 && j < nx - 1) {
        R Tl = s_T[i - 1], Pl = s_P[i - 1];
        df_interior<R>(r, c, kl, kr, Tm, Pm, Tl, Pl, Tr, Pr, Tn, Pn);
    } else {
        const int side = j == 0 ? 0 : 1;
        const KCoef<R> k = side == 0 ? kr : kl;
        R Tnb = side == 0 ? Tr : s_T[i - 1];
        R Pnb = side == 0 ? Pr : s_P[i - 1];
        double Tinf, Pinf;
        ambient(W, side, (double)n * rc.dt, roomT, roomP, Tinf, Pinf);
        // radiation at t^n: incident flux, long-wave exchange on the zone side
        double qx = 0.0;
        if constexpr (EXT) {
            qx = incident(W, side, (double)n * rc.dt);
            if (W.esig != 0.0 && W.room_side == side)
                qx += longwave<R>(W, walls, rooms, room_walls, cb ? T1b : T0b,
                                  Store<R>::tref(W) + (double)Tj);
        }
        const R Tid = (R)(Tinf - Store<R>::tref(W));
        const R Pid = (R)(Pinf - (double)pr);
        const R hM = (R)W.hM[side];
        df_surface<R>(r, (R)W.s, (R)W.hT[side], hM, (R)(rc.Lv * W.hM[side]),
                      (R)(W.qinf[side] + qx), (R)W.ginf[side], c, k, Tm, Pm, Tnb, Pnb, Tid,
                      Pid, Tn, Pn);
        surface_flux<R>(W, side, Tinf, Pinf, qx, Tn, Tm, Pn, Pm, rc.Lv, rc.dt,
                        flux + (int64_t)tile.x * 12);
    }
    if (!(isfinite(Tn) && isfinite(Pn))) atomicOr(bad, 1);
    To[j] = Tn;
    Po[j] = Pn;
}

// Advance the device step counter after a chunk (lane 0 of one workgroup).
__global__ void k_tick(int64_t *step_base, int k)
{
    if (threadIdx.x == 0) step_base[0] += k;
}

// --------------------------------------------------- forward-Euler start-up

constexpr int kStartBlock = 256;
constexpr int64_t kMaxSubsteps = int64_t(1) << 20;
constexpr int kStartNpt = kMaxNx / kStartBlock;

// One workgroup per wall; level 0 -> level 1 by m forward-Euler sub-steps of
// dt/m (FP64), m = max(1, ceil(2 dt / b)) with b the explicit stability
// bound (min over nodes of capacity / conductance, both fields, surface
// exchange included) of the initial state.
template <typename R>
__global__ void __launch_bounds__(kStartBlock)
k_startup(const WallDev *__restrict__ walls, R *T0b, R *T1b, R *P0b, R *P1b,
          const uint8_t *__restrict__ lay, const double *__restrict__ roomT,
          const double *__restrict__ roomP, const RoomDev *__restrict__ rooms,
          const int32_t *__restrict__ room_walls, double *__restrict__ flux,
          int *__restrict__ bad, RunConst rc, int law)
{
    __shared__ double sT[kMaxNx], sP[kMaxNx], skT[kMaxNx], skM[kMaxNx], skX[kMaxNx];
    __shared__ uint8_t sl[kMaxNx];
    __shared__ double red[kStartBlock];
    __shared__ double amb[6];           // per side: T_inf, P_inf, heat source

    const WallDev &W = walls[blockIdx.x];
    const int nx = W.nx;
    const int tid = threadIdx.x;
    const double tref = Store<R>::tref(W);
    const double pref = (double)Store<R>::pref(W);
    const double dx = W.dx;
    for (int j = tid; j < nx; j += kStartBlock) {
        sT[j] = tref + (double)T0b[W.off + j];
        sP[j] = pref + (double)P0b[W.off + j];
        sl[j] = lay[W.off + j];
    }
    __syncthreads();

    auto node_c = [&](const double *m, double T, double P) {
        return law == 1 ? t1_law_c<double>(m, T - 273.15, P, rc.cw)
                        : law_c<double>(m, P / psat_th(T - 273.15), T - 273.15);
    };
    auto faces = [&]() {
        for (int j = tid; j < nx - 1; j += kStartBlock) {
            double Tf = 0.5 * (sT[j] + sT[j + 1]);
            double Pf = 0.5 * (sP[j] + sP[j + 1]);
            KCoef<double> k = law == 1 ? t1_face_k<double>(W, sl[j], sl[j + 1], Tf - 273.15, Pf, rc.Lv)
                                       : face_k<double>(W, sl[j], sl[j + 1], Tf - 273.15, Pf);
            skT[j] = k.kT;
            skM[j] = k.kM;
            skX[j] = k.kX;
        }
    };

    // stability bound of the initial state
    faces();
    __syncthreads();
    double best = INFINITY;
    for (int j = tid; j < nx; j += kStartBlock) {
        CCoef<double> c = node_c(W.lay[sl[j]], sT[j], sP[j]);
        double width = (j == 0 || j == nx - 1) ? 0.5 * dx : dx;
        double gT = 0.0, gM = 0.0;
        if (j > 0) { gT += skT[j - 1] / dx; gM += skM[j - 1] / dx; }
        if (j < nx - 1) { gT += skT[j] / dx; gM += skM[j] / dx; }
        if (j == 0) { gT += W.hT[0]; gM += W.hM[0]; }
        if (j == nx - 1) { gT += W.hT[1]; gM += W.hM[1]; }
        double bT = c.cT * width / gT;
        double bM = c.cM * width / gM;
        best = fmin(best, fmin(bT, bM));
    }
    red[tid] = best;
    __syncthreads();
    for (int h = kStartBlock / 2; h > 0; h >>= 1) {
        if (tid < h) red[tid] = fmin(red[tid], red[tid + h]);
        __syncthreads();
    }
    const double mm = ceil(2.0 * rc.dt / red[0]);
    // at least one sub-step; at most kMaxSubsteps (also when the bound is 0)
    const int64_t m = !(mm >= 1.0) ? 1 : (mm > (double)kMaxSubsteps ? kMaxSubsteps : (int64_t)mm);
    const double dts = rc.dt / (double)m;

    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    double fs[2][2], fc[2][2];
    double *fw = flux + (int64_t)blockIdx.x * 12;
    if (tid == 0)
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 2; ++f) { fs[s][f] = fw[4 + s * 2 + f]; fc[s][f] = fw[8 + s * 2 + f]; }

    // long-wave exchange of the zone side, held at level 0 for the whole step
    double qlw[2] = {0.0, 0.0};
    if (tid == 0 && W.esig != 0.0)
        qlw[W.room_side] = longwave<R>(W, walls, rooms, room_walls, T0b,
                                       sT[W.room_side == 0 ? 0 : nx - 1]);

    double nT[kStartNpt], nP[kStartNpt];
    for (int64_t k = 0; k < m; ++k) {
        const double t = (double)k * rc.dt / (double)m;
        if (tid == 0) {
            for (int s = 0; s < 2; ++s) {
                ambient(W, s, t, roomT, roomP, amb[3 * s], amb[3 * s + 1]);
                amb[3 * s + 2] = W.qinf[s] + (incident(W, s, t) + qlw[s]);
            }
        }
        faces();
        __syncthreads();
        if (tid == 0) {
            for (int s = 0; s < 2; ++s) {
                int j = s == 0 ? 0 : nx - 1;
                double Tinf = amb[3 * s], Pinf = amb[3 * s + 1];
                double g = W.hM[s] * (Pinf - sP[j]) + W.ginf[s];
                double q = W.hT[s] * (Tinf - sT[j]) + rc.Lv * W.hM[s] * (Pinf - sP[j]) + amb[3 * s + 2];
                neumaier_add(fs[s][0], fc[s][0], dts * q);
                neumaier_add(fs[s][1], fc[s][1], dts * g);
                acc[s][0] += q;
                acc[s][1] += g;
            }
        }
        int q = 0;
        for (int j = tid; j < nx; j += kStartBlock, ++q) {
            double T = sT[j], P = sP[j];
            CCoef<double> c = node_c(W.lay[sl[j]], T, P);
            double width = (j == 0 || j == nx - 1) ? 0.5 * dx : dx;
            double dM = 0.0, dT = 0.0;
            if (j > 0) {
                dM += skM[j - 1] * (sP[j - 1] - P) / dx;
                dT += skT[j - 1] * (sT[j - 1] - T) / dx + skX[j - 1] * (sP[j - 1] - P) / dx;
            }
            if (j < nx - 1) {
                dM += skM[j] * (sP[j + 1] - P) / dx;
                dT += skT[j] * (sT[j + 1] - T) / dx + skX[j] * (sP[j + 1] - P) / dx;
            }
            if (j == 0 || j == nx - 1) {
                int s = j == 0 ? 0 : 1;
                double Tinf = amb[3 * s], Pinf = amb[3 * s + 1];
                dM += W.hM[s] * (Pinf - P) + W.ginf[s];
                dT += W.hT[s] * (Tinf - T) + rc.Lv * W.hM[s] * (Pinf - P) + amb[3 * s + 2];
            }
            double Pnew = P + dts * dM / (c.cM * width);
            double Tnew = T + (dts * dT / width - c.cX * (Pnew - P)) / c.cT;
            nT[q] = Tnew;
            nP[q] = Pnew;
        }
        __syncthreads();
        q = 0;
        for (int j = tid; j < nx; j += kStartBlock, ++q) { sT[j] = nT[q]; sP[j] = nP[q]; }
        __syncthreads();
    }
    for (int j = tid; j < nx; j += kStartBlock) {
        R Tv = (R)(sT[j] - tref), Pv = (R)(sP[j] - pref);
        if (!(isfinite(Tv) && isfinite(Pv))) atomicOr(bad, 1);
        T1b[W.off + j] = Tv;
        P1b[W.off + j] = Pv;
    }
    if (tid == 0) {
        for (int s = 0; s < 2; ++s)
            for (int f = 0; f < 2; ++f) {
                fw[s * 2 + f] = acc[s][f] / (double)m;
                fw[4 + s * 2 + f] = fs[s][f];
                fw[8 + s * 2 + f] = fc[s][f];
            }
    }
}

// ------------------------------------------------------------------ rooms

// One lane per zone: heat and vapour it gains from its linked zones (Sec.
// 5.1, inter-zone sources) at the level-n air, into inz[2 r], inz[2 r + 1];
// runs before k_room_step, which updates the air in place.
__global__ void __launch_bounds__(64)
k_zone_exchange(const RoomDev *__restrict__ rooms, const ZoneLinkDev *__restrict__ links,
                const double *__restrict__ roomT, const double *__restrict__ roomP,
                double *__restrict__ inz, int nr, RunConst rc)
{
    const int rix = blockIdx.x * blockDim.x + threadIdx.x;
    if (rix >= nr) return;
    const RoomDev &Rm = rooms[rix];
    const double Ta = roomT[rix], Pa = roomP[rix];
    const double cma = rc.c_pa + rc.c_pv * Pa / rc.Pv_ref;
    double Q = 0.0, G = 0.0;
    for (int l = Rm.l_begin; l < Rm.l_end; ++l) {
        const ZoneLinkDev L = links[l];
        const double Tj = roomT[L.partner], Pj = roomP[L.partner];
        const double cj = rc.c_pa + rc.c_pv * Pj / rc.Pv_ref;
        G += L.g * (Pj - Pa) / rc.Pv_ref;
        Q += L.g * (cj * (Tj - 273.15) - cma * (Ta - 273.15)) + rc.Lv * L.g * (Pj - Pa) / rc.Pv_ref;
    }
    inz[2 * rix] = Q;
    inz[2 * rix + 1] = G;
}

// One lane per zone: forward Euler of the zone balance with the level-n
// surface values of its walls (ascending wall order), sources at t^n and,
// when inz is given, the inter-zone gains of k_zone_exchange.
template <typename R>
__global__ void __launch_bounds__(64)
k_room_step(const RoomDev *__restrict__ rooms, const int32_t *__restrict__ room_walls,
            const WallDev *__restrict__ walls, const R *T0b, const R *T1b, const R *P0b,
            const R *P1b, double *roomT, double *roomP, const double *__restrict__ sched_go,
            const double *__restrict__ sched_qh, const double *__restrict__ inz, int nr,
            const int64_t *__restrict__ step_base, int step_off, RunConst rc)
{
    const int rix = blockIdx.x * blockDim.x + threadIdx.x;
    if (rix >= nr) return;
    const int64_t n = *step_base + step_off;
    const int cb = (int)(n & 1);
    const R *Tc = cb ? T1b : T0b;
    const R *Pc = cb ? P1b : P0b;
    const RoomDev &Rm = rooms[rix];
    const double t = (double)n * rc.dt;
    const double Ta = roomT[rix], Pa = roomP[rix];
    const double mass = rc.rho_a * Rm.volume;
    const double gv = Rm.ach * mass / 3600.0;
    const double cma = rc.c_pa + rc.c_pv * Pa / rc.Pv_ref;
    const int64_t slot = (int64_t)floor(t / Rm.sched_dt) % Rm.n_sched;
    const double go = sched_go[Rm.sched_off + slot], Qh = sched_qh[Rm.sched_off + slot];
    const double Tout = sine_at(Rm.Tout, t);
    const double Pout = sine_at(Rm.RHout, t) * psat_th(Tout - 273.15);
    double G = go + gv * (Pout - Pa) / rc.Pv_ref;
    double Q = Qh + rc.Lv * go + gv * cma * (Tout - Ta) + rc.Lv * gv * (Pout - Pa) / rc.Pv_ref;
    for (int q = Rm.w_begin; q < Rm.w_end; ++q) {
        const WallDev &W = walls[room_walls[q]];
        const int side = W.room_side;
        const int64_t g = (int64_t)W.off + (side == 0 ? 0 : W.nx - 1);
        const double Ts = Store<R>::tref(W) + (double)Tc[g];
        const double Ps = (double)Store<R>::pref(W) + (double)Pc[g];
        G += W.area * W.hM[side] * (Ps - Pa);
        Q += W.area * (W.hT[side] * (Ts - Ta) + rc.Lv * W.hM[side] * (Ps - Pa));
    }
    if (inz) {
        Q += inz[2 * rix];
        G += inz[2 * rix + 1];
    }
    roomP[rix] = Pa + rc.dt * G / (mass / rc.Pv_ref);
    roomT[rix] = Ta + rc.dt * Q / (mass * cma);
}

} // namespace dfhm
