// df_resident.hpp -- persistent DF kernel: one launch advances a chunk of k
// steps with every wall's two levels kept on chip.
//
// Work decomposition: the host packs whole walls (and, for coupled zones, a
// zone together with all of its walls) into workgroups.  The workgroup's
// walls are laid end to end in a block-local node space of threads x NPT
// slots; lane t owns the NPT consecutive nodes t*NPT .. t*NPT+NPT-1.  The
// levels n-1 and n of those nodes stay in VGPRs for the whole chunk (the
// VGPR file is 512 KB per CU, over three times the LDS), LDS only carries
// per-step halos, the face conductivities at the lane boundaries, the zone
// air, the wall table and the flux accumulators.  HBM is touched only at the
// chunk ends, so a step costs no HBM traffic and the kernel is bound by the
// VALU work of the material law.
//
// Per step (two workgroup barriers):
//   A  lanes publish their first / last node (level n) and surface values;
//   B  lanes read the neighbour halos, evaluate the NPT right faces at the
//      face-averaged state (Sec. 3.1) and publish the last one; one lane per
//      zone advances the zone air by forward Euler from the level-n surfaces
//      (Sec. 5.3, eq. wbse_tn_exp);
//   C  lanes take their first left face from LDS and update moisture, then
//      heat (App. A, eq. DF_eq2b); surface nodes use the DF-averaged Robin
//      half cell (eq. bc_v) with the outdoor air at t^n or the level-n zone
//      air, and accumulate the applied flux (Neumaier, FP64).
//
// All walls of one launch must share the law shape (a_T, a_M, b_TM, c_T,
// c_M, e_TM, f_TM), which is passed as an argument; then the face value at a
// layer interface is the harmonic mean of the layer scales times the common
// shape factor, and every per-node scale can be fixed once per chunk.  The
// update is written divided by r = dt/dx^2 (node capacities pre-divided by
// r), so interior nodes need no per-wall constant at all.
#pragma once
#include "df_kernels.hpp"

namespace dfhm {

constexpr int kResMaxWalls = 64;   // walls per workgroup (LDS wall table)
constexpr int kResMaxRooms = 16;   // zones per workgroup

struct ResBlock {
    int32_t w_begin, w_end;        // range in block_walls (ascending wall ids)
    int32_t r_begin, r_end;        // range in block_rooms
    int32_t n_nodes, pad;
};

struct Shape {
    double aT, aM, bTM, cT, aC, eTM, fTM;
};

// Dynamic LDS of one workgroup: halo [2][4][NT] (first T, first P, last T,
// last P of each lane) and faces [2][3][NT] (last right face of each lane).
template <typename R>
constexpr size_t res_dyn_lds(int nt) { return sizeof(R) * 14 * (size_t)nt; }

template <typename R, int NPT, int NT>
__global__ void __launch_bounds__(NT)
k_df_resident(const ResBlock *__restrict__ blocks, const int32_t *__restrict__ block_walls,
              const int32_t *__restrict__ block_rooms, const WallDev *__restrict__ walls,
              R *T0b, R *T1b, R *P0b, R *P1b, const uint8_t *__restrict__ lay,
              const RoomDev *__restrict__ rooms, double *roomT, double *roomP,
              const double *__restrict__ sched_go, const double *__restrict__ sched_qh,
              double *__restrict__ flux, int *__restrict__ bad,
              const int64_t *__restrict__ step_base, int ksteps, RunConst rc, Shape sh)
{
    static_assert(NT >= 2 * kResMaxWalls, "one lane per wall side computes the ambient");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t s_wstart[kResMaxWalls + 1];
    __shared__ int32_t s_wid[kResMaxWalls];
    __shared__ int32_t s_wroom[kResMaxWalls];           // local zone or -1
    __shared__ double s_flux[kResMaxWalls][12];
    __shared__ double s_surf[2][kResMaxWalls][2][2];   // [par][slot][side][T,P] level n
    __shared__ double s_amb[2][kResMaxWalls][2][2];    // [par][slot][side][T,P] ambient at t^n
    __shared__ double s_room[2][kResMaxRooms][2];      // [par][zone][T,P]
    __shared__ int32_t s_rid[kResMaxRooms];
    // outdoor sinusoids per wall side: T mean, T amp, RH mean, RH amp,
    // sin/cos of the T and RH phases at t^n, sin/cos of the per-step increments
    __shared__ double s_rot[kResMaxWalls][2][12];

    constexpr int nthreads = NT;
    const int t = threadIdx.x;
    R *halo = (R *)lds_raw;                  // [2][4][nthreads]
    R *facb = halo + 8 * nthreads;           // [2][3][nthreads]

    const ResBlock B = blocks[blockIdx.x];
    const int nwb = B.w_end - B.w_begin;
    const int nrb = B.r_end - B.r_begin;
    const int64_t n0 = *step_base;

    // ---- wall table, zone table, flux accumulators
    if (t == 0) {
        int acc = 0;
        for (int s = 0; s < nwb; ++s) {
            int w = block_walls[B.w_begin + s];
            s_wid[s] = w;
            s_wstart[s] = acc;
            acc += walls[w].nx;
        }
        s_wstart[nwb] = acc;
    }
    if (t < nrb) {
        int r = block_rooms[B.r_begin + t];
        s_rid[t] = r;
        s_room[n0 & 1][t][0] = roomT[r];
        s_room[n0 & 1][t][1] = roomP[r];
    }
    __syncthreads();
    for (int q = t; q < nwb * 12; q += nthreads) {
        int s = q / 12, k = q % 12;
        s_flux[s][k] = flux[(int64_t)s_wid[s] * 12 + k];
    }
    if (t < nwb) {
        const WallDev &W = walls[s_wid[t]];
        int lr = -1;
        for (int z = 0; z < nrb; ++z)
            if (s_rid[z] == W.room) lr = z;
        s_wroom[t] = lr;
    }

    // ---- ambient lanes: one per wall side; the outdoor sinusoids advance by
    // an exact rotation through the chunk, anchored at t^n0 (state in LDS)
    const bool amb_lane = t < 2 * nwb;
    const int amb_slot = t >> 1, amb_side = t & 1;
    if (amb_lane) {
        const WallDev &W = walls[block_walls[B.w_begin + amb_slot]];
        const double *ST = W.Tamb[amb_side], *SR = W.RHamb[amb_side];
        const double t0 = (double)n0 * rc.dt;
        double *st = s_rot[amb_slot][amb_side];
        st[0] = ST[0]; st[1] = ST[1]; st[2] = SR[0]; st[3] = SR[1];
        sincos(2.0 * dpi() * t0 / ST[2] + ST[3], &st[4], &st[5]);
        sincos(2.0 * dpi() * t0 / SR[2] + SR[3], &st[6], &st[7]);
        sincos(2.0 * dpi() * rc.dt / ST[2], &st[8], &st[9]);
        sincos(2.0 * dpi() * rc.dt / SR[2], &st[10], &st[11]);
    }

    // ---- per-node set-up: levels, scales, flags
    const int cb = (int)(n0 & 1);
    const R *Tc = cb ? T1b : T0b;
    const R *Pc = cb ? P1b : P0b;
    const R *Tp = (n0 == 0) ? Tc : (cb ? T0b : T1b);
    const R *Pp = (n0 == 0) ? Pc : (cb ? P0b : P1b);

    R Tm[NPT], Pm[NPT], Tn[NPT], Pn[NPT];       // levels n-1 and n
    R c0s[NPT], cM0s[NPT], kf0[NPT], kMf0[NPT];
    int info[NPT];                               // slot | left << 8 | right << 9 | active << 10
    {
        int slot = 0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int b = t * NPT + q;
            Tm[q] = Pm[q] = Tn[q] = Pn[q] = 0;
            c0s[q] = cM0s[q] = 1;
            kf0[q] = kMf0[q] = 0;
            info[q] = 0;
            if (b < B.n_nodes) {
                while (b >= s_wstart[slot + 1]) ++slot;
                const WallDev &W = walls[s_wid[slot]];
                const int j = b - s_wstart[slot];
                const int64_t g = (int64_t)W.off + j;
                Tm[q] = Tp[g]; Pm[q] = Pp[g];
                Tn[q] = Tc[g]; Pn[q] = Pc[g];
                const int la = lay[g];
                const double rinv = 1.0 / W.r;
                c0s[q] = (R)(W.lay[la][L_C0] * rinv);
                cM0s[q] = (R)(W.lay[la][L_CM0] * rinv);
                if (j < W.nx - 1) {
                    const int lb = lay[g + 1];
                    double a = W.lay[la][L_K0], bb = W.lay[lb][L_K0];
                    double am = W.lay[la][L_KM0], bm = W.lay[lb][L_KM0];
                    if (la != lb) {
                        double s1 = a + bb, s2 = am + bm;
                        a = s1 > 0.0 ? 2.0 * a * bb / s1 : 0.0;
                        am = s2 > 0.0 ? 2.0 * am * bm / s2 : 0.0;
                    }
                    kf0[q] = (R)a;
                    kMf0[q] = (R)am;
                }
                info[q] = slot | ((j == 0) << 8) | ((j == W.nx - 1) << 9) | (1 << 10);
            }
        }
    }
    const R aT = (R)sh.aT, aM = (R)sh.aM, bTM = (R)sh.bTM, cT = (R)sh.cT, aC = (R)sh.aC,
            eTM = (R)sh.eTM, fTM = (R)sh.fTM;
    // nodes of one lane may lie in different walls: per-node references
    R thref[NPT], pref[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const WallDev &W = walls[s_wid[info[q] & 0xff]];
        thref[q] = Store<R>::thref(W);
        pref[q] = Store<R>::pref(W);
    }
    const R ps_inv = (R)(1.0 / 610.94);
    __syncthreads();

    for (int i = 0; i < ksteps; ++i) {
        // Tm/Pm = level n-1, Tn/Pn = level n; the step leaves n+1 in Tm/Pm
        // and the swap at its end restores the roles
        const int64_t n = n0 + i;
        const int par = (int)(n & 1);
        // ---- A: publish halos, surface values and the ambient at t^n
        R *hp = halo + par * 4 * nthreads;
        hp[t] = Tn[0];
        hp[nthreads + t] = Pn[0];
        hp[2 * nthreads + t] = Tn[NPT - 1];
        hp[3 * nthreads + t] = Pn[NPT - 1];
        if (nrb > 0) {
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
                const int f = info[q];
                if (f & (3 << 8)) {
                    const int s = f & 0xff;
                    const int side = (f >> 8) & 1 ? 0 : 1;
                    s_surf[par][s][side][0] = Store<R>::tref(walls[s_wid[s]]) + (double)Tn[q];
                    s_surf[par][s][side][1] = (double)pref[q] + (double)Pn[q];
                }
            }
        }
        if (amb_lane) {
            const WallDev &W = walls[s_wid[amb_slot]];
            double Ta, Pa;
            double *st = s_rot[amb_slot][amb_side];
            if (W.room >= 0 && W.room_side == amb_side) {
                const int z = s_wroom[amb_slot];
                Ta = s_room[par][z][0];
                Pa = s_room[par][z][1];
            } else {
                Ta = st[0] + st[1] * st[4];
                Pa = (st[2] + st[3] * st[6]) * psat_th(Ta - 273.15);
            }
            s_amb[par][amb_slot][amb_side][0] = Ta;
            s_amb[par][amb_slot][amb_side][1] = Pa;
            const double sT = st[4], cT = st[5], sR = st[6], cR = st[7];
            st[4] = fma(sT, st[9], cT * st[8]);
            st[5] = fma(cT, st[9], -sT * st[8]);
            st[6] = fma(sR, st[11], cR * st[10]);
            st[7] = fma(cR, st[11], -sR * st[10]);
        }
        __syncthreads();
        // ---- B: faces and node humidity ratios, zones
        const R Tr_nb = t + 1 < nthreads ? hp[t + 1] : (R)0;
        const R Pr_nb = t + 1 < nthreads ? hp[nthreads + t + 1] : (R)0;
        const R Tl_nb = t > 0 ? hp[2 * nthreads + t - 1] : (R)0;
        const R Pl_nb = t > 0 ? hp[3 * nthreads + t - 1] : (R)0;
        if (t < nrb) {
            const RoomDev &Rm = rooms[s_rid[t]];
            const double tt = (double)n * rc.dt;
            const double Ta = s_room[par][t][0], Pa = s_room[par][t][1];
            const double mass = rc.rho_a * Rm.volume;
            const double gv = Rm.ach * mass / 3600.0;
            const double cma = rc.c_pa + rc.c_pv * Pa / rc.Pv_ref;
            const int64_t slot = (int64_t)floor(tt / Rm.sched_dt) % Rm.n_sched;
            const double go = sched_go[Rm.sched_off + slot], Qh = sched_qh[Rm.sched_off + slot];
            const double Tout = sine_at(Rm.Tout, tt);
            const double Pout = sine_at(Rm.RHout, tt) * psat_th(Tout - 273.15);
            double G = go + gv * (Pout - Pa) / rc.Pv_ref;
            double Q = Qh + rc.Lv * go + gv * cma * (Tout - Ta) + rc.Lv * gv * (Pout - Pa) / rc.Pv_ref;
            for (int s = 0; s < nwb; ++s) {
                if (s_wroom[s] != t) continue;
                const WallDev &W = walls[s_wid[s]];
                const int side = W.room_side;
                const double Ts = s_surf[par][s][side][0], Ps = s_surf[par][s][side][1];
                G += W.area * W.hM[side] * (Ps - Pa);
                Q += W.area * (W.hT[side] * (Ts - Ta) + rc.Lv * W.hM[side] * (Ps - Pa));
            }
            s_room[par ^ 1][t][1] = Pa + rc.dt * G / (mass / rc.Pv_ref);
            s_room[par ^ 1][t][0] = Ta + rc.dt * Q / (mass * cma);
        }
        R kT[NPT], kM[NPT], kX[NPT], phn[NPT];
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
            const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
            // a node without a right face (wall end, padding) has zero scales;
            // its face state is its own, so that nothing from the next wall or
            // from padding enters its arithmetic (and no NaN can leak in)
            const bool live = kf0[q] != (R)0 || kMf0[q] != (R)0;
            const R thn = thref[q] + Tn[q];
            const R thf = live ? fma((R)0.5, Tn[q] + Tr, thref[q]) : thn;
            const R Pf = live ? fma((R)0.5, Pn[q] + Pr, pref[q]) : pref[q] + Pn[q];
            // Magnus exponents of face and node (FP64: one shared reciprocal)
            const R df = thf + (R)243.04, dn = thn + (R)243.04;
            R af, an;
            if constexpr (sizeof(R) == 8) {
                const R inv = rcp_nr(df * dn);
                af = (thf * dn) * inv;
                an = (thn * df) * inv;
            } else {
                af = div_nr(thf, df);
                an = div_nr(thn, dn);
            }
            const R ef = exp_bounded(-(R)17.625 * af);
            const R en = exp_bounded(-(R)17.625 * an);
            const R phi = (Pf * ef) * ps_inv;               // phi = P / Ps
            phn[q] = ((pref[q] + Pn[q]) * en) * ps_inv;
            kT[q] = live ? kf0[q] * fma(aT, phi, (R)1) : (R)0;
            kM[q] = live ? kMf0[q] * fma(aM * phi, phi, (R)1) : (R)0;
            kX[q] = bTM * kM[q];
        }
        R *fp = facb + par * 3 * nthreads;
        fp[t] = kT[NPT - 1];
        fp[nthreads + t] = kM[NPT - 1];
        fp[2 * nthreads + t] = kX[NPT - 1];
        __syncthreads();
        // ---- C: node updates (moisture, then heat with the new Pv)
        const R klT = t > 0 ? fp[t - 1] : (R)0;
        const R klM = t > 0 ? fp[nthreads + t - 1] : (R)0;
        const R klX = t > 0 ? fp[2 * nthreads + t - 1] : (R)0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int f = info[q];
            const R th = thref[q] + Tn[q];
            const R phi = phn[q];
            const R ccT = c0s[q] * fma(cT, phi, (R)1);
            const R ccM = cM0s[q] * fma(aC, phi, (R)1);
            const R ccX = fma(fTM, th, eTM) * ccM;
            const R lT = q > 0 ? kT[q > 0 ? q - 1 : 0] : klT;
            const R lM = q > 0 ? kM[q > 0 ? q - 1 : 0] : klM;
            const R lX = q > 0 ? kX[q > 0 ? q - 1 : 0] : klX;
            const R Tl = q > 0 ? Tn[q > 0 ? q - 1 : 0] : Tl_nb;
            const R Pl = q > 0 ? Pn[q > 0 ? q - 1 : 0] : Pl_nb;
            const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
            const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
            R Tnew, Pnew;
            if (!(f & (3 << 8))) {
                const R KM = lM + kM[q];
                const R KT = lT + kT[q];
                const R KX = lX + kX[q];
                const R dM = ccM + KM, dT = ccT + KT;
                const R numM = fma(ccM - KM, Pm[q], (R)2 * fma(kM[q], Pr, lM * Pl));
                R inv = 0;
                if constexpr (sizeof(R) == 8) {
                    inv = rcp_nr(dM * dT);
                    Pnew = numM * (dT * inv);
                } else {
                    Pnew = div_nr(numM, dM);
                }
                const R rhs = fma(ccT - KT, Tm[q],
                                  fma((R)2, fma(kT[q], Tr, lT * Tl),
                                      fma(ccX - KX, Pm[q],
                                          fma(-(ccX + KX), Pnew,
                                              (R)2 * fma(kX[q], Pr, lX * Pl)))));
                if constexpr (sizeof(R) == 8) Tnew = rhs * (dM * inv);
                else Tnew = div_nr(rhs, dT);
            } else {
                const int s = f & 0xff;
                const int side = (f >> 8) & 1 ? 0 : 1;
                const WallDev &W = walls[s_wid[s]];
                const R k_T = side == 0 ? kT[q] : lT;
                const R k_M = side == 0 ? kM[q] : lM;
                const R k_X = side == 0 ? kX[q] : lX;
                const R Tnb = side == 0 ? Tr : Tl;
                const R Pnb = side == 0 ? Pr : Pl;
                const double Tinf = s_amb[par][s][side][0];
                const double Pinf = s_amb[par][s][side][1];
                const double tref = Store<R>::tref(W);
                const R Tid = (R)(Tinf - tref);
                const R Pid = (R)(Pinf - (double)pref[q]);
                const R d = (R)W.dx;                       // s / r
                const R hT = (R)W.hT[side], hM = (R)W.hM[side];
                const R hL = (R)(rc.Lv * W.hM[side]);
                const R ginf = (R)W.ginf[side], qinf = (R)W.qinf[side];
                const R gM = fma((R)2, k_M, (R)2 * d * hM);     // 2 r k + 2 s h (over r)
                const R gT = fma((R)2, k_T, (R)2 * d * hT);
                const R gX = fma((R)2, k_X, (R)2 * d * hL);
                const R dM = ccM + gM;
                const R dT = ccT + gT;
                const R numM = fma(ccM - gM, Pm[q],
                                   fma((R)4 * k_M, Pnb, (R)4 * d * fma(hM, Pid, ginf)));
                R inv = 0;
                if constexpr (sizeof(R) == 8) {
                    inv = rcp_nr(dM * dT);
                    Pnew = numM * (dT * inv);
                } else {
                    Pnew = div_nr(numM, dM);
                }
                const R rhs = fma(ccT - gT, Tm[q],
                              fma((R)4 * k_T, Tnb,
                              fma(ccX - gX, Pm[q],
                              fma(-(ccX + gX), Pnew,
                              fma((R)4 * k_X, Pnb,
                                  (R)4 * d * fma(hT, Tid, fma(hL, Pid, qinf)))))));
                if constexpr (sizeof(R) == 8) Tnew = rhs * (dM * inv);
                else Tnew = div_nr(rhs, dT);
                // applied flux (FP64) and its compensated integral
                const double Ts = 0.5 * ((double)Tnew + (double)Tm[q]);
                const double Ps = 0.5 * ((double)Pnew + (double)Pm[q]);
                const double g = W.hM[side] * ((Pinf - (double)pref[q]) - Ps) + W.ginf[side];
                const double qh = W.hT[side] * ((Tinf - tref) - Ts)
                                + rc.Lv * W.hM[side] * ((Pinf - (double)pref[q]) - Ps) + W.qinf[side];
                double *fw = s_flux[s];
                fw[side * 2] = qh;
                fw[side * 2 + 1] = g;
                neumaier_add(fw[4 + side * 2], fw[8 + side * 2], rc.dt * qh);
                neumaier_add(fw[5 + side * 2], fw[9 + side * 2], rc.dt * g);
            }
            if (!(f & (1 << 10))) { Tnew = 0; Pnew = 0; }
            Tm[q] = Tnew;   // level n-1 is no longer needed by node q
            Pm[q] = Pnew;
        }
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            R x = Tm[q]; Tm[q] = Tn[q]; Tn[q] = x;
            R y = Pm[q]; Pm[q] = Pn[q]; Pn[q] = y;
        }
    }

    // ---- write back: level n0+k and n0+k-1, fluxes, zone air
    const int64_t nend = n0 + ksteps;
    R *Tw_cur = (nend & 1) ? T1b : T0b;
    R *Pw_cur = (nend & 1) ? P1b : P0b;
    R *Tw_prv = (nend & 1) ? T0b : T1b;
    R *Pw_prv = (nend & 1) ? P0b : P1b;
    int nonfinite = 0;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int f = info[q];
        if (f & (1 << 10)) {
            const int b = t * NPT + q;
            const int s = f & 0xff;
            const WallDev &W = walls[s_wid[s]];
            const int64_t g = (int64_t)W.off + (b - s_wstart[s]);
            if (!(isfinite(Tn[q]) && isfinite(Pn[q]))) nonfinite = 1;
            Tw_cur[g] = Tn[q];
            Pw_cur[g] = Pn[q];
            Tw_prv[g] = Tm[q];
            Pw_prv[g] = Pm[q];
        }
    }
    if (nonfinite) atomicOr(bad, 1);
    __syncthreads();
    for (int q = t; q < nwb * 12; q += nthreads) {
        int s = q / 12, k = q % 12;
        flux[(int64_t)s_wid[s] * 12 + k] = s_flux[s][k];
    }
    if (t < nrb) {
        roomT[s_rid[t]] = s_room[nend & 1][t][0];
        roomP[s_rid[t]] = s_room[nend & 1][t][1];
    }
}

} // namespace dfhm
