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

template <typename R>
__device__ __forceinline__ R magnus_exp_neg(R th)
{
    // exp(-17.625 theta / (theta + 243.04)); phi = P exp(-a) / 610.94
    return exp(-(R)17.625 * th / (th + (R)243.04));
}
template <>
__device__ __forceinline__ float magnus_exp_neg<float>(float th)
{
    return __expf(-17.625f * th / (th + 243.04f));
}

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
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t s_wstart[kResMaxWalls + 1];
    __shared__ int32_t s_wid[kResMaxWalls];
    __shared__ int32_t s_wroom[kResMaxWalls];           // local zone or -1
    __shared__ double s_flux[kResMaxWalls][12];
    __shared__ double s_surf[2][kResMaxWalls][2][2];   // [par][slot][side][T,P] level n
    __shared__ double s_room[2][kResMaxRooms][2];      // [par][zone][T,P]
    __shared__ int32_t s_rid[kResMaxRooms];

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
    // nodes of one lane may lie in different walls: per-node references
    const R aT = (R)sh.aT, aM = (R)sh.aM, bTM = (R)sh.bTM, cT = (R)sh.cT, aC = (R)sh.aC,
            eTM = (R)sh.eTM, fTM = (R)sh.fTM;
    R thref[NPT], pref[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const WallDev &W = walls[s_wid[info[q] & 0xff]];
        thref[q] = Store<R>::thref(W);
        pref[q] = Store<R>::pref(W);
    }
    __syncthreads();

    for (int i = 0; i < ksteps; ++i) {
        // Tm/Pm = level n-1, Tn/Pn = level n; the step leaves n+1 in Tm/Pm
        // and the swap at its end restores the roles
        const int64_t n = n0 + i;
        const int par = (int)(n & 1);
        // ---- A: publish halos and surface values
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
                    const WallDev &W = walls[s_wid[s]];
                    const int side = (f >> 8) & 1 ? 0 : 1;
                    s_surf[par][s][side][0] = Store<R>::tref(W) + (double)Tn[q];
                    s_surf[par][s][side][1] = (double)pref[q] + (double)Pn[q];
                }
            }
        }
        __syncthreads();
        // ---- B: faces, zones
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
        R kT[NPT], kM[NPT], kX[NPT];
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
            const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
            const R thf = thref[q] + (R)0.5 * (Tn[q] + Tr);
            const R Pf = pref[q] + (R)0.5 * (Pn[q] + Pr);
            const R phi = Pf * magnus_exp_neg<R>(thf) * (R)(1.0 / 610.94);
            // a node without a right face (wall end, padding) has zero scales;
            // the select keeps a non-physical face state from leaking a NaN
            const bool live = kf0[q] != (R)0 || kMf0[q] != (R)0;
            kT[q] = live ? kf0[q] * ((R)1 + aT * phi) : (R)0;
            kM[q] = live ? kMf0[q] * ((R)1 + aM * phi * phi) : (R)0;
            kX[q] = bTM * kM[q];
        }
        R *fp = facb + par * 3 * nthreads;
        fp[t] = kT[NPT - 1];
        fp[nthreads + t] = kM[NPT - 1];
        fp[2 * nthreads + t] = kX[NPT - 1];
        __syncthreads();
        // ---- C: node updates
        const R klT = t > 0 ? fp[t - 1] : (R)0;
        const R klM = t > 0 ? fp[nthreads + t - 1] : (R)0;
        const R klX = t > 0 ? fp[2 * nthreads + t - 1] : (R)0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int f = info[q];
            const R th = thref[q] + Tn[q];
            const R P = pref[q] + Pn[q];
            const R phi = P * magnus_exp_neg<R>(th) * (R)(1.0 / 610.94);
            const R ccT = c0s[q] * ((R)1 + cT * phi);
            const R ccM = cM0s[q] * ((R)1 + aC * phi);
            const R ccX = (eTM + fTM * th) * ccM;
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
                Pnew = ((ccM - KM) * Pm[q] + (R)2 * (kM[q] * Pr + lM * Pl)) / (ccM + KM);
                const R KT = lT + kT[q];
                const R KX = lX + kX[q];
                const R rhs = (ccT - KT) * Tm[q] + (R)2 * (kT[q] * Tr + lT * Tl)
                            + (ccX - KX) * Pm[q] - (ccX + KX) * Pnew
                            + (R)2 * (kX[q] * Pr + lX * Pl);
                Tnew = rhs / (ccT + KT);
            } else {
                const int s = f & 0xff;
                const int side = (f >> 8) & 1 ? 0 : 1;
                const WallDev &W = walls[s_wid[s]];
                const R k_T = side == 0 ? kT[q] : lT;
                const R k_M = side == 0 ? kM[q] : lM;
                const R k_X = side == 0 ? kX[q] : lX;
                const R Tnb = side == 0 ? Tr : Tl;
                const R Pnb = side == 0 ? Pr : Pl;
                double Tinf, Pinf;
                if (W.room >= 0 && W.room_side == side) {
                    const int z = s_wroom[s];
                    Tinf = s_room[par][z][0];
                    Pinf = s_room[par][z][1];
                } else {
                    const double tt = (double)n * rc.dt;
                    Tinf = sine_at(W.Tamb[side], tt);
                    Pinf = sine_at(W.RHamb[side], tt) * psat_th(Tinf - 273.15);
                }
                const double tref = Store<R>::tref(W);
                const R Tid = (R)(Tinf - tref);
                const R Pid = (R)(Pinf - (double)pref[q]);
                const R d = (R)W.dx;                       // s / r
                const R hT = (R)W.hT[side], hM = (R)W.hM[side];
                const R hL = (R)(rc.Lv * W.hM[side]);
                const R ginf = (R)W.ginf[side], qinf = (R)W.qinf[side];
                Pnew = ((ccM - (R)2 * k_M - (R)2 * d * hM) * Pm[q] + (R)4 * k_M * Pnb
                        + (R)4 * d * (hM * Pid + ginf))
                     / (ccM + (R)2 * k_M + (R)2 * d * hM);
                const R rhs = (ccT - (R)2 * k_T - (R)2 * d * hT) * Tm[q] + (R)4 * k_T * Tnb
                            + (R)4 * d * hT * Tid
                            + (ccX - (R)2 * k_X - (R)2 * d * hL) * Pm[q]
                            - (ccX + (R)2 * k_X + (R)2 * d * hL) * Pnew
                            + (R)4 * k_X * Pnb + (R)4 * d * hL * Pid + (R)4 * d * qinf;
                Tnew = rhs / (ccT + (R)2 * k_T + (R)2 * d * hT);
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
        const R Tcur = Tn[q], Pcur = Pn[q];
        const R Tprv = Tm[q], Pprv = Pm[q];
        if (!(isfinite(Tcur) && isfinite(Pcur))) nonfinite = 1;
        Tw_cur[g] = Tcur;
        Pw_cur[g] = Pcur;
        Tw_prv[g] = Tprv;
        Pw_prv[g] = Pprv;
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
