// df_resident.hpp -- persistent DF kernel: one launch advances a chunk of k
// steps with every wall's two levels kept on chip.
//
// Work decomposition: the host packs whole walls (and, for coupled zones, a
// zone together with all of its walls) into workgroups.  The workgroup's
// walls are laid end to end in a block-local node space of threads x NPT
// slots; lane t owns the NPT consecutive nodes t*NPT .. t*NPT+NPT-1.  The
// levels n-1 and n of those nodes stay in VGPRs for the whole chunk; the
// per-node material scales are not kept per node but read from small
// per-wall LDS tables (capacity / r and conductivity scales per layer, the
// harmonic means at layer interfaces), so that a lane holds little more than
// its levels and four waves per SIMD fit.  LDS also carries the per-step lane
// halos, the lane-boundary faces, the surface constants, the zone air, the
// ambient and the flux accumulators, all sized by the largest number of walls
// and zones a workgroup of the launch holds.  HBM is touched only at the
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
// The step loop is unrolled by two so that levels n-1 and n exchange roles
// without register copies.
//
// All walls of one launch must share the law shape (a_T, a_M, b_TM, c_T,
// c_M, e_TM, f_TM), which is passed as an argument; then the face value at a
// layer interface is the harmonic mean of the layer scales times the common
// shape factor, and every scale is fixed per wall and layer.  The update is
// written divided by r = dt/dx^2 (capacities pre-divided by r), so interior
// nodes need no per-wall constant beyond the scales.
#pragma once
#include "df_kernels.hpp"

namespace dfhm {

constexpr int kResMaxWalls = 64;   // walls per workgroup (LDS tables)
constexpr int kResMaxRooms = 16;   // zones per workgroup

struct ResBlock {
    int32_t w_begin, w_end;        // range in block_walls (ascending wall ids)
    int32_t r_begin, r_end;        // range in block_rooms
    int32_t n_nodes, pad;
};

struct Shape {
    double aT, aM, bTM, cT, aC, eTM, fTM;
};

// Per-node flag word: slot (bits 0-7), left surface (8), right surface (9),
// active (10), layer (11-12), right-face table entry (13-15; kFaceNone = no
// right face: wall end or padding).
constexpr int kFaceNone = 6;

// Dynamic LDS layout of one workgroup for nt lanes, mw walls and mr zones.
struct ResLds {
    size_t halo, face, flux, surf, amb, rot, bc, room, cc, fk, wstart, wid, wroom, wside, rid, total;
};
template <typename R>
__host__ __device__ constexpr ResLds res_lds(int nt, int mw, int mr)
{
    ResLds o{};
    size_t p = 0;
    // halos and faces need one buffer each: a step's reads of them end
    // before the barrier that precedes their next write
    o.halo = p;  p += sizeof(R) * 4 * (size_t)nt;          // [4][nt]
    o.face = p;  p += sizeof(R) * 2 * (size_t)nt;          // [2][nt] kT, kM
    p = (p + 15) & ~(size_t)15;
    o.flux = p;  p += sizeof(double) * 12 * (size_t)mw;    // [mw][12]
    o.surf = p;  p += sizeof(double) * 8 * (size_t)mw;     // [2][mw][2][2]
    o.amb = p;   p += sizeof(double) * 8 * (size_t)mw;     // [2][mw][2][2]
    o.rot = p;   p += sizeof(double) * 24 * (size_t)mw;    // [mw][2][12]
    o.bc = p;    p += sizeof(double) * 16 * (size_t)mw;    // [mw][2][8]
    o.room = p;  p += sizeof(double) * 4 * (size_t)mr;     // [2][mr][2]
    p = (p + 15) & ~(size_t)15;
    o.cc = p;    p += sizeof(R) * 6 * (size_t)mw;          // [mw][3][2]
    p = (p + 15) & ~(size_t)15;
    o.fk = p;    p += sizeof(R) * 16 * (size_t)mw;         // [mw][8][2]
    o.wstart = p; p += sizeof(int32_t) * ((size_t)mw + 1);
    o.wid = p;   p += sizeof(int32_t) * (size_t)mw;
    o.wroom = p; p += sizeof(int32_t) * (size_t)mw;
    o.wside = p; p += sizeof(int32_t) * (size_t)mw;
    o.rid = p;   p += sizeof(int32_t) * (size_t)mr;
    o.total = (p + 15) & ~(size_t)15;
    return o;
}

// Keeps the scheduler from interleaving the nodes of a lane (bounds the
// live registers per lane so that more waves fit).
#ifndef SCHED_FENCE
#define SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)
#endif

// Two values of a scale pair from LDS (one 16- or 8-byte read).
template <typename R> struct Pair { R a, b; };
template <typename R>
__device__ __forceinline__ Pair<R> lds_pair(const unsigned char *base, int off)
{
    return *(const Pair<R> *)(base + off);
}

// Register budget: four waves per SIMD for up to 4 nodes per lane (at most
// 128 VGPRs; the few loop-invariant values that do not fit are re-read from
// the L1-resident spill area each step, which costs far less than halving
// the waves that hide the latency of the FP64 pipeline and of LDS), two
// waves for 8 nodes per lane.
template <int NPT> constexpr int res_waves_per_eu() { return NPT <= 4 ? 4 : 2; }

template <typename R, int NPT, int NT>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(res_waves_per_eu<NPT>())))
k_df_resident(const ResBlock *__restrict__ blocks, const int32_t *__restrict__ block_walls,
              const int32_t *__restrict__ block_rooms, const WallDev *__restrict__ walls,
              R *T0b, R *T1b, R *P0b, R *P1b, const uint8_t *__restrict__ lay,
              const RoomDev *__restrict__ rooms, double *roomT, double *roomP,
              const double *__restrict__ sched_go, const double *__restrict__ sched_qh,
              double *__restrict__ flux, int *__restrict__ bad,
              const int64_t *__restrict__ step_base, int ksteps, int mw, int mr, RunConst rc,
              Shape sh)
{
    static_assert(NT >= 2 * kResMaxWalls, "one lane per wall side computes the ambient");
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int nthreads = NT;
    const ResLds L = res_lds<R>(NT, mw, mr);
    R *halo = (R *)(lds + L.halo);                      // [4][NT]
    R *facb = (R *)(lds + L.face);                      // [2][NT]
    double (*s_flux)[12] = (double (*)[12])(lds + L.flux);
    double *s_surf = (double *)(lds + L.surf);          // [par][slot][side][T,P]
    double *s_amb = (double *)(lds + L.amb);            // [par][slot][side][T,P]
    double (*s_rot)[2][12] = (double (*)[2][12])(lds + L.rot);
    double (*s_bc)[2][8] = (double (*)[2][8])(lds + L.bc);
    double *s_room = (double *)(lds + L.room);          // [par][zone][T,P]
    R *s_cc = (R *)(lds + L.cc);                        // [slot][layer][c0/r, cM0/r]
    R *s_fk = (R *)(lds + L.fk);                        // [slot][entry][k0, kM0]
    int32_t *s_wstart = (int32_t *)(lds + L.wstart);
    int32_t *s_wid = (int32_t *)(lds + L.wid);
    int32_t *s_wroom = (int32_t *)(lds + L.wroom);      // local zone or -1
    int32_t *s_wside = (int32_t *)(lds + L.wside);      // side facing the zone
    int32_t *s_rid = (int32_t *)(lds + L.rid);
    auto SURF = [&](int par, int s, int side, int k) -> double & {
        return s_surf[((par * mw + s) * 2 + side) * 2 + k];
    };
    auto AMB = [&](int par, int s, int side, int k) -> double & {
        return s_amb[((par * mw + s) * 2 + side) * 2 + k];
    };
    auto ROOM = [&](int par, int z, int k) -> double & { return s_room[(par * mr + z) * 2 + k]; };

    const int t = threadIdx.x;
    const ResBlock B = blocks[blockIdx.x];
    const int nwb = B.w_end - B.w_begin;
    const int nrb = B.r_end - B.r_begin;
    const int64_t n0 = *step_base;

    // ---- wall table, zone table
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
        ROOM(n0 & 1, t, 0) = roomT[r];
        ROOM(n0 & 1, t, 1) = roomP[r];
    }
    __syncthreads();
    for (int q = t; q < nwb * 12; q += nthreads) {
        int s = q / 12, k = q % 12;
        s_flux[s][k] = flux[(int64_t)s_wid[s] * 12 + k];
    }
    // per-wall tables: zone link, surface constants, layer scales, face scales
    if (t < nwb) {
        const WallDev &W = walls[s_wid[t]];
        int lr = -1;
        for (int z = 0; z < nrb; ++z)
            if (s_rid[z] == W.room) lr = z;
        s_wroom[t] = lr;
        s_wside[t] = W.room_side;
        for (int side = 0; side < 2; ++side) {
            double *bc = s_bc[t][side];
            bc[0] = W.dx;                       // s / r
            bc[1] = W.hT[side];
            bc[2] = W.hM[side];
            bc[3] = rc.Lv * W.hM[side];
            bc[4] = W.ginf[side];
            bc[5] = W.qinf[side];
            bc[6] = Store<R>::tref(W);
            bc[7] = W.area;
        }
        const double rinv = 1.0 / W.r;
        R *cc = s_cc + 6 * t;
        R *fk = s_fk + 16 * t;
        for (int l = 0; l < 3; ++l) {
            const int la = l < W.n_layers ? l : 0;
            cc[2 * l] = (R)(W.lay[la][L_C0] * rinv);
            cc[2 * l + 1] = (R)(W.lay[la][L_CM0] * rinv);
            fk[4 * l] = (R)W.lay[la][L_K0];
            fk[4 * l + 1] = (R)W.lay[la][L_KM0];
            // interface with the next layer: harmonic mean, 0 when both are 0
            const int lb = l + 1 < W.n_layers ? l + 1 : la;
            double a = W.lay[la][L_K0], bb = W.lay[lb][L_K0];
            double am = W.lay[la][L_KM0], bm = W.lay[lb][L_KM0];
            double s1 = a + bb, s2 = am + bm;
            fk[4 * l + 2] = (R)(s1 > 0.0 ? 2.0 * a * bb / s1 : 0.0);
            fk[4 * l + 3] = (R)(s2 > 0.0 ? 2.0 * am * bm / s2 : 0.0);
        }
        fk[2 * kFaceNone] = (R)0;
        fk[2 * kFaceNone + 1] = (R)0;
        fk[2 * kFaceNone + 2] = (R)0;
        fk[2 * kFaceNone + 3] = (R)0;
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

    // ---- per-node set-up: levels, table offsets, flags
    const int cb = (int)(n0 & 1);
    const R *Tc = cb ? T1b : T0b;
    const R *Pc = cb ? P1b : P0b;
    const R *Tp = (n0 == 0) ? Tc : (cb ? T0b : T1b);
    const R *Pp = (n0 == 0) ? Pc : (cb ? P0b : P1b);

    R Ta_[NPT], Pa_[NPT], Tb_[NPT], Pb_[NPT];   // two level buffers (roles alternate)
    int info[NPT];
    int coff[NPT], koff[NPT];                   // byte offsets into the scale tables
    {
        int slot = 0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int b = t * NPT + q;
            Ta_[q] = Pa_[q] = Tb_[q] = Pb_[q] = 0;
            info[q] = kFaceNone << 13;
            coff[q] = (int)L.cc;
            koff[q] = (int)(L.fk + sizeof(R) * 2 * kFaceNone);
            if (b < B.n_nodes) {
                while (b >= s_wstart[slot + 1]) ++slot;
                const WallDev &W = walls[s_wid[slot]];
                const int j = b - s_wstart[slot];
                const int64_t g = (int64_t)W.off + j;
                Ta_[q] = Tp[g]; Pa_[q] = Pp[g];
                Tb_[q] = Tc[g]; Pb_[q] = Pc[g];
                const int la = lay[g];
                int fe = kFaceNone;
                if (j < W.nx - 1) fe = lay[g + 1] == la ? 2 * la : 2 * la + 1;
                info[q] = slot | ((j == 0) << 8) | ((j == W.nx - 1) << 9) | (1 << 10) | (la << 11) |
                          (fe << 13);
                coff[q] = (int)(L.cc + sizeof(R) * (6 * slot + 2 * la));
                koff[q] = (int)(L.fk + sizeof(R) * (16 * slot + 2 * fe));
            }
        }
    }
    const R aT = (R)sh.aT, aM = (R)sh.aM, bTM = (R)sh.bTM, cT = (R)sh.cT, aC = (R)sh.aC,
            eTM = (R)sh.eTM, fTM = (R)sh.fTM;
    // FP64 stores absolute values: references are constants; FP32 stores
    // deviations from each wall's initial state
    R thref[NPT], pref[NPT];
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        if constexpr (sizeof(R) == 8) {
            thref[q] = (R)-273.15;
            pref[q] = (R)0;
        } else {
            const WallDev &W = walls[s_wid[info[q] & 0xff]];
            thref[q] = Store<R>::thref(W);
            pref[q] = Store<R>::pref(W);
        }
    }
    const R ps_inv = (R)(1.0 / 610.94);
    __syncthreads();
    int amb_zone = -1;
    if (amb_lane && s_wroom[amb_slot] >= 0 && s_wside[amb_slot] == amb_side) amb_zone = s_wroom[amb_slot];

    // One DF step from (Tm, Pm) = level n-1 and (Tn, Pn) = level n; leaves
    // level n+1 in (Tm, Pm).
    auto step = [&](R (&Tm)[NPT], R (&Pm)[NPT], const R (&Tn)[NPT], const R (&Pn)[NPT],
                    const int64_t n) __attribute__((always_inline)) {
        const int par = (int)(n & 1);
        // ---- A: publish halos, surface values and the ambient at t^n
        R *hp = halo;
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
                    SURF(par, s, side, 0) = s_bc[s][side][6] + (double)Tn[q];
                    SURF(par, s, side, 1) = (double)pref[q] + (double)Pn[q];
                }
            }
        }
        if (amb_lane) {
            double Ta, Pa;
            double *st = s_rot[amb_slot][amb_side];
            if (amb_zone >= 0) {
                Ta = ROOM(par, amb_zone, 0);
                Pa = ROOM(par, amb_zone, 1);
            } else {
                Ta = st[0] + st[1] * st[4];
                Pa = (st[2] + st[3] * st[6]) * psat_th(Ta - 273.15);
            }
            AMB(par, amb_slot, amb_side, 0) = Ta;
            AMB(par, amb_slot, amb_side, 1) = Pa;
            const double sT = st[4], cTr = st[5], sR = st[6], cR = st[7];
            st[4] = fma(sT, st[9], cTr * st[8]);
            st[5] = fma(cTr, st[9], -sT * st[8]);
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
            const double Ta = ROOM(par, t, 0), Pa = ROOM(par, t, 1);
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
                const int side = s_wside[s];
                const double *bc = s_bc[s][side];
                const double Ts = SURF(par, s, side, 0), Ps = SURF(par, s, side, 1);
                G += bc[7] * bc[2] * (Ps - Pa);
                Q += bc[7] * (bc[1] * (Ts - Ta) + bc[3] * (Ps - Pa));
            }
            ROOM(par ^ 1, t, 1) = Pa + rc.dt * G / (mass / rc.Pv_ref);
            ROOM(par ^ 1, t, 0) = Ta + rc.dt * Q / (mass * cma);
        }
        R kT[NPT], kM[NPT], phn[NPT];
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const Pair<R> k0 = lds_pair<R>(lds, koff[q]);
            // a node without a right face (wall end, padding) has zero scales;
            // its face state is its own, so that nothing from the next wall or
            // from padding enters its arithmetic (and no NaN can leak in)
            const bool live = (info[q] >> 13) != kFaceNone;
            const R Tr = live ? (q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb) : Tn[q];
            const R Pr = live ? (q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb) : Pn[q];
            const R thn = thref[q] + Tn[q];
            const R thf = fma((R)0.5, Tn[q] + Tr, thref[q]);
            const R Pf = fma((R)0.5, Pn[q] + Pr, pref[q]);
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
            kT[q] = k0.a * fma(aT, phi, (R)1);
            kM[q] = k0.b * fma(aM * phi, phi, (R)1);
            SCHED_FENCE();
        }
        R *fp = facb;
        fp[t] = kT[NPT - 1];
        fp[nthreads + t] = kM[NPT - 1];
        __syncthreads();
        // ---- C: node updates (moisture, then heat with the new Pv)
        const R klT = t > 0 ? fp[t - 1] : (R)0;
        const R klM = t > 0 ? fp[nthreads + t - 1] : (R)0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int f = info[q];
            const Pair<R> c0 = lds_pair<R>(lds, coff[q]);
            const R th = thref[q] + Tn[q];
            const R phi = phn[q];
            const R ccT = c0.a * fma(cT, phi, (R)1);
            const R ccM = c0.b * fma(aC, phi, (R)1);
            const R ccX = fma(fTM, th, eTM) * ccM;
            const R lT = q > 0 ? kT[q > 0 ? q - 1 : 0] : klT;
            const R lM = q > 0 ? kM[q > 0 ? q - 1 : 0] : klM;
            const R lX = bTM * lM;
            const R kXq = bTM * kM[q];
            const R Tl = q > 0 ? Tn[q > 0 ? q - 1 : 0] : Tl_nb;
            const R Pl = q > 0 ? Pn[q > 0 ? q - 1 : 0] : Pl_nb;
            const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
            const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
            R Tnew, Pnew;
            if (!(f & (3 << 8))) {
                const R KM = lM + kM[q];
                const R KT = lT + kT[q];
                const R KX = lX + kXq;
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
                                              (R)2 * fma(kXq, Pr, lX * Pl)))));
                if constexpr (sizeof(R) == 8) Tnew = rhs * (dM * inv);
                else Tnew = div_nr(rhs, dT);
            } else {
                const int s = f & 0xff;
                const int side = (f >> 8) & 1 ? 0 : 1;
                const double *bc = s_bc[s][side];
                const R k_T = side == 0 ? kT[q] : lT;
                const R k_M = side == 0 ? kM[q] : lM;
                const R k_X = side == 0 ? kXq : lX;
                const R Tnb = side == 0 ? Tr : Tl;
                const R Pnb = side == 0 ? Pr : Pl;
                const double Tinf = AMB(par, s, side, 0);
                const double Pinf = AMB(par, s, side, 1);
                const double tref = bc[6];
                const R Tid = (R)(Tinf - tref);
                const R Pid = (R)(Pinf - (double)pref[q]);
                const R d = (R)bc[0];                      // s / r
                const R hT = (R)bc[1], hM = (R)bc[2];
                const R hL = (R)bc[3];
                const R ginf = (R)bc[4], qinf = (R)bc[5];
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
                const double g = bc[2] * ((Pinf - (double)pref[q]) - Ps) + bc[4];
                const double qh = bc[1] * ((Tinf - tref) - Ts)
                                + bc[3] * ((Pinf - (double)pref[q]) - Ps) + bc[5];
                double *fw = s_flux[s];
                fw[side * 2] = qh;
                fw[side * 2 + 1] = g;
                neumaier_add(fw[4 + side * 2], fw[8 + side * 2], rc.dt * qh);
                neumaier_add(fw[5 + side * 2], fw[9 + side * 2], rc.dt * g);
            }
            if (!(f & (1 << 10))) { Tnew = 0; Pnew = 0; }
            Tm[q] = Tnew;   // level n-1 is no longer needed by node q
            Pm[q] = Pnew;
            SCHED_FENCE();
        }
    };

    // buffers (a, b) hold (n-1, n); after a step a holds n+1, so the next
    // step runs with the roles exchanged
    int i = 0;
    for (; i + 1 < ksteps; i += 2) {
        step(Ta_, Pa_, Tb_, Pb_, n0 + i);
        step(Tb_, Pb_, Ta_, Pa_, n0 + i + 1);
    }
    if (i < ksteps) {
        step(Ta_, Pa_, Tb_, Pb_, n0 + i);
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            R x = Ta_[q]; Ta_[q] = Tb_[q]; Tb_[q] = x;
            R y = Pa_[q]; Pa_[q] = Pb_[q]; Pb_[q] = y;
        }
    }
    // now (Ta_, Pa_) = level n0+k-1 and (Tb_, Pb_) = level n0+k

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
            if (!(isfinite(Tb_[q]) && isfinite(Pb_[q]))) nonfinite = 1;
            Tw_cur[g] = Tb_[q];
            Pw_cur[g] = Pb_[q];
            Tw_prv[g] = Ta_[q];
            Pw_prv[g] = Pa_[q];
        }
    }
    if (nonfinite) atomicOr(bad, 1);
    __syncthreads();
    for (int q = t; q < nwb * 12; q += nthreads) {
        int s = q / 12, k = q % 12;
        flux[(int64_t)s_wid[s] * 12 + k] = s_flux[s][k];
    }
    if (t < nrb) {
        roomT[s_rid[t]] = ROOM(nend & 1, t, 0);
        roomP[s_rid[t]] = ROOM(nend & 1, t, 1);
    }
}

} // namespace dfhm
