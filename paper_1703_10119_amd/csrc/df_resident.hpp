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
//      one lane per wall side publishes the ambient and the incident
//      radiation at t^n;
//   B  lanes read the neighbour halos, evaluate the NPT right faces at the
//      face-averaged state (Sec. 3.1) and publish the last one; one lane per
//      zone advances the zone air by forward Euler from the level-n surfaces
//      (Sec. 5.3, eq. wbse_tn_exp) and adds the long-wave exchange among the
//      zone's surfaces (Sec. 2) to their heat sources;
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
constexpr int kResMaxLinks = 8;    // inter-zone links per zone

struct ResBlock {
    int32_t w_begin, w_end;        // range in the slot table (ascending wall ids)
    int32_t r_begin, r_end;        // range in block_rooms
    int32_t n_nodes, pad;
};

// One wall of a workgroup: its id, its node range in the workgroup
// ([wstart, wend), lanes own consecutive nodes) and its first node in the
// level arrays; written by the packer, so that the set-up reads one record
// per wall instead of walking the wall table.
struct ResSlot {
    int32_t wid, wstart, wend, off;
};

struct Shape {
    double aT, aM, bTM, cT, aC, eTM, fTM;
};

// Per-node flag word: slot (bits 0-7), left surface (8), right surface (9),
// active (10), layer (11-12), right-face table entry (13-15; kFaceNone = no
// right face: wall end or padding).
constexpr int kFaceNone = 6;

// One wall's record in LDS (fixed stride, so that every field sits at a
// compile-time offset from the record base).
template <typename R> struct WallRec {
    double flux[12];          // now q, g per side; Neumaier sums; compensations
    double surf[2][2][2];     // [parity][side][T, P] surface values of level n
    double amb[2][2][4];      // [parity][side]: the surface exchange with the air of
                              // t^n, A_q = h_T (T_inf - T ref) + L_v h_M (P_inf - P ref) + q_inf,
                              // A_g = h_M (P_inf - P ref) + g_inf, then 4 dx A_q, 4 dx A_g
    double rot[2][12];        // per side: T mean, amp, RH mean, amp, phase sin/cos, step sin/cos
    double bc[2][8];          // per side: 2 dx h_T, h_T, h_M, L_v h_M, 2 dx h_M, 2 dx L_v h_M,
                              // T ref, area (dx = s / r: the update is divided by r)
    double src[2][4];         // per side: g_inf, q_inf, 4 dx
    R cc[4][4];               // per layer: c0 / r, cM0 / r, theta ref, Pv ref
    R fk[8][4];               // per entry: k0, kM0 (layer, interface with the next, none),
                              // theta ref, Pv ref
    int32_t wstart, wend, wid, wroom, wside, off, pad[2];
};
// A wall's radiative sources (extended variant only, in LDS after the wall
// records, so that the other variants keep the smaller footprint).
struct RadRec {
    double qx[2][2];          // [parity][side] heat source at t^n (incident, plus the
                              // long-wave exchange on a zone side)
    double rotq[2][6];        // per side: incident mean, amp, phase sin/cos, step sin/cos
    double esig, pad;         // s eps sigma of the zone side
};
struct RoomRec {
    double air[2][2];         // [parity][T, P]
    double lg[kResMaxLinks];  // inter-zone links: flow (kg/s) and the partner's slot
    int32_t lslot[kResMaxLinks];
    int32_t rid, nlink, nwall, pad;
    uint8_t wslot[kResMaxWalls];   // slots of the zone's walls (ascending)
};
// Pointers the kernel needs only after its step loop (read from device
// memory there, so that they do not occupy scalar registers through the loop).
struct ResIO {
    void *T[2], *P[2];
    double *flux, *roomT, *roomP;
    int *bad;
};

// Dynamic LDS layout of one workgroup for nt lanes of npt nodes, mw walls and
// mr zones: FP32 first keeps the low parts of its compensated levels (two
// levels x two fields x npt per lane, private to the lane); then the halos
// and faces, one buffer each (a step's reads of them end before the barrier
// that precedes their next write).  (The Table 1 law keeps a third
// lane-boundary face value, k_TM.)
template <typename R> __host__ __device__ constexpr size_t res_off_halo(int nt, int npt)
{
    return sizeof(R) == 4 ? (size_t)16 * nt * npt : 0;
}
template <typename R> __host__ __device__ constexpr size_t res_off_rc(int nt, int npt, int law)
{
    return res_off_halo<R>(nt, npt) + (((sizeof(R) * (law ? 7 : 6) * (size_t)nt) + 15) & ~(size_t)15);
}
template <typename R> __host__ __device__ constexpr size_t res_off_walls(int nt, int npt, int law)
{
    return res_off_rc<R>(nt, npt, law) + 64;
}
template <typename R> __host__ __device__ constexpr size_t res_lds_bytes(int nt, int npt, int mw, int mr,
                                                                        bool ext, int law)
{
    return res_off_walls<R>(nt, npt, law) +
           (sizeof(WallRec<R>) + (ext ? sizeof(RadRec) : 0)) * (size_t)mw + sizeof(RoomRec) * (size_t)mr;
}

// FP32 level update with a compensated sum (Kahan): the level is the pair
// hi + lo, and the step adds its increment to it, so that the rounding of
// hi to FP32 is carried in lo instead of being lost.  Without it each step
// rounds every node to the FP32 grid of its deviation (about 1e-6 K), and
// where the state changes slowly those roundings repeat with the same sign
// for thousands of steps; the wall's slowest modes (decay times of 1e4 s
// and more) add them up to 1e-2 K over 1e5 steps.  The increment itself is
// small, so its own FP32 error is far below the grid.
template <typename R>
__device__ __forceinline__ void comp_add(R hi, R lo, R inc, R &nhi, R &nlo)
{
    const R y = inc + lo;
    const R s = hi + y;
    nlo = y - (s - hi);
    nhi = s;
}

// Keeps the scheduler from interleaving the nodes of a lane (bounds the
// live registers per lane so that more waves fit).
#define SCHED_FENCE() __builtin_amdgcn_sched_barrier(0)

// A scale pair and the node's storage references from LDS: FP64 stores
// absolute values (references are the constants -273.15 K and 0 Pa) and
// reads the pair (16 B); FP32 stores deviations from the wall's initial state
// and reads the pair with the wall's references (16 B).
template <typename R> struct Quad { R a, b, th, p; };
template <typename R>
__device__ __forceinline__ Quad<R> lds_scales(const unsigned char *base, int off)
{
    Quad<R> q;
    if constexpr (sizeof(R) == 8) {
        const double2 v = *(const double2 *)(base + off);
        q.a = v.x; q.b = v.y; q.th = -273.15; q.p = 0.0;
    } else {
        q = *(const Quad<R> *)(base + off);
    }
    return q;
}

// Register budget (waves per SIMD).  FP64 with up to 4 nodes per lane:
// three waves (168 VGPRs).  At four (128 VGPRs) the FP64 step loop fits only
// by spilling loop-invariant values -- chiefly the exponential's polynomial
// coefficients, which the compiler keeps in registers -- and every lane
// writes that spill area once per launch: 2.8 GB per launch of the 65,536 x
// 1001 batch.  Measured there: three waves 0.257 ms per step in 20-step
// launches against 0.282 with four, and 0.8 % slower in 1000-step launches.
// FP32 with up to 4 nodes per lane, and 512-lane workgroups: four waves
// (FP32 measured against three: +6 % on the 65,536 x 1001 batch, +2-4 % with
// zones).  8 nodes per lane: two waves.  (FP64 2 -> 4 waves once gave +27 %, before the LDS scale tables.)
// Kernel variants: only what a launch needs is compiled in, since every
// extra line of the step loop competes for the registers of the node work.
constexpr int kModePlain = 0;   // walls without zones or radiative sources
constexpr int kModeZones = 1;   // zones coupled to walls
constexpr int kModeExt = 2;     // radiative sources and / or linked zones

__host__ __device__ constexpr int res_waves(int rbytes, int npt, int nt)
{
    if (npt > 4) return 2;
    // 512-lane workgroups keep four (three would leave room for only one
    // workgroup per CU)
    return rbytes == 8 && nt <= 256 ? 3 : 4;
}
template <typename R, int NPT, int NT, int MODE, int LAW> constexpr int res_waves_per_eu()
{
    return res_waves((int)sizeof(R), NPT, NT);
}

// LAW: 0 = the shape law (scales x the launch's common shape factors),
// 1 = the Table 1 law (scales x that material's functions, which factor the
// same way: k_TT = k0 lambda, k_M = kM0 K, k_TM = kM0 L_v delta_v, so the
// harmonic interface means of the scale tables still apply).
template <typename R, int NPT, int NT, int MODE, int LAW>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(res_waves_per_eu<R, NPT, NT, MODE, LAW>())))
k_df_resident(const ResBlock *__restrict__ blocks, const ResSlot *__restrict__ slots,
              const int32_t *__restrict__ block_rooms, const WallDev *__restrict__ walls,
              const R *T0b, const R *T1b, const R *P0b, const R *P1b,
              const uint8_t *__restrict__ lay, const RoomDev *__restrict__ rooms,
              const double *roomT, const double *roomP, const double *__restrict__ sched_go,
              const double *__restrict__ sched_qh, const double *flux,
              const int64_t *__restrict__ step_base, const ResIO *__restrict__ io,
              const ZoneLinkDev *__restrict__ zlinks, int ksteps, int mw, RunConst rc, Shape sh)
{
    static_assert(NT >= 2 * kResMaxWalls, "one lane per wall side computes the ambient");
    constexpr bool ZON = MODE != kModePlain, EXT = MODE == kModeExt;
    static_assert(sizeof(WallRec<R>) % 16 == 0 && sizeof(RoomRec) % 16 == 0 &&
                      sizeof(RadRec) % 16 == 0,
                  "records keep 16-byte alignment");
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int nthreads = NT;
    constexpr size_t kRc = res_off_rc<R>(NT, NPT, LAW), kWalls = res_off_walls<R>(NT, NPT, LAW);
    constexpr bool CMP = sizeof(R) == 4;                 // compensated FP32 levels
    // low parts of the levels: [buffer][T, P][node of the lane][lane]; the
    // buffers pair with the two register level buffers below
    R *lo_a = (R *)lds;
    R *lo_b = lo_a + 2 * NPT * NT;
    R *halo = (R *)(lds + res_off_halo<R>(NT, NPT));    // [4][NT]
    R *facb = halo + 4 * NT;                             // [2][NT], [3][NT] under the Table 1 law
    double *s_rc = (double *)(lds + kRc);                // dt, Lv, rho_a, c_pa, c_pv, Pv_ref
    WallRec<R> *wr = (WallRec<R> *)(lds + kWalls);
    RadRec *xr = (RadRec *)(lds + kWalls + sizeof(WallRec<R>) * (size_t)mw);   // EXT only
    RoomRec *rr = (RoomRec *)(lds + kWalls + (sizeof(WallRec<R>) + (EXT ? sizeof(RadRec) : 0)) *
                                                 (size_t)mw);

    const int t = threadIdx.x;
    const ResBlock B = blocks[blockIdx.x];
    const int nwb = B.w_end - B.w_begin;
    const int nrb = B.r_end - B.r_begin;
    const int64_t n0 = *step_base;

    // ---- run constants, wall slots, zone table
    if (t == 0) {
        s_rc[0] = rc.dt; s_rc[1] = rc.Lv; s_rc[2] = rc.rho_a;
        s_rc[3] = rc.c_pa; s_rc[4] = rc.c_pv; s_rc[5] = rc.Pv_ref;
    }
    if (t < nwb) {
        const ResSlot S = slots[B.w_begin + t];
        wr[t].wid = S.wid;
        wr[t].wstart = S.wstart;
        wr[t].wend = S.wend;
        wr[t].off = S.off;
    }
    if (ZON && t < nrb) {
        int r = block_rooms[B.r_begin + t];
        rr[t].rid = r;
        rr[t].air[n0 & 1][0] = roomT[r];
        rr[t].air[n0 & 1][1] = roomP[r];
    }
    __syncthreads();
    for (int q = t; q < nwb * 12; q += nthreads) {
        int s = q / 12, k = q % 12;
        wr[s].flux[k] = flux[(int64_t)wr[s].wid * 12 + k];
    }
    // per-wall tables: zone link, surface constants, layer scales, face scales
    if (t < nwb) {
        WallRec<R> &X = wr[t];
        const WallDev &W = walls[X.wid];
        int lr = -1;
        for (int z = 0; z < nrb; ++z)
            if (rr[z].rid == W.room) lr = z;
        X.wroom = lr;
        X.wside = W.room_side;
        if constexpr (EXT) {
            xr[t].esig = W.esig;
            xr[t].qx[0][0] = xr[t].qx[0][1] = xr[t].qx[1][0] = xr[t].qx[1][1] = 0.0;
        }
        for (int side = 0; side < 2; ++side) {
            double *bc = X.bc[side];
            const double d2 = 2.0 * W.dx;       // 2 s / r
            bc[0] = d2 * W.hT[side];
            bc[1] = W.hT[side];
            bc[2] = W.hM[side];
            bc[3] = rc.Lv * W.hM[side];
            bc[4] = d2 * W.hM[side];
            bc[5] = d2 * (rc.Lv * W.hM[side]);
            bc[6] = Store<R>::tref(W);
            bc[7] = W.area;
            X.src[side][0] = W.ginf[side];
            X.src[side][1] = W.qinf[side];
            X.src[side][2] = 4.0 * W.dx;
            X.src[side][3] = 0.0;
        }
        const double rinv = 1.0 / W.r;
        for (int l = 0; l < 3; ++l) {
            const int la = l < W.n_layers ? l : 0;
            X.cc[l][0] = (R)(W.lay[la][L_C0] * rinv);
            X.cc[l][1] = (R)(W.lay[la][L_CM0] * rinv);
            X.fk[2 * l][0] = (R)W.lay[la][L_K0];
            X.fk[2 * l][1] = (R)W.lay[la][L_KM0];
            // interface with the next layer: harmonic mean, 0 when both are 0
            const int lb = l + 1 < W.n_layers ? l + 1 : la;
            double a = W.lay[la][L_K0], bb = W.lay[lb][L_K0];
            double am = W.lay[la][L_KM0], bm = W.lay[lb][L_KM0];
            double s1 = a + bb, s2 = am + bm;
            X.fk[2 * l + 1][0] = (R)(s1 > 0.0 ? 2.0 * a * bb / s1 : 0.0);
            X.fk[2 * l + 1][1] = (R)(s2 > 0.0 ? 2.0 * am * bm / s2 : 0.0);
        }
        X.cc[3][0] = X.cc[3][1] = (R)1;     // padding nodes: any finite capacity
        for (int e = 0; e < 4; ++e) { X.cc[e][2] = Store<R>::thref(W); X.cc[e][3] = Store<R>::pref(W); }
        for (int e = 0; e < 8; ++e) { X.fk[e][2] = Store<R>::thref(W); X.fk[e][3] = Store<R>::pref(W); }
        X.fk[kFaceNone][0] = X.fk[kFaceNone][1] = (R)0;
        X.fk[7][0] = X.fk[7][1] = (R)0;
        if constexpr (LAW == 1) X.fk[7][0] = (R)(rc.cw * rinv);   // c_w / r of the moisture heat
    }
    // each zone's wall slots, and its inter-zone links: partner zones sit in
    // this workgroup (the packer keeps linked zones together); resolve them to
    // local slots
    if (ZON && t < nrb) {
        int nwz = 0;
        for (int s = 0; s < nwb; ++s)
            if (walls[wr[s].wid].room == rr[t].rid) rr[t].wslot[nwz++] = (uint8_t)s;
        rr[t].nwall = nwz;
        rr[t].nlink = 0;
        if constexpr (EXT) {
            const RoomDev &Rm = rooms[rr[t].rid];
            int nl = 0;
            for (int l = Rm.l_begin; l < Rm.l_end && nl < kResMaxLinks; ++l) {
                const ZoneLinkDev L = zlinks[l];
                for (int z = 0; z < nrb; ++z)
                    if (rr[z].rid == L.partner) {
                        rr[t].lslot[nl] = z;
                        rr[t].lg[nl] = L.g;
                        ++nl;
                    }
            }
            rr[t].nlink = nl;
        }
    }

    // ---- ambient lanes: one per wall side; the outdoor sinusoids advance by
    // an exact rotation through the chunk, anchored at t^n0 (state in LDS)
    // In the walls-only variant they start at the second wave: the first wave
    // of every workgroup holds a left surface node, and the waves of equal
    // index of the resident workgroups share a SIMD, so the ambient work
    // would pile onto one SIMD per CU.  (With zones, measured, the first wave
    // is the better place.)
    constexpr int kAmb0 = (MODE == kModePlain && NT >= 64 + 2 * kResMaxWalls) ? 64 : 0;
    const int ta = t - kAmb0;
    const bool amb_lane = ta >= 0 && ta < 2 * nwb;
    const int amb_slot = ta >> 1, amb_side = ta & 1;
    if (amb_lane) {
        const WallDev &W = walls[wr[amb_slot].wid];
        const double *ST = W.Tamb[amb_side], *SR = W.RHamb[amb_side];
        const double t0 = (double)n0 * rc.dt;
        double *st = wr[amb_slot].rot[amb_side];
        st[0] = ST[0]; st[1] = ST[1]; st[2] = SR[0]; st[3] = SR[1];
        sincos(2.0 * dpi() * t0 / ST[2] + ST[3], &st[4], &st[5]);
        sincos(2.0 * dpi() * t0 / SR[2] + SR[3], &st[6], &st[7]);
        sincos(2.0 * dpi() * rc.dt / ST[2], &st[8], &st[9]);
        sincos(2.0 * dpi() * rc.dt / SR[2], &st[10], &st[11]);
        if constexpr (EXT) {
            const double *SQ = W.qsun[amb_side];
            double *sq = xr[amb_slot].rotq[amb_side];
            sq[0] = SQ[0]; sq[1] = SQ[1];
            sincos(2.0 * dpi() * t0 / SQ[2] + SQ[3], &sq[2], &sq[3]);
            sincos(2.0 * dpi() * rc.dt / SQ[2], &sq[4], &sq[5]);
        }
    }

    // ---- per-node set-up: levels, table offsets, flags
    const int cb = (int)(n0 & 1);
    const R *Tc = cb ? T1b : T0b;
    const R *Pc = cb ? P1b : P0b;
    const R *Tp = (n0 == 0) ? Tc : (cb ? T0b : T1b);
    const R *Pp = (n0 == 0) ? Pc : (cb ? P0b : P1b);

    R Ta_[NPT], Pa_[NPT], Tb_[NPT], Pb_[NPT];   // two level buffers (roles alternate)
    int info[NPT];
    // LDS byte offsets of a node's capacity and face scale entries, both
    // 16-byte aligned, packed as 16-byte units in one register (low: capacity,
    // high: face), so that they stay in registers through the loop
    uint32_t offs[NPT];
    {
        int slot = 0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int b = t * NPT + q;
            // padding: a physical state (FP64 stores absolute values; FP32
            // deviations, where 0 is the wall's initial state)
            Ta_[q] = Tb_[q] = (R)(sizeof(R) == 8 && LAW == 0 ? 293.15 : 0.0);
            Pa_[q] = Pb_[q] = (R)(sizeof(R) == 8 && LAW == 0 ? 1000.0 : 0.0);
            if constexpr (CMP) {
                lo_a[q * NT + t] = lo_a[(NPT + q) * NT + t] = (R)0;
                lo_b[q * NT + t] = lo_b[(NPT + q) * NT + t] = (R)0;
            }
            info[q] = kFaceNone << 13;
            offs[q] = (uint32_t)((kWalls + offsetof(WallRec<R>, cc) + sizeof(R) * 4 * 3) >> 4) |
                      ((uint32_t)((kWalls + offsetof(WallRec<R>, fk) + sizeof(R) * 4 * kFaceNone) >> 4) << 16);
            if (b < B.n_nodes) {
                while (b >= wr[slot].wend) ++slot;
                const int j = b - wr[slot].wstart, nx = wr[slot].wend - wr[slot].wstart;
                const int64_t g = (int64_t)wr[slot].off + j;
                Ta_[q] = Tp[g]; Pa_[q] = Pp[g];
                Tb_[q] = Tc[g]; Pb_[q] = Pc[g];
                const int la = lay[g];
                int fe = kFaceNone;
                if (j < nx - 1) fe = lay[g + 1] == la ? 2 * la : 2 * la + 1;
                info[q] = slot | ((j == 0) << 8) | ((j == nx - 1) << 9) | (1 << 10) | (la << 11) |
                          (fe << 13);
                const int rb = (int)(kWalls + sizeof(WallRec<R>) * (size_t)slot);
                const uint32_t co = (uint32_t)(rb + (int)(offsetof(WallRec<R>, cc) + sizeof(R) * 4 * la));
                const uint32_t ko = (uint32_t)(rb + (int)(offsetof(WallRec<R>, fk) + sizeof(R) * 4 * fe));
                offs[q] = (co >> 4) | ((ko >> 4) << 16);
            }
        }
    }
    const R aT = (R)sh.aT, aM = (R)sh.aM, bTM = (R)sh.bTM, cT = (R)sh.cT, aC = (R)sh.aC,
            eTM = (R)sh.eTM, fTM = (R)sh.fTM;
    const R ps_inv = (R)(1.0 / 610.94);
    __syncthreads();
    int amb_zone = -1;
    if (amb_lane && wr[amb_slot].wroom >= 0 && wr[amb_slot].wside == amb_side) amb_zone = wr[amb_slot].wroom;

    // One DF step from (Tm, Pm) = level n-1 and (Tn, Pn) = level n; leaves
    // level n+1 in (Tm, Pm).  FP32: lm / ln hold the low parts of the same
    // levels (lm is overwritten with those of level n+1).
    auto step = [&](R (&Tm)[NPT], R (&Pm)[NPT], const R (&Tn)[NPT], const R (&Pn)[NPT],
                    R *lm, const R *ln, const int64_t n) __attribute__((always_inline)) {
        const int par = (int)(n & 1);
        // ---- A: publish halos, surface values and the ambient at t^n
        halo[t] = Tn[0];
        halo[nthreads + t] = Pn[0];
        halo[2 * nthreads + t] = Tn[NPT - 1];
        halo[3 * nthreads + t] = Pn[NPT - 1];
        if (ZON && nrb > 0) {
#pragma unroll
            for (int q = 0; q < NPT; ++q) {
                const int f = info[q];
                if (f & (3 << 8)) {
                    const int s = f & 0xff;
                    const int side = (f >> 8) & 1 ? 0 : 1;
                    double Ts = (double)Tn[q], Ps = (double)Pn[q];
                    if constexpr (CMP) {
                        Ts += (double)ln[q * NT + t];
                        Ps += (double)ln[(NPT + q) * NT + t];
                    }
                    wr[s].surf[par][side][0] = wr[s].bc[side][6] + Ts;
                    wr[s].surf[par][side][1] = (double)wr[s].cc[0][3] + Ps;
                }
            }
        }
        if (amb_lane) {
            double Ta, Pa;
            double *st = wr[amb_slot].rot[amb_side];
            if (ZON && amb_zone >= 0) {
                Ta = rr[amb_zone].air[par][0];
                Pa = rr[amb_zone].air[par][1];
            } else {
                Ta = st[0] + st[1] * st[4];
                // Ps = 2^-(C0 + C1 / (theta + 243.04)): the node work's
                // exponential, whose coefficients are in registers already
                const double d = Ta - (273.15 - 243.04);
                Pa = (st[2] + st[3] * st[6]) * exp2_bounded(-fma(kMagC1, rcp_nr(d), kMagC0));
            }
            {
                // the surface exchange with this air, in the storage frame
                const double *bc = wr[amb_slot].bc[amb_side];
                const double *sc = wr[amb_slot].src[amb_side];
                const double dPa = Pa - (double)wr[amb_slot].cc[0][3];
                const double Ag = fma(bc[2], dPa, sc[0]);
                const double Aq = fma(bc[1], Ta - bc[6], fma(bc[3], dPa, sc[1]));
                double *A = wr[amb_slot].amb[par][amb_side];
                A[0] = Aq;
                A[1] = Ag;
                A[2] = sc[2] * Aq;
                A[3] = sc[2] * Ag;
            }
            if constexpr (EXT) {
                double *sq = xr[amb_slot].rotq[amb_side];
                const double qs = sq[0] + sq[1] * sq[2];
                xr[amb_slot].qx[par][amb_side] = qs > 0.0 ? qs : 0.0;
                const double sQ = sq[2], cQ = sq[3];
                sq[2] = fma(sQ, sq[5], cQ * sq[4]);
                sq[3] = fma(cQ, sq[5], -sQ * sq[4]);
            }
            const double sT = st[4], cTr = st[5], sR = st[6], cR = st[7];
            st[4] = fma(sT, st[9], cTr * st[8]);
            st[5] = fma(cTr, st[9], -sT * st[8]);
            st[6] = fma(sR, st[11], cR * st[10]);
            st[7] = fma(cR, st[11], -sR * st[10]);
        }
        __syncthreads();
        // ---- B: faces and node humidity ratios, zones
        const R Tr_nb = t + 1 < nthreads ? halo[t + 1] : (R)0;
        const R Pr_nb = t + 1 < nthreads ? halo[nthreads + t + 1] : (R)0;
        const R Tl_nb = t > 0 ? halo[2 * nthreads + t - 1] : (R)0;
        const R Pl_nb = t > 0 ? halo[3 * nthreads + t - 1] : (R)0;
        if (ZON && t < nrb) {
            const double dt = s_rc[0], Lv = s_rc[1], rho_a = s_rc[2], c_pa = s_rc[3];
            const double c_pv = s_rc[4], Pv_ref = s_rc[5];
            const RoomDev &Rm = rooms[rr[t].rid];
            const double tt = (double)n * dt;
            const double Ta = rr[t].air[par][0], Pa = rr[t].air[par][1];
            const double mass = rho_a * Rm.volume;
            const double gv = Rm.ach * mass / 3600.0;
            const double cma = c_pa + c_pv * Pa / Pv_ref;
            const int64_t slot = (int64_t)floor(tt / Rm.sched_dt) % Rm.n_sched;
            const double go = sched_go[Rm.sched_off + slot], Qh = sched_qh[Rm.sched_off + slot];
            const double Tout = sine_at(Rm.Tout, tt);
            const double Pout = sine_at(Rm.RHout, tt) *
                                exp2_bounded(-fma(kMagC1, rcp_nr(Tout - (273.15 - 243.04)), kMagC0));
            double G = go + gv * (Pout - Pa) / Pv_ref;
            double Q = Qh + Lv * go + gv * cma * (Tout - Ta) + Lv * gv * (Pout - Pa) / Pv_ref;
            double S4 = 0.0;            // sum of T_w^4 over the zone's surfaces
            const int m = rr[t].nwall;
            for (int k = 0; k < m; ++k) {
                const int s = rr[t].wslot[k];
                const int side = wr[s].wside;
                const double *bc = wr[s].bc[side];
                const double Ts = wr[s].surf[par][side][0], Ps = wr[s].surf[par][side][1];
                G += bc[7] * bc[2] * (Ps - Pa);
                Q += bc[7] * (bc[1] * (Ts - Ta) + bc[3] * (Ps - Pa));
                if constexpr (EXT) S4 += pow4(Ts);
            }
            // airflow from the linked zones (Sec. 5.1, inter-zone sources):
            // moist-air enthalpy with theta in degC, level-n air
            if constexpr (EXT)
                for (int l = 0; l < rr[t].nlink; ++l) {
                    const RoomRec &J = rr[rr[t].lslot[l]];
                    const double g = rr[t].lg[l];
                    const double Tj = J.air[par][0], Pj = J.air[par][1];
                    const double cj = c_pa + c_pv * Pj / Pv_ref;
                    G += g * (Pj - Pa) / Pv_ref;
                    Q += g * (cj * (Tj - 273.15) - cma * (Ta - 273.15)) + Lv * g * (Pj - Pa) / Pv_ref;
                }
            rr[t].air[par ^ 1][1] = Pa + dt * G / (mass / Pv_ref);
            rr[t].air[par ^ 1][0] = Ta + dt * Q / (mass * cma);
            // long-wave exchange among the zone's surfaces (Sec. 2), level n
            if constexpr (EXT)
                for (int k = 0; k < m; ++k) {
                    const int s = rr[t].wslot[k];
                    if (xr[s].esig == 0.0) continue;
                    const int side = wr[s].wside;
                    xr[s].qx[par][side] += xr[s].esig * (S4 - (double)m * pow4(wr[s].surf[par][side][0]));
                }
        }
        R kT[NPT], kM[NPT], phn[NPT], kX[NPT];
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const Quad<R> k0 = lds_scales<R>(lds, (int)((offs[q] >> 16) << 4));
            if constexpr (LAW == 1) {
                // Table 1 law at the face state; a node without a right face
                // gets zeros (its own state may be padding at 0 K)
                const bool live = (info[q] >> 13) != kFaceNone;
                const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
                const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
                const R thf = live ? fma((R)0.5, Tn[q] + Tr, k0.th) : (R)20;
                const R Pf = live ? fma((R)0.5, Pn[q] + Pr, k0.p) : (R)1000;
                const KCoef<R> g = t1_kfun<R>(thf, Pf, (R)s_rc[1]);
                kT[q] = live ? k0.a * g.kT : (R)0;
                kM[q] = live ? k0.b * g.kM : (R)0;
                kX[q] = live ? k0.b * g.kX : (R)0;
                phn[q] = 0;
                SCHED_FENCE();
                continue;
            }
            kX[q] = 0;
            const R thr = k0.th, pr = k0.p;
            // a node without a right face (wall end, padding) has zero face
            // scales; its face state, shared with the next wall's first node,
            // a padding node (which holds a physical state) or the
            // workgroup's end, is finite, so its face is zero
            const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
            const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
            const R Pf = fma((R)0.5, Pn[q] + Pr, pr);
            R phi;                                          // phi = P / Ps at the face
            if constexpr (sizeof(R) == 8) {
                // Magnus denominators theta + 243.04 of face and node (the
                // reference theta is -273.15: absolute storage), one shared
                // reciprocal, and 1 / Ps = 2^(C0 + C1 / d).  The node's value
                // goes through the shared reciprocal, so a node without a
                // right face takes its own temperature as the face's: its
                // result then does not depend on what lies to its right
                // (the next wall, padding), to the last bit
                const R Tf2 = (info[q] >> 13) != kFaceNone ? Tn[q] + Tr : (R)2 * Tn[q];
                const R df = fma((R)0.5, Tf2, thr + (R)243.04);
                const R dn = Tn[q] + (thr + (R)243.04);
                const R inv = rcp_nr(df * dn);
                phi = Pf * exp2_bounded(fma((R)kMagC1 * dn, inv, (R)kMagC0));
                phn[q] = (pr + Pn[q]) * exp2_bounded(fma((R)kMagC1 * df, inv, (R)kMagC0));
            } else {
                const R thn = thr + Tn[q];
                const R thf = fma((R)0.5, Tn[q] + Tr, thr);
                const R af = div_nr(thf, thf + (R)243.04);
                const R an = div_nr(thn, thn + (R)243.04);
                phi = (Pf * exp_bounded(-(R)17.625 * af)) * ps_inv;
                phn[q] = ((pr + Pn[q]) * exp_bounded(-(R)17.625 * an)) * ps_inv;
            }
            kT[q] = k0.a * fma(aT, phi, (R)1);
            kM[q] = k0.b * fma(aM * phi, phi, (R)1);
            SCHED_FENCE();
        }
        facb[t] = kT[NPT - 1];
        facb[nthreads + t] = kM[NPT - 1];
        if constexpr (LAW == 1) facb[2 * nthreads + t] = kX[NPT - 1];
        __syncthreads();
        // ---- C: node updates (moisture, then heat with the new Pv)
        const R klT = t > 0 ? facb[t - 1] : (R)0;
        const R klM = t > 0 ? facb[nthreads + t - 1] : (R)0;
        R klX = 0;
        if constexpr (LAW == 1) klX = t > 0 ? facb[2 * nthreads + t - 1] : (R)0;
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            const int f = info[q];
            const Quad<R> c0 = lds_scales<R>(lds, (int)((offs[q] & 0xffffu) << 4));
            const R pr = c0.p;
            const R th = c0.th + Tn[q];
            R ccT, ccM, ccX, lX, kXq;
            const R lT = q > 0 ? kT[q > 0 ? q - 1 : 0] : klT;
            const R lM = q > 0 ? kM[q > 0 ? q - 1 : 0] : klM;
            if constexpr (LAW == 1) {
                // capacities of the Table 1 law (divided by r like the scales):
                // c_TT = c0 rho_0 c_0 + c_w f, c_M = cM0 (df/dphi)/P_s, c_TM = c_w theta c_M
                const R P = pr + Pn[q];
                R fw, gw;
                t1_isotherm<R>(th + (R)273.15, t1_ln(div_nr(P, t1_psat(th))), fw, gw);
                ccT = fma(c0.a, (R)kT1Rho0c0, wr[f & 0xff].fk[7][0] * fw);
                ccM = c0.b * div_nr(gw, P);
                ccX = ((R)rc.cw * th) * ccM;
                lX = q > 0 ? kX[q > 0 ? q - 1 : 0] : klX;
                kXq = kX[q];
            } else {
                const R phi = phn[q];
                ccT = c0.a * fma(cT, phi, (R)1);
                ccM = c0.b * fma(aC, phi, (R)1);
                ccX = fma(fTM, th, eTM) * ccM;
                lX = kXq = 0;           // k_TM = b_TM k_M on every face (below)
            }
            const R Tl = q > 0 ? Tn[q > 0 ? q - 1 : 0] : Tl_nb;
            const R Pl = q > 0 ? Pn[q > 0 ? q - 1 : 0] : Pl_nb;
            const R Tr = q + 1 < NPT ? Tn[q + 1 < NPT ? q + 1 : q] : Tr_nb;
            const R Pr = q + 1 < NPT ? Pn[q + 1 < NPT ? q + 1 : q] : Pr_nb;
            R Tnew, Pnew, Tlo = 0, Plo = 0;
            if (CMP && !(f & (3 << 8))) {
                // FP32: the update as an increment of level n-1 (the same
                // equations as below, minus (c + K) u^{n-1} on both sides),
                // from differences to the neighbours of level n
                const R KM = lM + kM[q];
                const R KT = lT + kT[q];
                const R dM = ccM + KM, dT = ccT + KT;
                const R Tmq = Tm[q], Pmq = Pm[q];
                const R dPr = Pr - Pmq, dPl = Pl - Pmq;
                const R dP = div_nr<R>((R)2 * fma(kM[q], dPr, lM * dPl), dM);
                // heat: 2 k_TM differences - (c_TM + K_TM) dP; under the shape
                // law k_TM = b_TM k_M turns the first into b_TM dM dP
                const R hX = LAW == 1 ? fma((R)2, fma(kXq, dPr, lX * dPl), -(ccX + lX + kXq) * dP)
                                      : (bTM * ccM - ccX) * dP;
                const R dTn = div_nr<R>(fma((R)2, fma(kT[q], Tr - Tmq, lT * (Tl - Tmq)), hX), dT);
                comp_add<R>(Pmq, lm[(NPT + q) * NT + t], dP, Pnew, Plo);
                comp_add<R>(Tmq, lm[q * NT + t], dTn, Tnew, Tlo);
            } else if (!(f & (3 << 8))) {
                const R KM = lM + kM[q];
                const R KT = lT + kT[q];
                const R SM = fma(kM[q], Pr, lM * Pl);
                // the shape law's k_TM is b_TM k_M on every face, so its sums
                // are b_TM times the moisture ones
                const R KX = LAW == 1 ? lX + kXq : bTM * KM;
                const R SX = LAW == 1 ? fma(kXq, Pr, lX * Pl) : bTM * SM;
                const R dM = ccM + KM, dT = ccT + KT;
                const R numM = fma(ccM - KM, Pm[q], (R)2 * SM);
                R inv = 0;
                if constexpr (sizeof(R) == 8) {
                    inv = rcp_nr(dM * dT);
                    Pnew = numM * (dT * inv);
                } else {
                    Pnew = div_nr<R>(numM, dM);
                }
                const R rhs = fma(ccT - KT, Tm[q],
                                  fma((R)2, fma(kT[q], Tr, lT * Tl),
                                      fma(ccX - KX, Pm[q],
                                          fma(-(ccX + KX), Pnew, (R)2 * SX))));
                if constexpr (sizeof(R) == 8) Tnew = rhs * (dM * inv);
                else Tnew = div_nr<R>(rhs, dT);
            } else {
                const int s = f & 0xff;
                const int side = (f >> 8) & 1 ? 0 : 1;
                WallRec<R> &X = wr[s];
                const double *bc = X.bc[side];
                const R k_T = side == 0 ? kT[q] : lT;
                const R k_M = side == 0 ? kM[q] : lM;
                const R k_X = LAW == 1 ? (side == 0 ? kXq : lX) : bTM * k_M;
                const R Tnb = side == 0 ? Tr : Tl;
                const R Pnb = side == 0 ? Pr : Pl;
                // the exchange with the air of t^n (ambient lanes, phase A)
                const double *A = X.amb[par][side];
                double Aq = A[0], Bq = A[2];
                const double Ag = A[1], Bg = A[3];
                if constexpr (EXT) {
                    const double qx = xr[s].qx[par][side];   // radiative sources
                    Aq += qx;
                    Bq = fma(X.src[side][2], qx, Bq);
                }
                // 2 r k + 2 s h (over r) per field
                const R gM = fma((R)2, k_M, (R)bc[4]);
                const R gT = fma((R)2, k_T, (R)bc[0]);
                const R gX = fma((R)2, k_X, (R)bc[5]);
                const R dM = ccM + gM;
                const R dT = ccT + gT;
                double Tmf = (double)Tm[q], Pmf = (double)Pm[q];
                if constexpr (CMP) {
                    // increment form (as for the interior), with the exchange
                    // with the air, 4 s (A - h u^{n-1}) over r
                    const R Tlm = lm[q * NT + t], Plm = lm[(NPT + q) * NT + t];
                    Tmf += (double)Tlm;
                    Pmf += (double)Plm;
                    const R EM = fma((R)-2 * (R)bc[4], Pm[q], (R)Bg);
                    const R EQ = fma((R)-2 * (R)bc[0], Tm[q], fma((R)-2 * (R)bc[5], Pm[q], (R)Bq));
                    const R dPs = Pnb - Pm[q];
                    const R dP = div_nr<R>(fma((R)4 * k_M, dPs, EM), dM);
                    const R dTn = div_nr<R>(fma((R)4 * k_T, Tnb - Tm[q],
                                             fma((R)4 * k_X, dPs, fma(-(ccX + gX), dP, EQ))), dT);
                    comp_add<R>(Pm[q], Plm, dP, Pnew, Plo);
                    comp_add<R>(Tm[q], Tlm, dTn, Tnew, Tlo);
                } else {
                    const R numM = fma(ccM - gM, Pm[q], fma((R)4 * k_M, Pnb, (R)Bg));
                    const R inv = rcp_nr(dM * dT);
                    Pnew = numM * (dT * inv);
                    const R rhs = fma(ccT - gT, Tm[q],
                                  fma((R)4 * k_T, Tnb,
                                  fma(ccX - gX, Pm[q],
                                  fma(-(ccX + gX), Pnew,
                                  fma((R)4 * k_X, Pnb, (R)Bq)))));
                    Tnew = rhs * (dM * inv);
                }
                // applied flux (FP64) and its compensated integral
                const double dt = s_rc[0];
                const double Ts = 0.5 * ((double)Tnew + (double)Tlo + Tmf);
                const double Ps = 0.5 * ((double)Pnew + (double)Plo + Pmf);
                const double g = fma(-bc[2], Ps, Ag);
                const double qh = fma(-bc[1], Ts, fma(-bc[3], Ps, Aq));
                double *fw = X.flux;
                fw[side * 2] = qh;
                fw[side * 2 + 1] = g;
                neumaier_add(fw[4 + side * 2], fw[8 + side * 2], dt * qh);
                neumaier_add(fw[5 + side * 2], fw[9 + side * 2], dt * g);
            }
            // padding nodes: the Table 1 law keeps them at zero (its faces
            // test for them); under the shape law they keep a physical state
            if (LAW == 1 && !(f & (1 << 10))) { Tnew = 0; Pnew = 0; Tlo = 0; Plo = 0; }
            Tm[q] = Tnew;   // level n-1 is no longer needed by node q
            Pm[q] = Pnew;
            if constexpr (CMP) {
                lm[q * NT + t] = Tlo;
                lm[(NPT + q) * NT + t] = Plo;
            }
            SCHED_FENCE();
        }
    };

    // buffers (a, b) hold (n-1, n); after a step a holds n+1, so the next
    // step runs with the roles exchanged
    int i = 0;
    for (; i + 1 < ksteps; i += 2) {
        step(Ta_, Pa_, Tb_, Pb_, lo_a, lo_b, n0 + i);
        step(Tb_, Pb_, Ta_, Pa_, lo_b, lo_a, n0 + i + 1);
    }
    if (i < ksteps) {
        step(Ta_, Pa_, Tb_, Pb_, lo_a, lo_b, n0 + i);
#pragma unroll
        for (int q = 0; q < NPT; ++q) {
            R x = Ta_[q]; Ta_[q] = Tb_[q]; Tb_[q] = x;
            R y = Pa_[q]; Pa_[q] = Pb_[q]; Pb_[q] = y;
        }
    }
    // now (Ta_, Pa_) = level n0+k-1 and (Tb_, Pb_) = level n0+k; FP32 stores
    // the high parts (the nearest FP32 values of the compensated levels), so
    // a launch rounds to the storage grid once, at its end

    // ---- write back: level n0+k and n0+k-1, fluxes, zone air
    const ResIO O = *io;
    const int64_t nend = n0 + ksteps;
    // pointers picked by selects, not by indexing (an indexed local array
    // would live in scratch memory)
    const bool odd = (nend & 1) != 0;
    R *Tw_cur = (R *)(odd ? O.T[1] : O.T[0]);
    R *Pw_cur = (R *)(odd ? O.P[1] : O.P[0]);
    R *Tw_prv = (R *)(odd ? O.T[0] : O.T[1]);
    R *Pw_prv = (R *)(odd ? O.P[0] : O.P[1]);
    int nonfinite = 0;
#pragma unroll
    for (int q = 0; q < NPT; ++q) {
        const int f = info[q];
        if (f & (1 << 10)) {
            const int b = t * NPT + q;
            const int s = f & 0xff;
            const int64_t g = (int64_t)wr[s].off + (b - wr[s].wstart);
            if (!(isfinite(Tb_[q]) && isfinite(Pb_[q]))) nonfinite = 1;
            Tw_cur[g] = Tb_[q];
            Pw_cur[g] = Pb_[q];
            Tw_prv[g] = Ta_[q];
            Pw_prv[g] = Pa_[q];
        }
    }
    if (nonfinite) atomicOr(O.bad, 1);
    __syncthreads();
    for (int q = t; q < nwb * 12; q += nthreads) {
        int s = q / 12, k = q % 12;
        O.flux[(int64_t)wr[s].wid * 12 + k] = wr[s].flux[k];
    }
    if (ZON && t < nrb) {
        O.roomT[rr[t].rid] = rr[t].air[nend & 1][0];
        O.roomP[rr[t].rid] = rr[t].air[nend & 1][1];
    }
}

} // namespace dfhm
