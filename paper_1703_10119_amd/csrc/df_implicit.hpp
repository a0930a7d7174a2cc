// df_implicit.hpp -- batched implicit comparator: theta-scheme in time
// (theta = 1 Euler implicit, 1/2 Crank-Nicolson) with fixed-point
// sub-iterations on the coefficients (Sec. 5.2, Algorithm 1), FP64, walls
// with the outdoor air on both sides.
//
// Two lanes own one wall and solve its two tridiagonal systems per
// sub-iteration by a twisted Thomas elimination (from both surfaces towards
// the middle node, see k_imp_step): the forward eliminations evaluate the
// face and node coefficients on the fly (each face once, at the
// face-averaged theta-weighted state), store the normalised off-diagonal and
// right-hand side, and the back substitutions produce the new field and its
// largest change.  Moisture is solved first; heat uses the new vapour
// pressure.  A wave's 32 walls are stored node-major (index base + 32 j +
// wall), so every load and store of a sweep is two coalesced 256-byte
// accesses (one per half); a wall of 1001 nodes needs 56 KB of state, so the
// sweeps run out of HBM.  Walls whose fixed point has converged idle until
// the wave's last one has.
#pragma once
#include "dfhm_device.hpp"

namespace dfhm {

constexpr int kImpLanes = 64;
constexpr int kImpWalls = 32;   // walls per wave: two lanes per wall

struct ImpGroup {
    int64_t base;          // first slot of the group's node-major block
    int32_t w0, nw;        // first wall, walls in the group (<= 32)
};

struct ImpArrays {
    double *T[2], *P[2];   // levels by step parity
    double *Pn, *cp, *dp;  // new moisture iterate, Thomas workspace
};

__global__ void k_imp_init(const WallDev *__restrict__ walls, const ImpGroup *__restrict__ groups,
                           ImpArrays A)
{
    const ImpGroup G = groups[blockIdx.x];
    const int lane = threadIdx.x;
    if (lane >= G.nw) return;
    const WallDev &W = walls[G.w0 + lane];
    for (int j = 0; j < W.nx; ++j) {
        const int64_t i = G.base + (int64_t)j * kImpWalls + lane;
        A.T[0][i] = W.T0;
        A.P[0][i] = W.P0;
    }
}

// The law constants of a lane's wall live in LDS, parameter-major
// ([layer * L_COUNT + k][lane], consecutive lanes in consecutive banks), so
// the coefficient evaluations inside the sweeps read no global memory.
struct ImpLaw {
    const double *p;     // &s_law[0][lane]
    double Lv, cw;
    __device__ __forceinline__ double operator()(int la, int k) const
    {
        return p[(la * L_COUNT + k) * kImpLanes];
    }
};

// Coefficients of the law at a (T, P) state (T in K), as law_k / law_c.
struct ImpK { double kT, kM, kX; };
struct ImpC { double cT, cM, cX; };

__device__ __forceinline__ ImpK imp_law_k(const ImpLaw &m, int la, double phi)
{
    ImpK k;
    k.kT = m(la, L_K0) * (1.0 + m(la, L_AT) * phi);
    k.kM = m(la, L_KM0) * (1.0 + m(la, L_AM) * phi * phi);
    k.kX = m(la, L_BTM) * k.kM;
    return k;
}
// LAW: 0 = the shape law, 1 = the Table 1 material (the layer scales of the
// wall times that material's functions, evaluated once per face)
template <int LAW>
__device__ __forceinline__ ImpK imp_face(const ImpLaw &m, int la, int lb, double T, double P)
{
    if constexpr (LAW == 1) {
        const KCoef<double> f = t1_kfun<double>(T - 273.15, P, m.Lv);
        const ImpK a = {f.kT * m(la, L_K0), f.kM * m(la, L_KM0), f.kX * m(la, L_KM0)};
        if (la == lb) return a;
        const ImpK b = {f.kT * m(lb, L_K0), f.kM * m(lb, L_KM0), f.kX * m(lb, L_KM0)};
        return {harm(a.kT, b.kT), harm(a.kM, b.kM), harm(a.kX, b.kX)};
    }
    const double phi = P / psat_th(T - 273.15);
    const ImpK a = imp_law_k(m, la, phi);
    if (la == lb) return a;
    const ImpK b = imp_law_k(m, lb, phi);
    return {harm(a.kT, b.kT), harm(a.kM, b.kM), harm(a.kX, b.kX)};
}
template <int LAW>
__device__ __forceinline__ ImpC imp_node(const ImpLaw &m, int la, double T, double P)
{
    const double th = T - 273.15;
    if constexpr (LAW == 1) {
        double ml[L_COUNT];
        ml[L_C0] = m(la, L_C0);
        ml[L_CM0] = m(la, L_CM0);
        const CCoef<double> c = t1_law_c<double>(ml, th, P, m.cw);
        return {c.cT, c.cM, c.cX};
    }
    const double phi = P / psat_th(th);
    ImpC c;
    c.cT = m(la, L_C0) * (1.0 + m(la, L_CT) * phi);
    c.cM = m(la, L_CM0) * (1.0 + m(la, L_AC) * phi);
    c.cX = (m(la, L_ETM) + m(la, L_FTM) * th) * c.cM;
    return c;
}

// Two lanes per wall, twisted elimination: lane A (lanes 0-31) eliminates
// from the side-0 surface node 0 towards the meeting node m = (nx - 1) / 2,
// lane B (lanes 32-63, the same wall) from the side-1 surface node nx - 1
// towards it, both at once; A solves node m from the two one-sided
// recurrences and passes x_m to B, and each lane back-substitutes its half.
// A lane sweeps in its own direction d (A: +1, B: -1): for its node j the
// "near" face is the one it came through and the "far" face, to node j + d,
// is evaluated there, so every face is still evaluated once per sweep.  The
// elimination is the same for both lanes once the off-diagonal coefficients
// are named near and far: den = diag - near * r_prev, r = far / den,
// e = (rhs - near * e_prev) / den, and the back substitution is
// x_j = e_j - r_j x_(j+d).
// (One lane per wall left 64 walls per wave and one wave per SIMD on the
// 65,536-wall batches: the sweeps' dependent FP64 chains then had nothing to
// hide their latency behind.)
//
// Each sweep keeps the next kPf nodes' data in a register ring: step s reads
// slot s % kPf and refills it with the node of step s + kPf (the index
// clamped to the half, so that every read is issued).  The loop runs in
// blocks of kPf steps with the slot a compile-time index and no branch, so
// the wait for a node's data covers only the reads issued kPf steps before;
// the surface node (step 0) is peeled off and the last partial block is
// guarded.
//
// One time step n -> n+1 of every wall; iters[w] accumulates the number of
// sub-iterations.
template <int LAW>
__global__ void __launch_bounds__(kImpLanes) __attribute__((amdgpu_waves_per_eu(2)))
k_imp_step(const WallDev *__restrict__ walls, const ImpGroup *__restrict__ groups, ImpArrays A,
           int64_t n, double dt, double theta, double eta, int max_it, double Lv,
           double cw, int64_t *__restrict__ iters)
{
    __shared__ double s_law[kMaxLayers * L_COUNT][kImpLanes];
    const ImpGroup G = groups[blockIdx.x];
    const int lane = threadIdx.x;
    const int wl = lane & (kImpWalls - 1);
    const bool up = lane >= kImpWalls;      // lane B
    if (wl >= G.nw) return;                 // both lanes of an absent wall
    const int w = G.w0 + wl;
    const WallDev &W = walls[w];
    const int nx = W.nx;
    for (int q = 0; q < kMaxLayers * L_COUNT; ++q) s_law[q][lane] = W.lay[q / L_COUNT][q % L_COUNT];
    const ImpLaw law{&s_law[0][lane], Lv, cw};
    // first node of layers 1 and 2 (node j is in the first layer whose right
    // end is >= x_j), so that a node's layer is two compares
    int jb1 = nx, jb2 = nx;
    {
        double acc = 0.0;
        for (int l = 0; l < W.n_layers - 1; ++l) {
            acc += W.lay[l][L_THICK];
            int j = (int)(acc / W.dx);
            while (j > 0 && (double)(j - 1) * W.dx > acc) --j;
            while (j < nx && !((double)j * W.dx > acc)) ++j;
            if (l == 0) jb1 = j; else jb2 = j;
        }
    }
    auto layer_of = [&](int j) { return (j >= jb1) + (j >= jb2); };
    const double dx = W.dx;
    const double th1 = 1.0 - theta;
    const int p = (int)(n & 1);
    // The workspace (Pn, cp, dp) and level n never alias anything else, so
    // the loads of the next nodes of a sweep may be issued ahead of this
    // node's workspace stores.  The new level (Tw, Pw) is also the iterate
    // after the first sub-iteration and stays unqualified.
    const double *__restrict__ To = A.T[p];
    const double *__restrict__ Po = A.P[p];
    double *Tw = A.T[p ^ 1];
    double *Pw = A.P[p ^ 1];
    double *__restrict__ Pn = A.Pn;
    double *__restrict__ cp = A.cp;
    double *__restrict__ dp = A.dp;
    const int64_t b0 = G.base + wl;
    auto at = [&](int j) { return b0 + (int64_t)j * kImpWalls; };

    // this lane's half: ns nodes from its surface node j0 in direction d,
    // ending next to the meeting node m
    const int m = (nx - 1) / 2;
    const int d = up ? -1 : 1;
    const int j0 = up ? nx - 1 : 0;
    const int ns = up ? nx - 1 - m : m;
    const int side = up ? 1 : 0;
    auto fwd = [&](int s) { return j0 + d * min(s, ns); };          // node of forward step s (ns: m)
    auto bwd = [&](int s) { return m - d * (1 + min(s, ns - 1)); }; // node of back step s

    // outdoor air and surface heat sources (constant + incident radiation)
    // of this lane's surface at t^n and t^{n+1}, and its exchange coefficients
    const double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
    const double Ti0 = sine_at(W.Tamb[side], t0);
    const double Pi0 = sine_at(W.RHamb[side], t0) * psat_th(Ti0 - 273.15);
    const double Ti1 = sine_at(W.Tamb[side], t1);
    const double Pi1 = sine_at(W.RHamb[side], t1) * psat_th(Ti1 - 273.15);
    const double Q0 = W.qinf[side] + incident(W, side, t0);
    const double Q1 = W.qinf[side] + incident(W, side, t1);
    const double hM = W.hM[side], gI = W.ginf[side], hT = W.hT[side], hL = Lv * W.hM[side];

    // (three slots: 15.0 ms per step on the 65,536 x 1001 batch against 19.5
    // with a shifting queue, whose register moves waited for reads in flight)
    constexpr int kPf = 3;
    int it = 0;
    for (;;) {
        ++it;
        // the iterate: level n on the first pass, the last solution after
        const double *Tk = it == 1 ? To : Tw;
        const double *Pk = it == 1 ? Po : Pw;
        double xm;                                       // the meeting node's new value
        // ---- moisture: forward elimination with coefficients on the fly
        {
            double qTk[kPf], qTo[kPf], qPk[kPf], qPo[kPf];   // nodes of steps s + 1 .. s + kPf
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                const int jj = fwd(1 + q);
                qTk[q] = Tk[at(jj)]; qTo[q] = To[at(jj)]; qPk[q] = Pk[at(jj)]; qPo[q] = Po[at(jj)];
            }
            int la = layer_of(j0);
            double Tsj = theta * Tk[at(j0)] + th1 * To[at(j0)];
            double Psj = theta * Pk[at(j0)] + th1 * Po[at(j0)];
            double Poj = Po[at(j0)], Pol = 0.0;
            double gl = 0.0, rl = 0.0, el = 0.0;         // near face kM / dx; previous r, e
            // step s reads its far node from slot s % kPf and refills the slot
            // with the far node of step s + kPf
            auto step = [&](const bool surf, int s, double &fTk, double &fTo, double &fPk, double &fPo) {
                const int j = fwd(s);
                const ImpC cn = imp_node<LAW>(law, la, Tsj, Psj);
                const int lb = layer_of(j + d);
                const double Tsr = theta * fTk + th1 * fTo;
                const double Psr = theta * fPk + th1 * fPo;
                const double Por = fPo;
                const double gr = imp_face<LAW>(law, la, lb, 0.5 * (Tsj + Tsr), 0.5 * (Psj + Psr)).kM / dx;
                {
                    const int jn = fwd(s + 1 + kPf);
                    fTk = Tk[at(jn)]; fTo = To[at(jn)]; fPk = Pk[at(jn)]; fPo = Po[at(jn)];
                }
                const double width = surf ? 0.5 * dx : dx;
                double diag = width * cn.cM / dt, rhs = diag * Poj, a = 0.0;
                if (!surf) { diag += theta * gl; a = -theta * gl; rhs += th1 * gl * (Pol - Poj); }
                diag += theta * gr;
                const double c = -theta * gr;
                rhs += th1 * gr * (Por - Poj);
                if (surf) {
                    diag += theta * hM;
                    rhs += theta * (hM * Pi1 + gI) + th1 * (hM * (Pi0 - Poj) + gI);
                }
                const double den = diag - a * rl;
                rl = c / den;
                el = (rhs - a * el) / den;
                cp[at(j)] = rl;
                dp[at(j)] = el;
                gl = gr; Pol = Poj; Poj = Por; Tsj = Tsr; Psj = Psr; la = lb;
            };
            step(true, 0, qTk[0], qTo[0], qPk[0], qPo[0]);
            int s = 1;
            for (; s + kPf <= ns; s += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) {
                    const int k = (1 + q) % kPf;
                    step(false, s + q, qTk[k], qTo[k], qPk[k], qPo[k]);
                }
            }
#pragma unroll
            for (int q = 0; q + 1 < kPf; ++q) {
                const int k = (1 + q) % kPf;
                if (s + q < ns) step(false, s + q, qTk[k], qTo[k], qPk[k], qPo[k]);
            }
            // the meeting node: A takes B's far face, its neighbour's level n
            // and B's last r, e (each lane's carried state is now node m)
            const double gB = __shfl_xor(gl, kImpWalls), PoB = __shfl_xor(Pol, kImpWalls);
            const double rB = __shfl_xor(rl, kImpWalls), eB = __shfl_xor(el, kImpWalls);
            {
                const ImpC cn = imp_node<LAW>(law, la, Tsj, Psj);
                const double diag0 = dx * cn.cM / dt;
                const double diag = diag0 + theta * (gl + gB);
                const double rhs = diag0 * Poj + th1 * gl * (Pol - Poj) + th1 * gB * (PoB - Poj);
                const double aA = -theta * gl, aB = -theta * gB;
                const double x = (rhs - aA * el - aB * eB) / (diag - aA * rl - aB * rB);
                xm = __shfl_xor(x, kImpWalls);
                if (!up) xm = x;
            }
        }
        // back substitution -> Pn, largest change and scale
        double dP = 0.0, sP = 0.0;
        {
            if (!up) {
                Pn[at(m)] = xm;
                dP = fabs(xm - Pk[at(m)]);
                sP = fabs(xm);
            }
            double qc[kPf], qd[kPf], qk[kPf];                 // nodes of back steps s .. s + kPf - 1
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                const int jj = bwd(q);
                qc[q] = cp[at(jj)]; qd[q] = dp[at(jj)]; qk[q] = Pk[at(jj)];
            }
            double x = xm;
            auto bstep = [&](int s, double &fc, double &fd, double &fk) {
                x = fd - fc * x;
                const double pk = fk;
                {
                    const int jn = bwd(s + kPf);
                    fc = cp[at(jn)]; fd = dp[at(jn)]; fk = Pk[at(jn)];
                }
                Pn[at(bwd(s))] = x;
                dP = fmax(dP, fabs(x - pk));
                sP = fmax(sP, fabs(x));
            };
            int s = 0;
            for (; s + kPf <= ns; s += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) bstep(s + q, qc[q], qd[q], qk[q]);
            }
#pragma unroll
            for (int q = 0; q + 1 < kPf; ++q)
                if (s + q < ns) bstep(s + q, qc[q], qd[q], qk[q]);
        }
        // the other lane reads the new moisture next to the meeting node
        __threadfence_block();
        // ---- heat with the new vapour pressure
        {
            double qTk[kPf], qTo[kPf], qPk[kPf], qPo[kPf], qPn[kPf];   // nodes of steps s + 1 ..
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                const int jj = fwd(1 + q);
                qTk[q] = Tk[at(jj)]; qTo[q] = To[at(jj)]; qPk[q] = Pk[at(jj)]; qPo[q] = Po[at(jj)];
                qPn[q] = Pn[at(jj)];
            }
            int la = layer_of(j0);
            double Tsj = theta * Tk[at(j0)] + th1 * To[at(j0)];
            double Psj = theta * Pk[at(j0)] + th1 * Po[at(j0)];
            double Toj = To[at(j0)], Poj = Po[at(j0)], Pnj = Pn[at(j0)];
            double Tol = 0.0, Pol = 0.0, Pnl = 0.0;
            double gTl = 0.0, gXl = 0.0, rl = 0.0, el = 0.0;
            auto step = [&](const bool surf, int s, double &fTk, double &fTo, double &fPk, double &fPo,
                            double &fPn) {
                const int j = fwd(s);
                const ImpC cn = imp_node<LAW>(law, la, Tsj, Psj);
                const int lb = layer_of(j + d);
                const double Tsr = theta * fTk + th1 * fTo;
                const double Psr = theta * fPk + th1 * fPo;
                const double Tor = fTo, Por = fPo, Pnr = fPn;
                const ImpK kf = imp_face<LAW>(law, la, lb, 0.5 * (Tsj + Tsr), 0.5 * (Psj + Psr));
                const double gTr = kf.kT / dx, gXr = kf.kX / dx;
                {
                    const int jn = fwd(s + 1 + kPf);
                    fTk = Tk[at(jn)]; fTo = To[at(jn)]; fPk = Pk[at(jn)]; fPo = Po[at(jn)];
                    fPn = Pn[at(jn)];
                }
                const double width = surf ? 0.5 * dx : dx;
                double diag = width * cn.cT / dt;
                double rhs = diag * Toj - width * cn.cX * (Pnj - Poj) / dt;
                double a = 0.0;
                if (!surf) {
                    diag += theta * gTl; a = -theta * gTl;
                    rhs += th1 * gTl * (Tol - Toj) + gXl * (theta * (Pnl - Pnj) + th1 * (Pol - Poj));
                }
                diag += theta * gTr;
                const double c = -theta * gTr;
                rhs += th1 * gTr * (Tor - Toj) + gXr * (theta * (Pnr - Pnj) + th1 * (Por - Poj));
                if (surf) {
                    diag += theta * hT;
                    rhs += theta * (hT * Ti1 + hL * (Pi1 - Pnj) + Q1)
                         + th1 * (hT * (Ti0 - Toj) + hL * (Pi0 - Poj) + Q0);
                }
                const double den = diag - a * rl;
                rl = c / den;
                el = (rhs - a * el) / den;
                cp[at(j)] = rl;
                dp[at(j)] = el;
                gTl = gTr; gXl = gXr; Tol = Toj; Pol = Poj; Pnl = Pnj;
                Toj = Tor; Poj = Por; Pnj = Pnr; Tsj = Tsr; Psj = Psr; la = lb;
            };
            step(true, 0, qTk[0], qTo[0], qPk[0], qPo[0], qPn[0]);
            int s = 1;
            for (; s + kPf <= ns; s += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) {
                    const int k = (1 + q) % kPf;
                    step(false, s + q, qTk[k], qTo[k], qPk[k], qPo[k], qPn[k]);
                }
            }
#pragma unroll
            for (int q = 0; q + 1 < kPf; ++q) {
                const int k = (1 + q) % kPf;
                if (s + q < ns) step(false, s + q, qTk[k], qTo[k], qPk[k], qPo[k], qPn[k]);
            }
            const double gTB = __shfl_xor(gTl, kImpWalls), gXB = __shfl_xor(gXl, kImpWalls);
            const double ToB = __shfl_xor(Tol, kImpWalls), PoB = __shfl_xor(Pol, kImpWalls);
            const double PnB = __shfl_xor(Pnl, kImpWalls);
            const double rB = __shfl_xor(rl, kImpWalls), eB = __shfl_xor(el, kImpWalls);
            {
                const ImpC cn = imp_node<LAW>(law, la, Tsj, Psj);
                const double diag0 = dx * cn.cT / dt;
                const double diag = diag0 + theta * (gTl + gTB);
                const double rhs = diag0 * Toj - dx * cn.cX * (Pnj - Poj) / dt
                                 + th1 * gTl * (Tol - Toj) + gXl * (theta * (Pnl - Pnj) + th1 * (Pol - Poj))
                                 + th1 * gTB * (ToB - Toj) + gXB * (theta * (PnB - Pnj) + th1 * (PoB - Poj));
                const double aA = -theta * gTl, aB = -theta * gTB;
                const double x = (rhs - aA * el - aB * eB) / (diag - aA * rl - aB * rB);
                xm = __shfl_xor(x, kImpWalls);
                if (!up) xm = x;
            }
        }
        // back substitution -> the new iterate (T, and Pn copied into P)
        double dT = 0.0, sT = 0.0;
        {
            if (!up) {
                dT = fabs(xm - Tk[at(m)]);
                sT = fabs(xm);
                const double pn = Pn[at(m)];
                Tw[at(m)] = xm;
                Pw[at(m)] = pn;
            }
            double qc[kPf], qd[kPf], qk[kPf], qn[kPf];        // nodes of back steps s ..
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                const int jj = bwd(q);
                qc[q] = cp[at(jj)]; qd[q] = dp[at(jj)]; qk[q] = Tk[at(jj)]; qn[q] = Pn[at(jj)];
            }
            double x = xm;
            // node s + kPf is read before this step's write of node s (a node
            // is written only at its own step, after every read of it)
            auto bstep = [&](int s, double &fc, double &fd, double &fk, double &fn) {
                x = fd - fc * x;
                const double tk = fk, pn = fn;
                {
                    const int jn = bwd(s + kPf);
                    fc = cp[at(jn)]; fd = dp[at(jn)]; fk = Tk[at(jn)]; fn = Pn[at(jn)];
                }
                const int j = bwd(s);
                dT = fmax(dT, fabs(x - tk));
                sT = fmax(sT, fabs(x));
                Tw[at(j)] = x;
                Pw[at(j)] = pn;
            };
            int s = 0;
            for (; s + kPf <= ns; s += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) bstep(s + q, qc[q], qd[q], qk[q], qn[q]);
            }
#pragma unroll
            for (int q = 0; q + 1 < kPf; ++q)
                if (s + q < ns) bstep(s + q, qc[q], qd[q], qk[q], qn[q]);
        }
        // the next sub-iteration's sweeps read the other lane's new nodes
        __threadfence_block();
        // both lanes of a wall take the same decision
        dT = fmax(dT, __shfl_xor(dT, kImpWalls));
        sT = fmax(sT, __shfl_xor(sT, kImpWalls));
        dP = fmax(dP, __shfl_xor(dP, kImpWalls));
        sP = fmax(sP, __shfl_xor(sP, kImpWalls));
        if ((dT <= eta * sT && dP <= eta * sP) || it >= max_it) break;
    }
    if (!up) iters[w] += it;
}

} // namespace dfhm
