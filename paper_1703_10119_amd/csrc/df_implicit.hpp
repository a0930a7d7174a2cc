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
    int law;             // 0: shape law (from p); 1: Table 1 material (from W)
    const WallDev *W;
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
__device__ __forceinline__ ImpK imp_face(const ImpLaw &m, int la, int lb, double T, double P)
{
    if (m.law == 1) {          // Table 1 material (layer scales from the descriptor)
        const KCoef<double> k = t1_face_k<double>(*m.W, la, lb, T - 273.15, P, m.Lv);
        return {k.kT, k.kM, k.kX};
    }
    const double phi = P / psat_th(T - 273.15);
    const ImpK a = imp_law_k(m, la, phi);
    if (la == lb) return a;
    const ImpK b = imp_law_k(m, lb, phi);
    return {harm(a.kT, b.kT), harm(a.kM, b.kM), harm(a.kX, b.kX)};
}
__device__ __forceinline__ ImpC imp_node(const ImpLaw &m, int la, double T, double P)
{
    const double th = T - 273.15;
    if (m.law == 1) {
        const CCoef<double> c = t1_law_c<double>(m.W->lay[la], th, P, m.cw);
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
// One time step n -> n+1 of every wall; iters[w] accumulates the number of
// sub-iterations.
__global__ void __launch_bounds__(kImpLanes) __attribute__((amdgpu_waves_per_eu(2)))
k_imp_step(const WallDev *__restrict__ walls, const ImpGroup *__restrict__ groups, ImpArrays A,
           int64_t n, double dt, double theta, double eta, int max_it, double Lv,
           int law_id, double cw, int64_t *__restrict__ iters)
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
    const ImpLaw law{&s_law[0][lane], law_id, &W, Lv, cw};
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
    auto fwd = [&](int s) { return j0 + d * s; };        // node of forward step s (s = ns: m)
    auto bwd = [&](int s) { return m - d * (1 + s); };   // node of back step s

    // outdoor air and surface heat sources (constant + incident radiation)
    // of this lane's surface at t^n and t^{n+1}
    const double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
    const double Ti0 = sine_at(W.Tamb[side], t0);
    const double Pi0 = sine_at(W.RHamb[side], t0) * psat_th(Ti0 - 273.15);
    const double Ti1 = sine_at(W.Tamb[side], t1);
    const double Pi1 = sine_at(W.RHamb[side], t1) * psat_th(Ti1 - 273.15);
    const double Q0 = W.qinf[side] + incident(W, side, t0);
    const double Q1 = W.qinf[side] + incident(W, side, t1);

    // Each sweep keeps the data of the next kPf nodes in a register ring:
    // the loads of node (step + kPf) are issued while a node is computed, so
    // HBM latency overlaps the coefficient arithmetic.  (Ring slots are
    // indexed by the unrolled inner loop, so the ring stays in registers.)
    // Two nodes ahead and two waves per SIMD: on the 65,536-wall batches
    // that measured 10-12 % faster than eight ahead at one wave per SIMD
    // (one lane per wall), and the twisted sweeps at eight ahead needed
    // more registers than two waves leave.
    constexpr int kPf = 2;
    int it = 0;
    for (;;) {
        ++it;
        // the iterate: level n on the first pass, the last solution after
        const double *Tk = it == 1 ? To : Tw;
        const double *Pk = it == 1 ? Po : Pw;
        // ---- moisture: forward elimination with coefficients on the fly
        double xm;                                       // the meeting node's new value
        {
            double rTk[kPf], rTo[kPf], rPk[kPf], rPo[kPf];   // node of step s + 1
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                if (1 + q <= ns) {
                    const int jj = fwd(1 + q);
                    rTk[q] = Tk[at(jj)]; rTo[q] = To[at(jj)]; rPk[q] = Pk[at(jj)]; rPo[q] = Po[at(jj)];
                }
            }
            int la = layer_of(j0);
            double Tsj = theta * Tk[at(j0)] + th1 * To[at(j0)];
            double Psj = theta * Pk[at(j0)] + th1 * Po[at(j0)];
            double Poj = Po[at(j0)], Pol = 0.0;
            double gl = 0.0, rl = 0.0, el = 0.0;         // near face kM / dx; previous r, e
            for (int s0 = 0; s0 < ns; s0 += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) {
                    const int s = s0 + q;
                    if (s < ns) {
                        const int j = fwd(s);
                        const ImpC cn = imp_node(law, la, Tsj, Psj);
                        const int lb = layer_of(j + d);
                        const double Tsr = theta * rTk[q] + th1 * rTo[q];
                        const double Psr = theta * rPk[q] + th1 * rPo[q];
                        const double Por = rPo[q];
                        const double gr = imp_face(law, la, lb, 0.5 * (Tsj + Tsr), 0.5 * (Psj + Psr)).kM / dx;
                        if (s + 1 + kPf <= ns) {
                            const int jn = fwd(s + 1 + kPf);
                            rTk[q] = Tk[at(jn)]; rTo[q] = To[at(jn)]; rPk[q] = Pk[at(jn)]; rPo[q] = Po[at(jn)];
                        }
                        const bool surf = s == 0;
                        const double width = surf ? 0.5 * dx : dx;
                        double diag = width * cn.cM / dt, rhs = diag * Poj, a = 0.0;
                        if (!surf) { diag += theta * gl; a = -theta * gl; rhs += th1 * gl * (Pol - Poj); }
                        diag += theta * gr;
                        const double c = -theta * gr;
                        rhs += th1 * gr * (Por - Poj);
                        if (surf) {
                            const double h = W.hM[side];
                            diag += theta * h;
                            rhs += theta * (h * Pi1 + W.ginf[side]) + th1 * (h * (Pi0 - Poj) + W.ginf[side]);
                        }
                        const double den = diag - a * rl;
                        rl = c / den;
                        el = (rhs - a * el) / den;
                        cp[at(j)] = rl;
                        dp[at(j)] = el;
                        gl = gr; Pol = Poj; Poj = Por; Tsj = Tsr; Psj = Psr; la = lb;
                    }
                }
            }
            // the meeting node: A takes B's far face, its neighbour's level n
            // and B's last r, e (each lane's carried state is now node m)
            const double gB = __shfl_xor(gl, kImpWalls), PoB = __shfl_xor(Pol, kImpWalls);
            const double rB = __shfl_xor(rl, kImpWalls), eB = __shfl_xor(el, kImpWalls);
            {
                const ImpC cn = imp_node(law, la, Tsj, Psj);
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
            double rc[kPf], rd[kPf], rk[kPf];                 // node of back step s
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                if (q < ns) { const int jj = bwd(q); rc[q] = cp[at(jj)]; rd[q] = dp[at(jj)]; rk[q] = Pk[at(jj)]; }
            }
            double x = xm;
            for (int s0 = 0; s0 < ns; s0 += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) {
                    const int s = s0 + q;
                    if (s < ns) {
                        x = rd[q] - rc[q] * x;
                        Pn[at(bwd(s))] = x;
                        dP = fmax(dP, fabs(x - rk[q]));
                        sP = fmax(sP, fabs(x));
                        if (s + kPf < ns) {
                            const int jn = bwd(s + kPf);
                            rc[q] = cp[at(jn)]; rd[q] = dp[at(jn)]; rk[q] = Pk[at(jn)];
                        }
                    }
                }
            }
        }
        // the other lane reads the new moisture next to the meeting node
        __threadfence_block();
        // ---- heat with the new vapour pressure
        {
            double rTk[kPf], rTo[kPf], rPk[kPf], rPo[kPf], rPn[kPf];   // node of step s + 1
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                if (1 + q <= ns) {
                    const int jj = fwd(1 + q);
                    rTk[q] = Tk[at(jj)]; rTo[q] = To[at(jj)]; rPk[q] = Pk[at(jj)]; rPo[q] = Po[at(jj)];
                    rPn[q] = Pn[at(jj)];
                }
            }
            int la = layer_of(j0);
            double Tsj = theta * Tk[at(j0)] + th1 * To[at(j0)];
            double Psj = theta * Pk[at(j0)] + th1 * Po[at(j0)];
            double Toj = To[at(j0)], Poj = Po[at(j0)], Pnj = Pn[at(j0)];
            double Tol = 0.0, Pol = 0.0, Pnl = 0.0;
            double gTl = 0.0, gXl = 0.0, rl = 0.0, el = 0.0;
            for (int s0 = 0; s0 < ns; s0 += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) {
                    const int s = s0 + q;
                    if (s < ns) {
                        const int j = fwd(s);
                        const ImpC cn = imp_node(law, la, Tsj, Psj);
                        const int lb = layer_of(j + d);
                        const double Tsr = theta * rTk[q] + th1 * rTo[q];
                        const double Psr = theta * rPk[q] + th1 * rPo[q];
                        const double Tor = rTo[q], Por = rPo[q], Pnr = rPn[q];
                        const ImpK kf = imp_face(law, la, lb, 0.5 * (Tsj + Tsr), 0.5 * (Psj + Psr));
                        const double gTr = kf.kT / dx, gXr = kf.kX / dx;
                        if (s + 1 + kPf <= ns) {
                            const int jn = fwd(s + 1 + kPf);
                            rTk[q] = Tk[at(jn)]; rTo[q] = To[at(jn)]; rPk[q] = Pk[at(jn)]; rPo[q] = Po[at(jn)];
                            rPn[q] = Pn[at(jn)];
                        }
                        const bool surf = s == 0;
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
                            const double hT = W.hT[side], hL = Lv * W.hM[side];
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
                    }
                }
            }
            const double gTB = __shfl_xor(gTl, kImpWalls), gXB = __shfl_xor(gXl, kImpWalls);
            const double ToB = __shfl_xor(Tol, kImpWalls), PoB = __shfl_xor(Pol, kImpWalls);
            const double PnB = __shfl_xor(Pnl, kImpWalls);
            const double rB = __shfl_xor(rl, kImpWalls), eB = __shfl_xor(el, kImpWalls);
            {
                const ImpC cn = imp_node(law, la, Tsj, Psj);
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
            double rc[kPf], rd[kPf], rk[kPf], rn[kPf];        // node of back step s
#pragma unroll
            for (int q = 0; q < kPf; ++q) {
                if (q < ns) {
                    const int jj = bwd(q);
                    rc[q] = cp[at(jj)]; rd[q] = dp[at(jj)]; rk[q] = Tk[at(jj)]; rn[q] = Pn[at(jj)];
                }
            }
            double x = xm;
            for (int s0 = 0; s0 < ns; s0 += kPf) {
#pragma unroll
                for (int q = 0; q < kPf; ++q) {
                    const int s = s0 + q;
                    if (s < ns) {
                        x = rd[q] - rc[q] * x;
                        dT = fmax(dT, fabs(x - rk[q]));
                        sT = fmax(sT, fabs(x));
                        const double pn = rn[q];
                        // node jn is not written before it is read here: the
                        // ring reads it now, the write of node jn comes later
                        if (s + kPf < ns) {
                            const int jn = bwd(s + kPf);
                            rc[q] = cp[at(jn)]; rd[q] = dp[at(jn)]; rk[q] = Tk[at(jn)]; rn[q] = Pn[at(jn)];
                        }
                        const int j = bwd(s);
                        Tw[at(j)] = x;
                        Pw[at(j)] = pn;
                    }
                }
            }
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
