// df_implicit.hpp -- batched implicit comparator: theta-scheme in time
// (theta = 1 Euler implicit, 1/2 Crank-Nicolson) with fixed-point
// sub-iterations on the coefficients (Sec. 5.2, Algorithm 1), FP64, walls
// with the outdoor air on both sides.
//
// Each lane owns one wall and solves its two tridiagonal systems per
// sub-iteration by the Thomas algorithm: the forward elimination evaluates
// the face and node coefficients on the fly (each face once, at the
// face-averaged theta-weighted state), stores the normalised super-diagonal
// and right-hand side, and the back substitution produces the new field and
// its largest change.  Moisture is solved first; heat uses the new vapour
// pressure.  A wave's 64 walls are stored node-major (index base + 64 j +
// lane), so every load and store of a sweep is one coalesced 512-byte
// access; a wall of 1001 nodes needs 56 KB of state, so the sweeps run out of
// HBM.  Lanes whose wall has converged idle until the wave's last one has.
#pragma once
#include "dfhm_device.hpp"

namespace dfhm {

constexpr int kImpLanes = 64;

struct ImpGroup {
    int64_t base;          // first slot of the group's node-major block
    int32_t w0, nw;        // first wall, walls in the group (<= 64)
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
        const int64_t i = G.base + (int64_t)j * kImpLanes + lane;
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

// One time step n -> n+1 of every wall; iters[w] accumulates the number of
// sub-iterations.
__global__ void __launch_bounds__(kImpLanes)
k_imp_step(const WallDev *__restrict__ walls, const ImpGroup *__restrict__ groups, ImpArrays A,
           int64_t n, double dt, double theta, double eta, int max_it, double Lv,
           int law_id, double cw, int64_t *__restrict__ iters)
{
    __shared__ double s_law[kMaxLayers * L_COUNT][kImpLanes];
    const ImpGroup G = groups[blockIdx.x];
    const int lane = threadIdx.x;
    if (lane >= G.nw) return;
    const int w = G.w0 + lane;
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
    const int64_t b0 = G.base + lane;
    auto at = [&](int j) { return b0 + (int64_t)j * kImpLanes; };

    // outdoor air and surface heat sources (constant + incident radiation)
    // at t^n and t^{n+1} on both sides
    double Ti0[2], Pi0[2], Ti1[2], Pi1[2], Q0[2], Q1[2];
    for (int side = 0; side < 2; ++side) {
        const double t0 = (double)n * dt, t1 = (double)(n + 1) * dt;
        Ti0[side] = sine_at(W.Tamb[side], t0);
        Pi0[side] = sine_at(W.RHamb[side], t0) * psat_th(Ti0[side] - 273.15);
        Ti1[side] = sine_at(W.Tamb[side], t1);
        Pi1[side] = sine_at(W.RHamb[side], t1) * psat_th(Ti1[side] - 273.15);
        Q0[side] = W.qinf[side] + incident(W, side, t0);
        Q1[side] = W.qinf[side] + incident(W, side, t1);
    }

    // Each sweep keeps the data of the next kPf nodes in a register ring:
    // the loads of node j + kPf are issued while node j is computed, so HBM
    // latency overlaps the coefficient arithmetic.  (Ring slots are indexed
    // by the unrolled inner loop, so the ring stays in registers.)
    constexpr int kPf = 8;
    int it = 0;
    for (;;) {
        ++it;
        // the iterate: level n on the first pass, the last solution after
        const double *Tk = it == 1 ? To : Tw;
        const double *Pk = it == 1 ? Po : Pw;
        // ---- moisture: forward elimination with coefficients on the fly
        {
            double rTk[kPf], rTo[kPf], rPk[kPf], rPo[kPf];   // node j + 1 + d
#pragma unroll
            for (int d = 0; d < kPf; ++d) {
                const int jj = 1 + d;
                if (jj < nx) { rTk[d] = Tk[at(jj)]; rTo[d] = To[at(jj)]; rPk[d] = Pk[at(jj)]; rPo[d] = Po[at(jj)]; }
            }
            int la = layer_of(0);
            double Tsj = theta * Tk[at(0)] + th1 * To[at(0)];
            double Psj = theta * Pk[at(0)] + th1 * Po[at(0)];
            double Poj = Po[at(0)], Pol = 0.0;
            double gl = 0.0, cpl = 0.0, dpl = 0.0;         // left face kM / dx; previous cp, dp
            for (int j0 = 0; j0 < nx; j0 += kPf) {
#pragma unroll
                for (int d = 0; d < kPf; ++d) {
                    const int j = j0 + d;
                    if (j < nx) {
                        const ImpC cn = imp_node(law, la, Tsj, Psj);
                        double gr = 0.0, Por = 0.0, Tsr = 0.0, Psr = 0.0;
                        int lb = la;
                        if (j < nx - 1) {
                            lb = layer_of(j + 1);
                            Tsr = theta * rTk[d] + th1 * rTo[d];
                            Psr = theta * rPk[d] + th1 * rPo[d];
                            Por = rPo[d];
                            gr = imp_face(law, la, lb, 0.5 * (Tsj + Tsr), 0.5 * (Psj + Psr)).kM / dx;
                        }
                        const int jn = j + 1 + kPf;
                        if (jn < nx) { rTk[d] = Tk[at(jn)]; rTo[d] = To[at(jn)]; rPk[d] = Pk[at(jn)]; rPo[d] = Po[at(jn)]; }
                        const bool surf = j == 0 || j == nx - 1;
                        const double width = surf ? 0.5 * dx : dx;
                        double diag = width * cn.cM / dt, rhs = diag * Poj, a = 0.0, c = 0.0;
                        if (j > 0) { diag += theta * gl; a = -theta * gl; rhs += th1 * gl * (Pol - Poj); }
                        if (j < nx - 1) { diag += theta * gr; c = -theta * gr; rhs += th1 * gr * (Por - Poj); }
                        if (surf) {
                            const int side = j == 0 ? 0 : 1;
                            const double h = W.hM[side];
                            diag += theta * h;
                            rhs += theta * (h * Pi1[side] + W.ginf[side])
                                 + th1 * (h * (Pi0[side] - Poj) + W.ginf[side]);
                        }
                        const double den = diag - a * cpl;
                        cpl = c / den;
                        dpl = (rhs - a * dpl) / den;
                        cp[at(j)] = cpl;
                        dp[at(j)] = dpl;
                        gl = gr; Pol = Poj; Poj = Por; Tsj = Tsr; Psj = Psr; la = lb;
                    }
                }
            }
        }
        // back substitution -> Pn, largest change and scale
        double dP = 0.0, sP = 0.0;
        {
            double rc[kPf], rd[kPf], rk[kPf];                 // node j - d
#pragma unroll
            for (int d = 0; d < kPf; ++d) {
                const int jj = nx - 1 - d;
                if (jj >= 0) { rc[d] = cp[at(jj)]; rd[d] = dp[at(jj)]; rk[d] = Pk[at(jj)]; }
            }
            double x = 0.0;
            for (int j0 = nx - 1; j0 >= 0; j0 -= kPf) {
#pragma unroll
                for (int d = 0; d < kPf; ++d) {
                    const int j = j0 - d;
                    if (j >= 0) {
                        x = rd[d] - (j < nx - 1 ? rc[d] * x : 0.0);
                        Pn[at(j)] = x;
                        dP = fmax(dP, fabs(x - rk[d]));
                        sP = fmax(sP, fabs(x));
                        const int jn = j - kPf;
                        if (jn >= 0) { rc[d] = cp[at(jn)]; rd[d] = dp[at(jn)]; rk[d] = Pk[at(jn)]; }
                    }
                }
            }
        }
        // ---- heat with the new vapour pressure
        {
            double rTk[kPf], rTo[kPf], rPk[kPf], rPo[kPf], rPn[kPf];   // node j + 1 + d
#pragma unroll
            for (int d = 0; d < kPf; ++d) {
                const int jj = 1 + d;
                if (jj < nx) {
                    rTk[d] = Tk[at(jj)]; rTo[d] = To[at(jj)]; rPk[d] = Pk[at(jj)]; rPo[d] = Po[at(jj)];
                    rPn[d] = Pn[at(jj)];
                }
            }
            int la = layer_of(0);
            double Tsj = theta * Tk[at(0)] + th1 * To[at(0)];
            double Psj = theta * Pk[at(0)] + th1 * Po[at(0)];
            double Toj = To[at(0)], Poj = Po[at(0)], Pnj = Pn[at(0)];
            double Tol = 0.0, Pol = 0.0, Pnl = 0.0;
            double gTl = 0.0, gXl = 0.0, cpl = 0.0, dpl = 0.0;
            for (int j0 = 0; j0 < nx; j0 += kPf) {
#pragma unroll
                for (int d = 0; d < kPf; ++d) {
                    const int j = j0 + d;
                    if (j < nx) {
                        const ImpC cn = imp_node(law, la, Tsj, Psj);
                        double gTr = 0.0, gXr = 0.0, Tor = 0.0, Por = 0.0, Pnr = 0.0, Tsr = 0.0, Psr = 0.0;
                        int lb = la;
                        if (j < nx - 1) {
                            lb = layer_of(j + 1);
                            Tsr = theta * rTk[d] + th1 * rTo[d];
                            Psr = theta * rPk[d] + th1 * rPo[d];
                            Tor = rTo[d];
                            Por = rPo[d];
                            Pnr = rPn[d];
                            const ImpK kf = imp_face(law, la, lb, 0.5 * (Tsj + Tsr), 0.5 * (Psj + Psr));
                            gTr = kf.kT / dx;
                            gXr = kf.kX / dx;
                        }
                        const int jn = j + 1 + kPf;
                        if (jn < nx) {
                            rTk[d] = Tk[at(jn)]; rTo[d] = To[at(jn)]; rPk[d] = Pk[at(jn)]; rPo[d] = Po[at(jn)];
                            rPn[d] = Pn[at(jn)];
                        }
                        const bool surf = j == 0 || j == nx - 1;
                        const double width = surf ? 0.5 * dx : dx;
                        double diag = width * cn.cT / dt;
                        double rhs = diag * Toj - width * cn.cX * (Pnj - Poj) / dt;
                        double a = 0.0, c = 0.0;
                        if (j > 0) {
                            diag += theta * gTl; a = -theta * gTl;
                            rhs += th1 * gTl * (Tol - Toj) + gXl * (theta * (Pnl - Pnj) + th1 * (Pol - Poj));
                        }
                        if (j < nx - 1) {
                            diag += theta * gTr; c = -theta * gTr;
                            rhs += th1 * gTr * (Tor - Toj) + gXr * (theta * (Pnr - Pnj) + th1 * (Por - Poj));
                        }
                        if (surf) {
                            const int side = j == 0 ? 0 : 1;
                            const double hT = W.hT[side], hL = Lv * W.hM[side];
                            diag += theta * hT;
                            rhs += theta * (hT * Ti1[side] + hL * (Pi1[side] - Pnj) + Q1[side])
                                 + th1 * (hT * (Ti0[side] - Toj) + hL * (Pi0[side] - Poj) + Q0[side]);
                        }
                        const double den = diag - a * cpl;
                        cpl = c / den;
                        dpl = (rhs - a * dpl) / den;
                        cp[at(j)] = cpl;
                        dp[at(j)] = dpl;
                        gTl = gTr; gXl = gXr; Tol = Toj; Pol = Poj; Pnl = Pnj;
                        Toj = Tor; Poj = Por; Pnj = Pnr; Tsj = Tsr; Psj = Psr; la = lb;
                    }
                }
            }
        }
        // back substitution -> the new iterate (T, and Pn copied into P)
        double dT = 0.0, sT = 0.0;
        {
            double rc[kPf], rd[kPf], rk[kPf], rn[kPf];        // node j - d
#pragma unroll
            for (int d = 0; d < kPf; ++d) {
                const int jj = nx - 1 - d;
                if (jj >= 0) { rc[d] = cp[at(jj)]; rd[d] = dp[at(jj)]; rk[d] = Tk[at(jj)]; rn[d] = Pn[at(jj)]; }
            }
            double x = 0.0;
            for (int j0 = nx - 1; j0 >= 0; j0 -= kPf) {
#pragma unroll
                for (int d = 0; d < kPf; ++d) {
                    const int j = j0 - d;
                    if (j >= 0) {
                        x = rd[d] - (j < nx - 1 ? rc[d] * x : 0.0);
                        dT = fmax(dT, fabs(x - rk[d]));
                        sT = fmax(sT, fabs(x));
                        const double pn = rn[d];
                        const int jn = j - kPf;
                        // node jn is not written before it is read here: the
                        // ring reads it now, the write of node jn comes later
                        if (jn >= 0) { rc[d] = cp[at(jn)]; rd[d] = dp[at(jn)]; rk[d] = Tk[at(jn)]; rn[d] = Pn[at(jn)]; }
                        Tw[at(j)] = x;
                        Pw[at(j)] = pn;
                    }
                }
            }
        }
        if ((dT <= eta * sT && dP <= eta * sP) || it >= max_it) break;
    }
    iters[w] += it;
}

} // namespace dfhm
