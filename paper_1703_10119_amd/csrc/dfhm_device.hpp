// dfhm_device.hpp -- device-side data layout and material law of the
// Dufort-Frankel wall / room kernels (gfx950).
//
// Layout in HBM (one context):
//   walls   WallDev[W]           descriptor per wall (read with scalar loads)
//   T, P    level buffers [2][N] of the storage type, walls concatenated;
//           level n lives in buffer n & 1, level n-1 in the other one and
//           level n+1 overwrites n-1 in place.  FP64 stores absolute K / Pa,
//           FP32 stores deviations from the wall's initial (T0, Pv0).
//   lay     uint8 [N]            layer of each node
//   flux    double [W][12]       now[4], Neumaier sum[4], compensation[4]
//                                (index side * 2 + field, field 0 = heat)
//   rooms   RoomDev[R] + schedules + room air (FP64)
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dfhm {

constexpr int kMaxLayers = 3;
constexpr int kMaxNx = 2048;

// law parameter slots of a layer (thickness first)
enum LawSlot {
    L_THICK = 0, L_K0, L_AT, L_KM0, L_AM, L_BTM, L_C0, L_CT, L_CM0, L_AC, L_ETM, L_FTM,
    L_COUNT
};

struct WallDev {
    int32_t off, nx, n_layers, room;   // room = -1 when no zone is coupled
    int32_t room_side, pad0, pad1, pad2;
    double dx, r, s, area;             // r = dt/dx^2, s = dt/dx (set on device)
    double T0, RH0, P0, th0;           // initial state; P0, th0 set on device
    double hT[2], hM[2], qinf[2], ginf[2];
    double Tamb[2][4], RHamb[2][4];    // mean, amp, period, phase
    double lay[kMaxLayers][L_COUNT];
    double qsun[2][4];                 // incident radiation sinusoid (clipped at 0)
    double emis[2];                    // surface emissivities
    double esig;                       // s eps sigma of the zone side (0: no exchange)
    int32_t room_walls;                // walls of the coupled zone (0: none)
    int32_t pad3;
};

struct RoomDev {
    double volume, ach, T0, RH0;
    double Tout[4], RHout[4];
    double sched_dt;
    int32_t n_sched, sched_off;        // offset into the schedule arrays
    int32_t w_begin, w_end;            // range in the room -> wall index list
    double view;                       // view factor between two surfaces
    int32_t l_begin, l_end;            // range in the zone-link table
};

// One direction of an inter-zone link, listed under the receiving zone.
struct ZoneLinkDev {
    int32_t partner, pad;
    double g;                          // kg/s of dry air each way
};

// Stefan-Boltzmann constant, W/(m2 K4).
constexpr double kSigma = 5.670374419e-8;

// Global constants of a run (kernel argument).
struct RunConst {
    double dt, Lv, cw, rho_a, c_pa, c_pv, Pv_ref;
};

__device__ __forceinline__ double dpi() { return 3.14159265358979323846; }

// Magnus saturation pressure from theta = T - 273.15 (degC).
__device__ __forceinline__ double psat_th(double th)
{
    return 610.94 * exp(17.625 * th / (th + 243.04));
}
__device__ __forceinline__ float psat_th(float th)
{
    return 610.94f * __expf(17.625f * th / (th + 243.04f));
}

__device__ __forceinline__ double sine_at(const double *s, double t)
{
    return s[0] + s[1] * sin(2.0 * dpi() * t / s[2] + s[3]);
}

// Incident radiation of one side at time t (W/m2): the sinusoid clipped at 0.
__device__ __forceinline__ double incident(const WallDev &W, int side, double t)
{
    if (!(W.qsun[side][0] + fabs(W.qsun[side][1]) > 0.0)) return 0.0;   // never positive
    const double q = sine_at(W.qsun[side], t);
    return q > 0.0 ? q : 0.0;
}

// Fourth power of an absolute temperature (K).
__device__ __forceinline__ double pow4(double T)
{
    const double T2 = T * T;
    return T2 * T2;
}

template <typename R> struct KCoef { R kT, kM, kX; };
template <typename R> struct CCoef { R cT, cM, cX; };

template <typename R>
__device__ __forceinline__ KCoef<R> law_k(const double *m, R phi)
{
    KCoef<R> k;
    k.kT = (R)m[L_K0] * ((R)1 + (R)m[L_AT] * phi);
    k.kM = (R)m[L_KM0] * ((R)1 + (R)m[L_AM] * phi * phi);
    k.kX = (R)m[L_BTM] * k.kM;
    return k;
}

template <typename R>
__device__ __forceinline__ CCoef<R> law_c(const double *m, R phi, R th)
{
    CCoef<R> c;
    c.cT = (R)m[L_C0] * ((R)1 + (R)m[L_CT] * phi);
    c.cM = (R)m[L_CM0] * ((R)1 + (R)m[L_AC] * phi);
    c.cX = ((R)m[L_ETM] + (R)m[L_FTM] * th) * c.cM;
    return c;
}

template <typename R>
__device__ __forceinline__ R harm(R a, R b)
{
    R s = a + b;
    return s > (R)0 ? (R)2 * a * b / s : (R)0;
}

// Face conductivities at the face state (theta_f, P_f) between two nodes of
// layers la and lb (harmonic mean across an interface).
template <typename R>
__device__ __forceinline__ KCoef<R> face_k(const WallDev &W, int la, int lb, R thf, R Pf)
{
    R phi = Pf / psat_th(thf);
    KCoef<R> a = law_k<R>(W.lay[la], phi);
    if (la == lb) return a;
    KCoef<R> b = law_k<R>(W.lay[lb], phi);
    KCoef<R> k;
    k.kT = harm(a.kT, b.kT);
    k.kM = harm(a.kM, b.kM);
    k.kX = harm(a.kX, b.kX);
    return k;
}

// ------------------------------------------------------- fast arithmetic
// Reciprocal: hardware estimate refined by two Newton-Raphson steps
// x <- x + x (1 - b x) (quadratic convergence; ~1 ulp in FP64).  FP32 keeps
// the 1-ulp hardware estimate, well inside the FP32 path's error budget.
__device__ __forceinline__ double rcp_nr(double b)
{
    double x = __builtin_amdgcn_rcp(b);
    double e = fma(-b, x, 1.0);
    x = fma(x, e, x);
    e = fma(-b, x, 1.0);
    return fma(x, e, x);
}
__device__ __forceinline__ float rcp_nr(float b)
{
    float x = __builtin_amdgcn_rcpf(b);
    return fmaf(x, fmaf(-b, x, 1.0f), x);
}

// a / b from the refined reciprocal plus one residual correction
// q <- q + (a - b q) / b (within about one ulp of the rounded quotient).
template <typename R>
__device__ __forceinline__ R div_nr(R a, R b)
{
    const R x = rcp_nr(b);
    const R q = a * x;
    return fma(fma(-b, q, a), x, q);
}

// exp(a) for |a| well inside the FP64 range (no overflow / special-value
// handling): Cody-Waite reduction a = k ln2 + r, |r| <= ln2/2, with ln2 split
// into a 32-bit head and a tail, then the degree-9 polynomial that
// interpolates exp at the 10 Chebyshev nodes of [-ln2/2, ln2/2] (coefficients
// computed in 60-digit arithmetic and rounded to FP64; relative error on the
// interval 1.9e-14, far below what the FP64 parity bar of 1e-12 on the fields
// can see: degree 11, at 4e-18, cost two more dependent FMAs per call and
// 2.7 % of the FP64 step) and a scaling by 2^k.
__device__ __forceinline__ double exp_bounded(double a)
{
    const double k = rint(a * 1.4426950408889634074);
    double r = fma(-k, 6.93147180369123816490e-01, a);
    r = fma(-k, 1.90821492927058770002e-10, r);
    double p = 2.7632640675430236e-06;
    p = fma(p, r, 2.4884459751751116e-05);
    p = fma(p, r, 0.0001984119064754424);
    p = fma(p, r, 0.0013888801749656543);
    p = fma(p, r, 0.008333333367311603);
    p = fma(p, r, 0.04166666704055191);
    p = fma(p, r, 0.16666666666615648);
    p = fma(p, r, 0.4999999999943859);
    p = fma(p, r, 1.0000000000000013);
    p = fma(p, r, 1.0000000000000135);
    return __builtin_amdgcn_ldexp(p, (int)k);
}
__device__ __forceinline__ float exp_bounded(float a) { return __expf(a); }

// 2^y for |y| well inside the FP64 exponent range: y = k + f with k the
// nearest integer (f = y - k is exact), |f| <= 1/2, then the degree-9
// polynomial that interpolates 2^f at the 10 Chebyshev nodes of [-1/2, 1/2]
// (coefficients computed in 60-digit arithmetic and rounded to FP64;
// relative error on the interval 1.8e-14) and a scaling by 2^k.
__device__ __forceinline__ double exp2_bounded(double y)
{
    const double k = rint(y);
    const double f = y - k;
    double p = 1.0205905413765595e-07;
    p = fma(p, f, 1.325964524488711e-06);
    p = fma(p, f, 1.5252672924850737e-05);
    p = fma(p, f, 0.0001540343375125101);
    p = fma(p, f, 0.0013333558200794592);
    p = fma(p, f, 0.009618129193934313);
    p = fma(p, f, 0.05550410866465167);
    p = fma(p, f, 0.2402265069564034);
    p = fma(p, f, 0.6931471805599462);
    p = fma(p, f, 1.0000000000000135);
    return __builtin_amdgcn_ldexp(p, (int)k);
}

// The Magnus saturation pressure in the form 1 / Ps(theta) = 2^(C0 + C1 / d),
// d = theta + 243.04: with 17.625 theta / d = 17.625 - 17.625 x 243.04 / d,
// C1 = 17.625 x 243.04 / ln 2 and C0 = -17.625 / ln 2 - log2(610.94).
constexpr double kMagC1 = 6179.899623251146;
constexpr double kMagC0 = -34.6823869863494;

// ------------------------------------------------- Table 1 material law
// The load-bearing material of Sec. 6 (Table 1), read as follows (every
// coefficient of Table 2 is reproduced within 1.5 % at 20 degC):
//   suction s = -R_v T ln(phi) (J/kg, Kelvin's law with rho_l dropped);
//   f = sum_i w_i [1 + (c_i s)^n_i]^(-m_i), (w, c, n) = (47.1, 1.25e-5, 1.65)
//       and (109.9, 1.8e-5, 6), m_i = 1 - 1/n_i;
//   c_M = (df/dphi) / P_s, c_TT = rho_0 c_0 + c_w f, c_TM = c_w theta c_M;
//   k_TT = 0.2 + 0.0045 f, k_TM = L_v delta_v,
//   delta_v = 1.88e-6 / T (1 - f/157) / (0.503 (1 - f/157)^2 + 0.497),
//   k_M = 1.97e-10 10^(1.44 - 0.07 log10(2 phi)) + 1.77e-7 exp(-8 (2 phi - 2)^2).
// A layer's k0, kM0, c0 and cM0 multiply lambda, (k_M, k_TM), rho_0 c_0 and
// (c_M, c_TM).  Powers are written as exponentials of logarithms (FP64: the
// bounded exponential above and the library logarithm; FP32: the hardware
// base-2 exponential and logarithm).
constexpr double kT1Rv = 461.5, kT1Rho0c0 = 790.0 * 870.0;

// ln(x) for a positive normal x: x = m 2^e with m in [1/sqrt2, sqrt2), then
// ln m = 2 artanh(z), z = (m - 1)/(m + 1), |z| <= 0.1716, by its Taylor
// series through z^21 (truncation below 1e-18 relative), and e ln2 with ln2
// split into a head and a tail.
__device__ __forceinline__ double log_bounded(double x)
{
    int e;
    double m = frexp(x, &e);
    if (m < 0.70710678118654752440) { m *= 2.0; e -= 1; }
    const double z = div_nr(m - 1.0, m + 1.0);
    const double z2 = z * z;
    double p = 1.0 / 21.0;
    p = fma(p, z2, 1.0 / 19.0);
    p = fma(p, z2, 1.0 / 17.0);
    p = fma(p, z2, 1.0 / 15.0);
    p = fma(p, z2, 1.0 / 13.0);
    p = fma(p, z2, 1.0 / 11.0);
    p = fma(p, z2, 1.0 / 9.0);
    p = fma(p, z2, 1.0 / 7.0);
    p = fma(p, z2, 1.0 / 5.0);
    p = fma(p, z2, 1.0 / 3.0);
    p = fma(p, z2, 1.0);
    const double de = (double)e;
    return fma(de, 6.93147180369123816490e-01, fma(de, 1.90821492927058770002e-10, 2.0 * z * p));
}
__device__ __forceinline__ double t1_ln(double x) { return log_bounded(x); }
__device__ __forceinline__ float t1_ln(float x) { return __builtin_amdgcn_logf(x) * 0.69314718f; }
__device__ __forceinline__ double t1_exp(double x) { return exp_bounded(x); }
__device__ __forceinline__ float t1_exp(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504f); }

// Moisture content f and df/dphi at temperature T (K), given ln(phi).
template <typename R>
__device__ __forceinline__ void t1_isotherm(R T, R lnphi, R &f, R &dfdphi_phi)
{
    // s is clamped away from 0 (phi >= 1): the powers then vanish
    const R s = fmax(-(R)kT1Rv * T * lnphi, (R)1e-30);
    // mode 1: n = 1.65, m = 1 - 1/1.65; with p = x^n, a = 1 + p and e = a^-m
    // the derivative term x^(n-1) a^(-m-1) is p e / (x a): four
    // transcendentals and one division instead of five transcendentals
    const R m1 = (R)(1.0 - 1.0 / 1.65);
    const R x1 = (R)1.25e-5 * s;
    const R p1 = t1_exp((R)1.65 * t1_ln(x1));
    const R a1 = (R)1 + p1;
    const R e1 = t1_exp(-m1 * t1_ln(a1));
    const R f1 = (R)47.1 * e1;
    const R g1 = (R)(47.1 * (1.0 - 1.0 / 1.65) * 1.65 * 1.25e-5) * div_nr(p1 * e1, x1 * a1);
    // mode 2: n = 6, m = 5/6 (integer powers by products; a^(-m-1) = e / a)
    const R m2 = (R)(5.0 / 6.0);
    const R x = (R)1.8e-5 * s;
    const R x2 = x * x, x4 = x2 * x2;
    const R a2 = (R)1 + x4 * x2;
    const R e2 = t1_exp(-m2 * t1_ln(a2));
    const R f2 = (R)109.9 * e2;
    const R g2 = (R)(109.9 * (5.0 / 6.0) * 6.0 * 1.8e-5) * div_nr((x4 * x) * e2, a2);
    f = f1 + f2;
    // -df/ds = g1 + g2; ds/dphi = -R_v T / phi: phi df/dphi = (g1 + g2) R_v T
    dfdphi_phi = (g1 + g2) * ((R)kT1Rv * T);
}

// Magnus saturation pressure for the Table 1 law (bounded exponential).
__device__ __forceinline__ double t1_psat(double th)
{
    return 610.94 * exp_bounded(div_nr(17.625 * th, th + 243.04));
}
__device__ __forceinline__ float t1_psat(float th) { return psat_th(th); }

// The Table 1 law's conductivity functions at (theta, P), before the layer
// scales: (lambda, k_M, L_v delta_v).
template <typename R>
__device__ __forceinline__ KCoef<R> t1_kfun(R th, R P, R Lv)
{
    const R T = th + (R)273.15;
    const R phi = div_nr(P, t1_psat(th));
    const R lnphi = t1_ln(phi);
    R f, g;
    t1_isotherm<R>(T, lnphi, f, g);
    const R u = (R)1 - f * (R)(1.0 / 157.0);
    const R dv = div_nr((R)1.88e-6 * u, T * ((R)0.503 * u * u + (R)0.497));
    // 10^(1.44 - 0.07 log10(2 phi)) = 10^1.44 (2 phi)^(-0.07)
    const R a = (R)2 * phi - (R)2;
    KCoef<R> k;
    k.kT = (R)0.2 + (R)0.0045 * f;
    k.kM = (R)(1.97e-10 * 27.542287033381662) * t1_exp((R)-0.07 * (lnphi + (R)0.69314718055994531)) +
           (R)1.77e-7 * t1_exp((R)-8 * a * a);
    k.kX = Lv * dv;
    return k;
}

// Conductivities of the Table 1 law at (theta, P) for layer scales m.
template <typename R>
__device__ __forceinline__ KCoef<R> t1_law_k(const double *m, R th, R P, R Lv)
{
    KCoef<R> k = t1_kfun<R>(th, P, Lv);
    k.kT *= (R)m[L_K0];
    k.kM *= (R)m[L_KM0];
    k.kX *= (R)m[L_KM0];
    return k;
}

// Capacities of the Table 1 law at (theta, P) for layer scales m.
template <typename R>
__device__ __forceinline__ CCoef<R> t1_law_c(const double *m, R th, R P, R cw)
{
    const R T = th + (R)273.15;
    const R ps = t1_psat(th);
    R f, g;
    t1_isotherm<R>(T, t1_ln(div_nr(P, ps)), f, g);
    CCoef<R> c;
    c.cT = (R)m[L_C0] * (R)kT1Rho0c0 + cw * f;
    c.cM = (R)m[L_CM0] * div_nr(g, P);          // (df/dphi) / P_s = (phi df/dphi) / P
    c.cX = cw * th * c.cM;
    return c;
}

// Face conductivities under the Table 1 law (harmonic mean across layers).
template <typename R>
__device__ __forceinline__ KCoef<R> t1_face_k(const WallDev &W, int la, int lb, R thf, R Pf, R Lv)
{
    KCoef<R> a = t1_law_k<R>(W.lay[la], thf, Pf, Lv);
    if (la == lb) return a;
    KCoef<R> b = t1_law_k<R>(W.lay[lb], thf, Pf, Lv);
    KCoef<R> k;
    k.kT = harm(a.kT, b.kT);
    k.kM = harm(a.kM, b.kM);
    k.kX = harm(a.kX, b.kX);
    return k;
}

// Neumaier (1974) compensated accumulation.
__device__ __forceinline__ void neumaier_add(double &s, double &c, double x)
{
    double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

// Storage traits: FP64 keeps absolute values, FP32 deviations from (T0, P0).
template <typename R> struct Store;
template <> struct Store<double> {
    static __device__ __forceinline__ double thref(const WallDev &W) { return -273.15; }
    static __device__ __forceinline__ double pref(const WallDev &W) { return 0.0; }
    static __device__ __forceinline__ double tref(const WallDev &W) { return 0.0; }
};
template <> struct Store<float> {
    static __device__ __forceinline__ float thref(const WallDev &W) { return (float)W.th0; }
    static __device__ __forceinline__ float pref(const WallDev &W) { return (float)W.P0; }
    static __device__ __forceinline__ double tref(const WallDev &W) { return W.T0; }
};

} // namespace dfhm
