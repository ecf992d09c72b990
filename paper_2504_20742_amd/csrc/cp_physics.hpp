// cp_physics.hpp -- device functions of the contrail finite-volume step (gfx950).
//
// Gas model, phase-change rates and the sub-cycled source of Tegethoff & Wheeler
// (arXiv 2504.20742), Sec. 2.2 (Eq. 1-21) and Sec. 3.1 (Eq. 22-26); Roe flux,
// MUSCL / van Leer and central viscous fluxes of Sec. 3.2.  Flux helpers are
// templated on the arithmetic type (double for the FP64 path, float for the mixed
// path); the phase-change source is always evaluated in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cp {

constexpr int NVAR = 15;
// With two liquid populations (Sec. 2.2) the homogeneously nucleated droplets take
// four more variables, 15..18; the soot-activated ones keep 5..8.
constexpr int NVAR_BI = 19;

// -------------------------------------------------------------- constants
// Calorically perfect carrier: dry-air pseudo-component (78/21/1 % N2/O2/Ar of the
// paper's free stream, diatomic) + water vapour (triatomic); reference 273.15 K.
constexpr double kTref = 273.15;
constexpr double kRa = 287.0, kCpa = 1004.5;
constexpr double kRv = 461.52, kCpv = 1846.08;
constexpr double kCva = kCpa - kRa, kCvv = kCpv - kRv;
constexpr double kGv = 4.0 / 3.0;
constexpr double kCl = 4218.0, kCi = 2106.0;
constexpr double kLv0 = 2.5008e6, kLs0 = 2.8345e6;
constexpr double kRhoL = 1000.0, kRhoS = 917.0;
constexpr double kKb = 1.380649e-23;
constexpr double kPr = 0.71, kPrT = 0.9, kPrV = 1.0, kSct = 0.7;
constexpr double kMu0 = 1.716e-5, kSuth = 110.4;
constexpr double kD0 = 2.11e-5, kDexp = 1.94, kP0 = 101325.0;
constexpr double kQc = 1.0, kYoungA = 11.0;
constexpr double kNmin = 1.0, kSubSafety = 0.2;
// floor of p_v [Pa] under the logarithm: below p_sat over ice at 150 K (6e-6 Pa), the
// cold end of the property range, so a cell without vapour never reads as supersaturated
constexpr double kPvFloor = 1.0e-9;
constexpr double kRmin2 = 1.0e-20, kRmin3 = 1.0e-30;   // (1e-10 m)^2, (1e-10 m)^3
constexpr double kPi = 3.14159265358979323846;
constexpr double kFourThirdsPi = 4.0 / 3.0 * kPi;
constexpr double kLn100 = 4.605170185988092;   // ln(100): hPa -> Pa

// Sonntag coefficients, ln p [hPa] = a/T + b + c T + d T^2 + e ln T (Sec. 2.1)
struct Sonntag { double a, b, c, d, e; };
constexpr Sonntag kSonW = {-6096.9385, 16.635794, -2.711193e-2, 1.673952e-5, 2.433502};
constexpr Sonntag kSonI = {-6024.5282, 24.7219, 1.0613868e-2, -1.3198825e-5, -0.49382577};

// Case constants the host derives once (transcendentals evaluated on the host).
struct SourceParams {
    double f_theta;        // Eq. 9 at the contact angle
    double het_freeze;     // k_imm * n_s * 4 pi r_g^2 exp(2 ln^2 s_g)  (Eq. 14)
    double cnt_const;      // q_c sqrt(2 N_A^3 / (pi M^3)) / rho_l        (Eq. 4)
    double ice_ratio[4];   // (rho_l / rho_s)^(k/3)
    int n_sub_max;
    int enabled;
    int equilibrium;       // 1: the equilibrium comparison model replaces the kinetics
    // water property table (null: closed forms): nodes T0 + k h, k < n, each holding
    // (f, f', f''/2) of ln p_sat over liquid, ln p_sat over ice, surface tension
    const double *ptab;
    double ptab_T0, ptab_h;
    int ptab_n;
};

// Division: IEEE in FP64; a hardware reciprocal (about 1 ulp) in the FP32 path.
__device__ __forceinline__ double fdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Division for the transport terms: FP32 as fdiv; FP64 from the hardware
// reciprocal refined by two Newton steps, with one residual correction of the
// quotient (within about 1 ulp of the IEEE quotient, at a fraction of its cost).
// The phase-change source keeps IEEE division.
__device__ __forceinline__ double trcp(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    r = fma(fma(-b, r, 1.0), r, r);
    return fma(fma(-b, r, 1.0), r, r);
}
__device__ __forceinline__ float trcp(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double tdiv(double a, double b)
{
    const double r = trcp(b), q = a * r;
    return fma(fma(-b, q, a), r, q);
}
__device__ __forceinline__ float tdiv(float a, float b) { return fdiv(a, b); }

// Square root and positive power for the transport terms: IEEE in FP64; the
// hardware instructions (v_sqrt_f32, v_log_f32 / v_exp_f32, about 1 ulp) in FP32.
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fpow_pos(double x, double e) { return exp(e * log(x)); }
__device__ __forceinline__ float fpow_pos(float x, float e)
{
    return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(x));
}

// -------------------------------------------------------------- gas model
template <class R> __device__ __forceinline__ R gas_R(R Y) { return (R(1) - Y) * R(kRa) + Y * R(kRv); }
template <class R> __device__ __forceinline__ R gas_cp(R Y) { return (R(1) - Y) * R(kCpa) + Y * R(kCpv); }
template <class R> __device__ __forceinline__ R gas_cv(R Y) { return (R(1) - Y) * R(kCva) + Y * R(kCvv); }
// h = cp(Y) T + h0(Y), with h_air = cp_a (T - Tref) and h_vap = L0 + cp_v (T - Tref)
template <class R> __device__ __forceinline__ R gas_h0(R Y)
{
    return -(R(1) - Y) * R(kCpa * kTref) + Y * R(kLv0 - kCpv * kTref);
}

// Temperature from specific internal energy e and vapour fraction Y (Eq. 23).
template <class R> __device__ __forceinline__ R gas_T(R e, R Y)
{
    return fdiv(e + (R(1) - Y) * R(kCpa * kTref) - Y * R(kLv0 - kCpv * kTref), gas_cv(Y));
}

template <class R> __device__ __forceinline__ R sutherland(R T)
{
    R t = T * R(1.0 / kTref);
    return fdiv(R(kMu0) * t * fsqrt(t) * R(kTref + kSuth), T + R(kSuth));
}
// the same law with the transport division, for the flux kernels
template <class R> __device__ __forceinline__ R sutherland_t(R T)
{
    R t = T * R(1.0 / kTref);
    return tdiv(R(kMu0) * t * fsqrt(t) * R(kTref + kSuth), T + R(kSuth));
}

// ======================================================================
//  Phase-change source (Sec. 2.2), FP64
// ======================================================================
__device__ __forceinline__ double ln_psat(const Sonntag &s, double T)
{
    return s.a / T + s.b + s.c * T + s.d * T * T + s.e * log(T) + kLn100;
}

// T_sat(p_v): Newton in x = 1/T, four steps from the gas temperature (Eq. 1).
__device__ __forceinline__ double t_sat(const Sonntag &s, double lnpv, double T)
{
    double x = 1.0 / T;
    #pragma unroll
    for (int it = 0; it < 4; ++it) {
        double ix = 1.0 / x;
        double g = s.a * x + s.b + s.c * ix + s.d * ix * ix - s.e * log(x) + kLn100 - lnpv;
        double gp = s.a - s.c * ix * ix - 2.0 * s.d * ix * ix * ix - s.e * ix;
        x -= g / gp;
    }
    return 1.0 / x;
}

__device__ __forceinline__ double surface_tension(double T)
{
    double tau = 1.0 - T / 647.096;              // IAPWS 1994; zero at and above the critical point
    if (!(tau > 0.0)) return 0.0;
    return 0.2358 * pow(tau, 1.256) * (1.0 - 0.625 * tau);
}

// ------------------------------------------------ tabulated water properties
// The paper interpolates pre-tabulated water properties with a second-order
// Taylor expansion (Sec. 3.2): about the node nearest T (the end node outside the
// table), f + f' d + (f''/2) d^2.  Without a table the closed forms are used.
constexpr int kPropLnpw = 0, kPropLnpi = 1, kPropSigma = 2, kPropStride = 9;

__device__ __forceinline__ double ptab_eval(const SourceParams &sp, int q, double T, double *dfdT)
{
    const double kd = fmin(fmax(floor((T - sp.ptab_T0) / sp.ptab_h + 0.5), 0.0), (double)(sp.ptab_n - 1));
    const int k = (int)kd;
    const double *c = sp.ptab + kPropStride * k + 3 * q;
    const double d = T - (sp.ptab_T0 + k * sp.ptab_h);
    if (dfdT) *dfdT = c[1] + 2.0 * c[2] * d;
    return c[0] + d * (c[1] + d * c[2]);
}

__device__ __forceinline__ double prop_lnp(const SourceParams &sp, bool ice, double T)
{
    if (sp.ptab) return ptab_eval(sp, ice ? kPropLnpi : kPropLnpw, T, nullptr);
    return ln_psat(ice ? kSonI : kSonW, T);
}

__device__ __forceinline__ double prop_sigma(const SourceParams &sp, double T)
{
    if (sp.ptab) return ptab_eval(sp, kPropSigma, T, nullptr);
    return surface_tension(T);
}

// T_sat: four Newton steps in x = 1/T from the gas temperature, or from 373.15 K in
// hotter gas (the upper end of the Sonntag fits, beyond which the extrapolated
// ln p_sat bends and the steps can settle on a spurious root); with a table the same
// steps on the expanded ln p_sat (slope in x: -T^2 d ln p_sat / dT).
__device__ __forceinline__ double prop_tsat(const SourceParams &sp, bool ice, double lnpv, double T)
{
    T = fmin(T, 373.15);
    if (!sp.ptab) return t_sat(ice ? kSonI : kSonW, lnpv, T);
    double x = 1.0 / T;
    #pragma unroll
    for (int it = 0; it < 4; ++it) {
        const double t = 1.0 / x;
        double g;
        const double f = ptab_eval(sp, ice ? kPropLnpi : kPropLnpw, t, &g) - lnpv;
        x = x - f / (-t * t * g);
    }
    return 1.0 / x;
}

// Young's parameter nu (Eq. 16) with gamma, c_p of the vapour and q_c.
__device__ __forceinline__ double young_nu(double Tsat, double h)
{
    const double q = Tsat / h;
    return kRv * q * (kYoungA - 0.5 - (2.0 - kQc) / (2.0 * kQc) * (kGv + 1.0) / (2.0 * kGv) * kCpv * q);
}

// Young's growth law, beta = 0 (Eq. 16): Kn = lbar / 2r.
__device__ __forceinline__ double young_G(double lam, double drive, double r, double rho_p, double h,
                                          double nu, double lbar)
{
    // r (1 + 3.78 (1 - nu) Kn / Pr_v) with Kn = lbar / (2 r): one division
    return lam * drive / (rho_p * h * (r + (1.89 / kPrV) * (1.0 - nu) * lbar));
}

// A particle population (mu0 > N_MIN) is valid while r20 and r30 are at least a
// molecular radius (1e-10 m); below that its mass has evaporated.
__device__ __forceinline__ bool pop_valid(double m0, double m2, double m3)
{
    return m0 > kNmin && m2 > m0 * kRmin2 && m3 > m0 * kRmin3;
}

struct CellThermo {      // quantities of one state that the rates need
    double T, u, v, rho, cpm, Rm, p;
};

__device__ __forceinline__ void cell_thermo(const double *U, CellThermo &c)
{
    c.rho = U[0];
    const double ir = 1.0 / U[0];
    c.u = U[1] * ir;
    c.v = U[2] * ir;
    double Y = U[4] * ir;
    double e = U[3] * ir - 0.5 * (c.u * c.u + c.v * c.v);
    c.T = gas_T<double>(e, Y);
    c.Rm = gas_R<double>(Y);
    c.cpm = gas_cp<double>(Y);
    c.p = c.rho * c.Rm * c.T;
}

struct Rates {
    double dM[4], dN[4], act, mdot_f, Gl, Gs;
    bool gone_l, gone_s;   // droplets / crystals left without mass (r20 below 1e-10 m)
};

// One evaluation of nucleation (Eq. 3-11), growth (Eq. 16, 21), freezing
// (Eq. 12-15) and moment rates (Eq. 21); h bounds the activation rate.
__device__ inline void phase_rates(const double *U, double h, const SourceParams &sp, const CellThermo &th,
                                   Rates &r)
{
    const double T = th.T;
    const double rv = U[4];
    const double M0 = U[5], M1 = U[6], M2 = U[7], M3 = U[8];
    const double N0 = U[9], N1 = U[10], N2 = U[11];
    const double Ns = U[13], Na = U[14];

    double pv = fmax(rv * kRv * T, kPvFloor);
    const double lnpv = log(pv);
    const double lw = prop_lnp(sp, false, T);
    const double lnSl = lnpv - lw;
    const double sig = prop_sigma(sp, T);
    const double hfg = kLv0 + (kCpv - kCl) * (T - kTref);
    const double hsg = kLs0 + (kCpv - kCi) * (T - kTref);
    const double mu = sutherland<double>(T);
    const double lam = th.cpm * mu * (1.0 / kPr);
    const double lbar = 1.5 * mu * sqrt(th.Rm * T) / th.p;
    // Kelvin radius 2 sigma / (rho_l R_v T ln S_l) (Eq. 3): the critical radius where
    // S_l > 1, the curvature term of the droplets' growth drive either way
    const double kel = fabs(lnSl) < 1e-12 ? 0.0 : 2.0 * sig / (kRhoL * kRv * T * lnSl);

    double Jl = 0.0, rc = 0.0;
    r.act = 0.0;
    if (lnSl > 0.0 && rv > 0.0) {
        rc = kel;                                                       // Eq. 3
        const double iT = 1.0 / T, hT = hfg * iT;
        const double x = (kFourThirdsPi / kKb) * sig * rc * rc * iT;    // dG*/kT
        const double K = sp.cnt_const * sqrt(sig) * rv * rv;            // Eq. 4
        const double phi = 2.0 * kQc * kGv / ((kGv + 1.0) * kCpv)
                           * hT * (hT * (1.0 / kRv) - 1.0);             // Eq. 5
        const double inv1p = 1.0 / (1.0 + phi);
        Jl = K * exp(-x) * inv1p;
        if (Ns > Na) {                                                  // Eq. 10 on free soot
            double Jh = K * exp(-sp.f_theta * x) * inv1p;
            r.act = fmin(Jh, (Ns - Na) / h);
        }
        Jl += r.act;
    }

    r.Gl = 0.0;
    r.Gs = 0.0;
    const bool liq = pop_valid(M0, M2, M3);
    const bool ice = pop_valid(N0, N2, U[12]);
    r.gone_l = M0 > kNmin && !liq;
    r.gone_s = N0 > kNmin && !ice;
    if (liq) {
        double r20 = sqrt(M2 / M0);
        double Ts = prop_tsat(sp, false, lnpv, T);
        double dT = Ts - T;
        double drive = fabs(lnSl) < 1e-12 ? dT - 2.0 * sig * Ts / (kRhoL * hfg * r20) : dT * (1.0 - kel / r20);
        r.Gl = young_G(lam, drive, r20, kRhoL, hfg, young_nu(Ts, hfg), lbar);
    }
    if (ice) {
        double r20 = sqrt(N2 / N0);
        double Ts = prop_tsat(sp, true, lnpv, T);
        r.Gs = young_G(lam, Ts - T, r20, kRhoS, hsg, young_nu(Ts, hsg), lbar);
    }

    double F[4] = {0.0, 0.0, 0.0, 0.0};
    r.mdot_f = 0.0;
    if (T < kTref && liq) {
        double l2 = log(M2 / M0), l3 = log(M3 / M0);
        double s2 = fmax(2.0 / 3.0 * l3 - l2, 0.0);
        double lrg = 0.5 * l2 - s2;
        double daw = 1.0 - exp(prop_lnp(sp, true, T) - lw);
        daw = fmin(fmax(daw, 0.26), 0.34);
        double lg = -906.7 + 8502.0 * daw - 26924.0 * daw * daw + 29180.0 * daw * daw * daw;
        double Jf = 1.0e6 * exp(lg * 2.302585092994046) + sp.het_freeze * Ns;   // Eq. 12 + 14
        double c = Jf * kFourThirdsPi;
        F[0] = c * M3;
        F[1] = c * M0 * exp(4.0 * lrg + 8.0 * s2);
        F[2] = c * M0 * exp(5.0 * lrg + 12.5 * s2);
        F[3] = c * M0 * exp(6.0 * lrg + 18.0 * s2);
        r.mdot_f = kRhoL * kFourThirdsPi * F[3];
    }

    const double Mm[3] = {M0, M1, M2};
    const double Nm[3] = {N0, N1, N2};
    double rk = 1.0;
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        double gl = k ? k * Mm[k - 1] * r.Gl : 0.0;
        double gs = k ? k * Nm[k - 1] * r.Gs : 0.0;
        r.dM[k] = gl + Jl * rk - F[k];
        r.dN[k] = gs + sp.ice_ratio[k] * F[k];
        rk *= rc;
    }
}

// Source vector from moment rates (Eq. 25-26 exchange): water exact to rounding.
__device__ __forceinline__ void exchange(const CellThermo &th, const double *dM, const double *dN, double act,
                                         double mdot_f, double *S)
{
    #pragma unroll
    for (int k = 0; k < 4; ++k) { S[5 + k] = dM[k]; S[9 + k] = dN[k]; }
    S[13] = 0.0;
    S[14] = act;
    S[4] = -kFourThirdsPi * (kRhoL * S[8] + kRhoS * S[12]);
    S[0] = S[4];
    S[1] = S[4] * th.u;
    S[2] = S[4] * th.v;
    const double T = th.T;
    const double ml = kFourThirdsPi * kRhoL * S[8] + mdot_f;
    const double ms = kFourThirdsPi * kRhoS * S[12] - mdot_f;
    const double hfg = kLv0 + (kCpv - kCl) * (T - kTref);
    const double hsg = kLs0 + (kCpv - kCi) * (T - kTref);
    const double hv = kLv0 + kCpv * (T - kTref);
    const double ke = 0.5 * (th.u * th.u + th.v * th.v);
    S[3] = -ml * (hv - hfg + ke) - ms * (hv - hsg + ke) + mdot_f * (hsg - hfg);
}


// Two liquid populations (the bimodal moments of Sec. 2.2): the soot-activated
// droplets in 5..8 (population 0), the homogeneously nucleated ones in 15..18
// (population 1).  The one-population functions above are kept as their own code:
// folding them into these templates (NP = 1) made the table-driven source 7 %
// slower on the GPU.
__device__ __forceinline__ constexpr int liq_base(int pop) { return pop ? 15 : 5; }

template <int NP> struct RatesN {
    double dM[NP][4], dN[4], act, mdot_f, Gl[NP], Gs;
    double F[NP][4];         // moments each liquid population loses to freezing
    bool gone_l[NP], gone_s; // droplets / crystals left without mass (r20 below 1e-10 m)
};

// One evaluation of nucleation (Eq. 3-11), growth (Eq. 16, 21), freezing
// (Eq. 12-15) and moment rates (Eq. 21) for NP liquid populations (used with NP = 2);
// h bounds the activation rate.  The soot-activated droplets (population 0)
// gain the activation rate and freeze by the homogeneous and immersion rates, the
// homogeneously nucleated ones (population 1) gain the homogeneous rate and freeze
// by the homogeneous rate alone (immersion needs a soot core).
template <int NP>
__device__ inline void phase_rates_n(const double *U, double h, const SourceParams &sp, const CellThermo &th,
                                     RatesN<NP> &r)
{
    const double T = th.T;
    const double rv = U[4];
    const double N0 = U[9], N1 = U[10], N2 = U[11];
    const double Ns = U[13], Na = U[14];

    double pv = fmax(rv * kRv * T, kPvFloor);
    const double lnpv = log(pv);
    const double lw = prop_lnp(sp, false, T);
    const double lnSl = lnpv - lw;
    const double sig = prop_sigma(sp, T);
    const double hfg = kLv0 + (kCpv - kCl) * (T - kTref);
    const double hsg = kLs0 + (kCpv - kCi) * (T - kTref);
    const double mu = sutherland<double>(T);
    const double lam = th.cpm * mu * (1.0 / kPr);
    const double lbar = 1.5 * mu * sqrt(th.Rm * T) / th.p;
    // Kelvin radius 2 sigma / (rho_l R_v T ln S_l) (Eq. 3): the critical radius where
    // S_l > 1, the curvature term of the droplets' growth drive either way
    const double kel = fabs(lnSl) < 1e-12 ? 0.0 : 2.0 * sig / (kRhoL * kRv * T * lnSl);

    double J[NP], rc = 0.0;
    #pragma unroll
    for (int pop = 0; pop < NP; ++pop) J[pop] = 0.0;
    r.act = 0.0;
    if (lnSl > 0.0 && rv > 0.0) {
        rc = kel;                                                       // Eq. 3
        const double iT = 1.0 / T, hT = hfg * iT;
        const double x = (kFourThirdsPi / kKb) * sig * rc * rc * iT;    // dG*/kT
        const double K = sp.cnt_const * sqrt(sig) * rv * rv;            // Eq. 4
        const double phi = 2.0 * kQc * kGv / ((kGv + 1.0) * kCpv)
                           * hT * (hT * (1.0 / kRv) - 1.0);             // Eq. 5
        const double inv1p = 1.0 / (1.0 + phi);
        const double Jhom = K * exp(-x) * inv1p;
        if (Ns > Na) {                                                  // Eq. 10 on free soot
            double Jh = K * exp(-sp.f_theta * x) * inv1p;
            r.act = fmin(Jh, (Ns - Na) / h);
        }
        if constexpr (NP == 1) {
            J[0] = Jhom;
            J[0] += r.act;
        } else {
            J[0] = r.act;
            J[1] = Jhom;
        }
    }

    // growth (Eq. 16, 21) of each droplet population, then of the crystals
    bool liq[NP];
    #pragma unroll
    for (int pop = 0; pop < NP; ++pop) {
        const double *M = U + liq_base(pop);
        liq[pop] = pop_valid(M[0], M[2], M[3]);
        r.gone_l[pop] = M[0] > kNmin && !liq[pop];
        r.Gl[pop] = 0.0;
        if (liq[pop]) {
            double r20 = sqrt(M[2] / M[0]);
            double Ts = prop_tsat(sp, false, lnpv, T);
            double dT = Ts - T;
            double drive = fabs(lnSl) < 1e-12 ? dT - 2.0 * sig * Ts / (kRhoL * hfg * r20) : dT * (1.0 - kel / r20);
            r.Gl[pop] = young_G(lam, drive, r20, kRhoL, hfg, young_nu(Ts, hfg), lbar);
        }
    }
    r.Gs = 0.0;
    const bool ice = pop_valid(N0, N2, U[12]);
    r.gone_s = N0 > kNmin && !ice;
    if (ice) {
        double r20 = sqrt(N2 / N0);
        double Ts = prop_tsat(sp, true, lnpv, T);
        r.Gs = young_G(lam, Ts - T, r20, kRhoS, hsg, young_nu(Ts, hsg), lbar);
    }

    // freezing (Eq. 12-15) and the moment rates (Eq. 21) of each droplet population
    r.mdot_f = 0.0;
    #pragma unroll
    for (int pop = 0; pop < NP; ++pop) {
        const double *M = U + liq_base(pop);
        const double M0 = M[0], M1 = M[1], M2 = M[2], M3 = M[3];
        double *F = r.F[pop];
        F[0] = F[1] = F[2] = F[3] = 0.0;
        if (T < kTref && liq[pop]) {
            double l2 = log(M2 / M0), l3 = log(M3 / M0);
            double s2 = fmax(2.0 / 3.0 * l3 - l2, 0.0);
            double lrg = 0.5 * l2 - s2;
            double daw = 1.0 - exp(prop_lnp(sp, true, T) - lw);
            daw = fmin(fmax(daw, 0.26), 0.34);
            double lg = -906.7 + 8502.0 * daw - 26924.0 * daw * daw + 29180.0 * daw * daw * daw;
            double Jf = 1.0e6 * exp(lg * 2.302585092994046);                           // Eq. 12
            if (pop == 0) Jf += sp.het_freeze * Ns;                                      // Eq. 14
            double c = Jf * kFourThirdsPi;
            F[0] = c * M3;
            F[1] = c * M0 * exp(4.0 * lrg + 8.0 * s2);
            F[2] = c * M0 * exp(5.0 * lrg + 12.5 * s2);
            F[3] = c * M0 * exp(6.0 * lrg + 18.0 * s2);
            r.mdot_f += kRhoL * kFourThirdsPi * F[3];
        }
        const double Mm[3] = {M0, M1, M2};
        double rk = 1.0;
        #pragma unroll
        for (int k = 0; k < 4; ++k) {
            double gl = k ? k * Mm[k - 1] * r.Gl[pop] : 0.0;
            r.dM[pop][k] = gl + J[pop] * rk - F[k];
            rk *= rc;
        }
    }
    const double Nm[3] = {N0, N1, N2};
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        double gs = k ? k * Nm[k - 1] * r.Gs : 0.0;
        double Ft = r.F[0][k];
        if constexpr (NP == 2) Ft += r.F[1][k];
        r.dN[k] = gs + sp.ice_ratio[k] * Ft;
    }
}

// Source vector from moment rates (Eq. 25-26 exchange): water exact to rounding.
template <int NP>
__device__ __forceinline__ void exchange_n(const CellThermo &th, const double (*dM)[4], const double *dN, double act,
                                           double mdot_f, double *S)
{
    #pragma unroll
    for (int k = 0; k < 4; ++k) {
        S[5 + k] = dM[0][k];
        S[9 + k] = dN[k];
        if constexpr (NP == 2) S[15 + k] = dM[1][k];
    }
    S[13] = 0.0;
    S[14] = act;
    double liq3 = S[8];
    if constexpr (NP == 2) liq3 += S[18];
    S[4] = -kFourThirdsPi * (kRhoL * liq3 + kRhoS * S[12]);
    S[0] = S[4];
    S[1] = S[4] * th.u;
    S[2] = S[4] * th.v;
    const double T = th.T;
    const double ml = kFourThirdsPi * kRhoL * liq3 + mdot_f;
    const double ms = kFourThirdsPi * kRhoS * S[12] - mdot_f;
    const double hfg = kLv0 + (kCpv - kCl) * (T - kTref);
    const double hsg = kLs0 + (kCpv - kCi) * (T - kTref);
    const double hv = kLv0 + kCpv * (T - kTref);
    const double ke = 0.5 * (th.u * th.u + th.v * th.v);
    S[3] = -ml * (hv - hfg + ke) - ms * (hv - hsg + ke) + mdot_f * (hsg - hfg);
}

// True when every phase-change rate vanishes identically at U (subsaturated
// vapour, no droplets, no crystals): Q = 0 exactly, no sub-cycling needed.
template <int NV = NVAR> __device__ __forceinline__ bool source_inactive(const double *U, double T)
{
    if (U[5] > kNmin || U[9] > kNmin) return false;
    if constexpr (NV == NVAR_BI)
        if (U[15] > kNmin) return false;
    if (!(U[4] > 0.0)) return true;
    double pv = fmax(U[4] * kRv * T, kPvFloor);
    return !(log(pv) - ln_psat(kSonW, T) > 0.0);
}

// Conservative pre-filter in the storage precision: true when the cell certainly
// has no phase change (no particles and ln S_l below -0.01, far outside the FP32
// rounding of ln S_l); otherwise the FP64 test decides.
// Natural logarithm for the pre-filter: the hardware log2 (about 1 ulp) in FP32.
__device__ __forceinline__ float filter_ln(float x) { return __builtin_amdgcn_logf(x) * 0.6931471805599453f; }
__device__ __forceinline__ double filter_ln(double x) { return log(x); }

template <class R> __device__ __forceinline__ bool clearly_inactive(R rho_v, R M0, R N0, R T)
{
    if (M0 > R(kNmin) || N0 > R(kNmin)) return false;
    if (!(rho_v > R(0))) return true;
    const R lnSl = filter_ln(rho_v * R(kRv) * T) - (R(kSonW.a) / T + R(kSonW.b) + R(kSonW.c) * T +
                                                    R(kSonW.d) * T * T + R(kSonW.e) * filter_ln(T) + R(kLn100));
    return lnSl < R(-0.01);
}

// ----------------------------------------------- equilibrium comparison model
// Sec. 4.2 compares the kinetics with a model in which the cell's water is in
// phase equilibrium at every instant: the condensate is liquid at or above the
// melting point, ice below it (both at the melting point when the liquid branch
// settles below it and the ice branch above), the vapour at saturation over that
// phase, or all water evaporated.  Dry air, velocity and water are kept; the gas
// energy follows the kinetic exchange (condensate leaves with h_l or h_i at the end
// temperature), so the end temperature solves T_gas(T) = T on the chosen branch.
constexpr double kTmelt = 273.15;
constexpr double kRnew = 1.0e-7;   // m: particles of condensate that forms without soot

struct EqCell {
    double rho_a, rho_v, m_l, m_s, W, u, v, ke, rhoE;
};

// Gas temperature of the branch end state at trial temperature Ts (ice: condensate
// is ice); also the vapour density and condensate mass of that state.
__device__ __forceinline__ double eq_gas_T(const SourceParams &sp, const EqCell &e, bool ice, double Ts, double &rho_v,
                                           double &cond)
{
    const double rho_sat = exp(prop_lnp(sp, ice, Ts)) / (kRv * Ts);
    cond = fmax(e.W - rho_sat, 0.0);
    rho_v = e.W - cond;
    const double hv = kLv0 + kCpv * (Ts - kTref);
    const double hl = hv - (kLv0 + (kCpv - kCl) * (Ts - kTref)), hi = hv - (kLs0 + (kCpv - kCi) * (Ts - kTref));
    const double dL = (ice ? 0.0 : cond) - e.m_l, dI = (ice ? cond : 0.0) - e.m_s;
    const double rhoE = e.rhoE - dL * (hl + e.ke) - dI * (hi + e.ke);
    const double rho = e.rho_a + rho_v, Y = rho_v / rho;
    return gas_T<double>(rhoE / rho - e.ke, Y);
}

// The branch's end temperature: T_gas falls as Ts rises (warmer saturation keeps
// more vapour and releases less heat), so bisection on [100, 1000] K.
__device__ __forceinline__ double eq_root(const SourceParams &sp, const EqCell &e, bool ice)
{
    double a = 100.0, b = 1000.0, rv, c;
    for (int it = 0; it < 64; ++it) {
        const double m = 0.5 * (a + b);
        if (eq_gas_T(sp, e, ice, m, rv, c) > m) a = m;
        else b = m;
    }
    return 0.5 * (a + b);
}

__device__ __forceinline__ void eq_moments(double M, double N, double rho_p, double *mom)
{
    if (!(M > 0.0) || !(N > 0.0)) {
        mom[0] = mom[1] = mom[2] = mom[3] = 0.0;
        return;
    }
    const double r = cbrt(M / (kFourThirdsPi * rho_p * N));
    mom[0] = N;
    mom[1] = N * r;
    mom[2] = N * r * r;
    mom[3] = N * r * r * r;
}

// Q = (Phi_eq(U) - U) / dt; returns 1 when the cell changed phase state, else 0.
__device__ inline int source_equilibrium(const double *U, double dt, const SourceParams &sp, double *Q)
{
    CellThermo th;
    cell_thermo(U, th);
    if (source_inactive(U, th.T)) return 0;   // no condensate, not supersaturated over liquid
    EqCell e;
    e.rho_v = U[4];
    e.rho_a = U[0] - U[4];
    e.m_l = U[5] > kNmin ? kFourThirdsPi * kRhoL * U[8] : 0.0;
    e.m_s = U[9] > kNmin ? kFourThirdsPi * kRhoS * U[12] : 0.0;
    e.W = e.rho_v + e.m_l + e.m_s;
    e.u = th.u;
    e.v = th.v;
    e.ke = 0.5 * (th.u * th.u + th.v * th.v);
    e.rhoE = U[3];

    double T, rho_v, L = 0.0, I = 0.0, c;
    const double TL = eq_root(sp, e, false);
    eq_gas_T(sp, e, false, TL, rho_v, c);
    if (TL >= kTmelt) {
        T = TL;
        L = c;
    } else {
        const double TI = eq_root(sp, e, true);
        eq_gas_T(sp, e, true, TI, rho_v, c);
        if (TI < kTmelt) {
            T = TI;
            I = c;
        } else {   // both phases at the melting point; the ice share closes the energy balance
            T = kTmelt;
            const double C = fmax(e.W - exp(prop_lnp(sp, false, kTmelt)) / (kRv * kTmelt), 0.0);
            rho_v = e.W - C;
            const double hv = kLv0 + kCpv * (kTmelt - kTref);
            const double hl = hv - (kLv0 + (kCpv - kCl) * (kTmelt - kTref));
            const double hi = hv - (kLs0 + (kCpv - kCi) * (kTmelt - kTref));
            const double rho = e.rho_a + rho_v, Y = rho_v / rho;
            const double need = rho * (gas_h0<double>(Y) + gas_cv<double>(Y) * kTmelt + e.ke);
            const double all_liquid = e.rhoE - (C - e.m_l) * (hl + e.ke) + e.m_s * (hi + e.ke);
            I = fmin(fmax((need - all_liquid) / (hl - hi), 0.0), C);
            L = C - I;
        }
    }
    double Un[NVAR];
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) Un[v] = U[v];
    const double rho = e.rho_a + rho_v;
    const double hv = kLv0 + kCpv * (T - kTref);
    const double hl = hv - (kLv0 + (kCpv - kCl) * (T - kTref)), hi = hv - (kLs0 + (kCpv - kCi) * (T - kTref));
    Un[0] = rho;
    Un[1] = rho * e.u;
    Un[2] = rho * e.v;
    Un[3] = e.rhoE - (L - e.m_l) * (hl + e.ke) - (I - e.m_s) * (hi + e.ke);
    Un[4] = rho_v;
    // particles: kept across freezing and melting; new condensate on the soot, or on
    // kRnew particles without soot
    const double C = L + I;
    double N = (U[5] > kNmin ? U[5] : 0.0) + (U[9] > kNmin ? U[9] : 0.0);
    bool seeded = false;
    if (C > 0.0 && !(N > kNmin)) {
        if (U[13] > kNmin) {
            N = U[13];
            seeded = true;
        } else {
            N = C / (kFourThirdsPi * (I > 0.0 ? kRhoS : kRhoL) * kRnew * kRnew * kRnew);
        }
    }
    eq_moments(L, C > 0.0 ? N * L / C : 0.0, kRhoL, Un + 5);
    eq_moments(I, C > 0.0 ? N * I / C : 0.0, kRhoS, Un + 9);
    if (seeded) Un[14] = U[13];
    if (!(C > 0.0)) Un[14] = 0.0;
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) Q[v] = (Un[v] - U[v]) / dt;
    return 1;
}

// Q(U, dt) = (Phi_dt(U) - U) / dt by explicit sub-cycling with positivity
// scaling, complete evaporation / sublimation and the mu1 realisability clamp
// (or by the equilibrium model when selected).  Returns the number of sub-steps
// (0 when the cell is inactive).
__device__ inline int source_integrate(const double *U0, double dt, const SourceParams &sp, double *Q)
{
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) Q[v] = 0.0;
    if (!sp.enabled) return 0;
    if (sp.equilibrium) return source_equilibrium(U0, dt, sp, Q);
    CellThermo th;
    cell_thermo(U0, th);
    if (source_inactive(U0, th.T)) return 0;

    double U[NVAR];
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) U[v] = U0[v];
    Rates r;
    double S[NVAR];
    phase_rates(U, dt, sp, th, r);
    exchange(th, r.dM, r.dN, r.act, r.mdot_f, S);
    double tau = __builtin_huge_val();
    for (int c = 4; c <= 12; ++c)
        if (U[c] >= 0.0 && S[c] < 0.0) tau = fmin(tau, U[c] / (-S[c]));   // a negative component cannot be protected
    int nsub = 1;
    if (tau < __builtin_huge_val()) {
        double want = ceil(dt / (kSubSafety * tau));
        if (want > (double)sp.n_sub_max) nsub = sp.n_sub_max;
        else if (want > 1.0) nsub = (int)want;
    }
    const double h = dt / nsub;
    for (int s = 0; s < nsub; ++s) {
        if (s > 0) cell_thermo(U, th);
        phase_rates(U, h, sp, th, r);
        double act = r.act, mdf = r.mdot_f;
        bool el = false, es = false;
        // evaporation alone (the growth term of mu3, not the freezing sink) empties the
        // droplets within the sub-step
        if (r.gone_l || (r.Gl < 0.0 && U[8] + h * (3.0 * U[7] * r.Gl) <= 0.0)) {
            el = true;
            #pragma unroll
            for (int k = 0; k < 4; ++k) {
                r.dM[k] = -U[5 + k] / h;
                r.dN[k] = k ? k * U[8 + k] * r.Gs : 0.0;
            }
            mdf = 0.0;
            act = -U[14] / h;
        }
        if (r.gone_s || (r.Gs < 0.0 && U[12] + h * r.dN[3] <= 0.0)) {
            es = true;
            #pragma unroll
            for (int k = 0; k < 4; ++k) r.dN[k] = -U[9 + k] / h;
        }
        exchange(th, r.dM, r.dN, act, mdf, S);
        // positivity scaling; components of an evaporating population reach zero at
        // theta = 1 exactly and do not take part
        // the component that sets theta < 1 (the first of equals) is set to zero
        // exactly, not left at the rounding residue of its update
        double theta = 1.0;
        int cz = -1;
        for (int c = 4; c <= 12; ++c) {
            const bool skip = (el && c >= 5 && c <= 8) || (es && c >= 9);
            if (!skip && U[c] >= 0.0 && S[c] < 0.0) {
                const double t = U[c] / (-h * S[c]);
                if (t < theta) { theta = t; cz = c; }
            }
        }
        #pragma unroll
        for (int v = 0; v < NVAR; ++v) U[v] = v == cz ? 0.0 : U[v] + theta * h * S[v];
        if (theta == 1.0) {
            if (el) { U[5] = U[6] = U[7] = U[8] = 0.0; U[14] = 0.0; }
            if (es) { U[9] = U[10] = U[11] = U[12] = 0.0; }
        }
        #pragma unroll
        for (int b = 5; b <= 9; b += 4) {
            if (pop_valid(U[b], U[b + 2], U[b + 3])) {
                // Hoelder interval for mu1; an empty interval collapses to its upper end
                double hi = sqrt(U[b] * U[b + 2]);
                double lo = fmin(U[b + 2] * U[b + 2] / U[b + 3], hi);
                U[b + 1] = fmin(fmax(U[b + 1], lo), hi);
            }
        }
    }
    const double idt = 1.0 / dt;
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) Q[v] = (U[v] - U0[v]) * idt;
    return nsub;
}


// Components whose depletion bounds the sub-step and the positivity scaling:
// vapour, liquid and ice moments.
__device__ __forceinline__ constexpr bool depletable(int c) { return (c >= 4 && c <= 12) || (c >= 15 && c <= 18); }

// The same integration with two liquid populations (NV = NVAR_BI): each population
// has its own complete-evaporation rule, positivity exclusion and mu1 clamp; the
// crystals keep the freezing of a population that survives the sub-step.
template <int NV>
__device__ inline int source_integrate_n(const double *U0, double dt, const SourceParams &sp, double *Q)
{
    constexpr int NP = NV == NVAR_BI ? 2 : 1;
    #pragma unroll
    for (int v = 0; v < NV; ++v) Q[v] = 0.0;
    if (!sp.enabled) return 0;
    CellThermo th;
    cell_thermo(U0, th);
    if (source_inactive<NV>(U0, th.T)) return 0;

    double U[NV];
    #pragma unroll
    for (int v = 0; v < NV; ++v) U[v] = U0[v];
    RatesN<NP> r;
    double S[NV];
    phase_rates_n<NP>(U, dt, sp, th, r);
    exchange_n<NP>(th, r.dM, r.dN, r.act, r.mdot_f, S);
    double tau = __builtin_huge_val();
    #pragma unroll
    for (int c = 4; c < NV; ++c)
        if (depletable(c) && U[c] >= 0.0 && S[c] < 0.0) tau = fmin(tau, U[c] / (-S[c]));
    int nsub = 1;
    if (tau < __builtin_huge_val()) {
        double want = ceil(dt / (kSubSafety * tau));
        if (want > (double)sp.n_sub_max) nsub = sp.n_sub_max;
        else if (want > 1.0) nsub = (int)want;
    }
    const double h = dt / nsub;
    for (int s = 0; s < nsub; ++s) {
        if (s > 0) cell_thermo(U, th);
        phase_rates_n<NP>(U, h, sp, th, r);
        double act = r.act, mdf = r.mdot_f;
        bool el[NP], es = false, any_el = false;
        #pragma unroll
        for (int pop = 0; pop < NP; ++pop) {
            const int b = liq_base(pop);
            el[pop] = r.gone_l[pop] || (r.Gl[pop] < 0.0 && U[b + 3] + h * (3.0 * U[b + 2] * r.Gl[pop]) <= 0.0);
            if (el[pop]) {
                // evaporation alone (the growth term of mu3, not the freezing sink)
                // empties the population within the sub-step: none of it freezes;
                // soot-activated droplets release their soot
                #pragma unroll
                for (int k = 0; k < 4; ++k) r.dM[pop][k] = -U[b + k] / h;
                if (pop == 0) act = -U[14] / h;
                any_el = true;
            }
        }
        if (any_el) {
            // the crystals keep their growth and the freezing of a surviving population
            mdf = 0.0;
            #pragma unroll
            for (int k = 0; k < 4; ++k) r.dN[k] = k ? k * U[8 + k] * r.Gs : 0.0;
            if constexpr (NP == 2) {   // with one population nothing survives
                #pragma unroll
                for (int pop = 0; pop < NP; ++pop) {
                    if (el[pop]) continue;
                    #pragma unroll
                    for (int k = 0; k < 4; ++k) r.dN[k] += sp.ice_ratio[k] * r.F[pop][k];
                    mdf += kRhoL * kFourThirdsPi * r.F[pop][3];
                }
            }
        }
        if (r.gone_s || (r.Gs < 0.0 && U[12] + h * r.dN[3] <= 0.0)) {
            es = true;
            #pragma unroll
            for (int k = 0; k < 4; ++k) r.dN[k] = -U[9 + k] / h;
        }
        exchange_n<NP>(th, r.dM, r.dN, act, mdf, S);
        // positivity scaling; components of an evaporating population reach zero at
        // theta = 1 exactly and do not take part
        double theta = 1.0;
        int cz = -1;
        #pragma unroll
        for (int c = 4; c < NV; ++c) {
            if (!depletable(c)) continue;
            bool skip = (el[0] && c >= 5 && c <= 8) || (es && c >= 9 && c <= 12);
            if constexpr (NP == 2) skip = skip || (el[1] && c >= 15);
            if (!skip && U[c] >= 0.0 && S[c] < 0.0) {
                const double t = U[c] / (-h * S[c]);
                if (t < theta) { theta = t; cz = c; }
            }
        }
        #pragma unroll
        for (int v = 0; v < NV; ++v) U[v] = v == cz ? 0.0 : U[v] + theta * h * S[v];
        if (theta == 1.0) {
            if (el[0]) { U[5] = U[6] = U[7] = U[8] = 0.0; U[14] = 0.0; }
            if constexpr (NP == 2)
                if (el[1]) { U[15] = U[16] = U[17] = U[18] = 0.0; }
            if (es) { U[9] = U[10] = U[11] = U[12] = 0.0; }
        }
        #pragma unroll
        for (int set = 0; set < NP + 1; ++set) {
            const int b = set == 0 ? 5 : (set == 1 ? 9 : 15);
            if (pop_valid(U[b], U[b + 2], U[b + 3])) {
                // Hoelder interval for mu1; an empty interval collapses to its upper end
                double hi = sqrt(U[b] * U[b + 2]);
                double lo = fmin(U[b + 2] * U[b + 2] / U[b + 3], hi);
                U[b + 1] = fmin(fmax(U[b + 1], lo), hi);
            }
        }
    }
    const double idt = 1.0 / dt;
    #pragma unroll
    for (int v = 0; v < NV; ++v) Q[v] = (U[v] - U0[v]) * idt;
    return nsub;
}

// Q(U, dt) for NV variables per cell: NVAR (one liquid population) or NVAR_BI (two).
template <int NV> __device__ __forceinline__ int source_integrate_nv(const double *U0, double dt,
                                                                      const SourceParams &sp, double *Q)
{
    if constexpr (NV == NVAR) return source_integrate(U0, dt, sp, Q);
    else return source_integrate_n<NV>(U0, dt, sp, Q);
}

// ======================================================================
//  Fluxes (Sec. 3.2), templated arithmetic
// ======================================================================
template <class R> __device__ __forceinline__ R van_leer(R a, R b)
{
    return (a * b > R(0)) ? R(2) * a * b / (a + b) : R(0);
}

// c = sqrt(c^2), 1 / c and 1 / c^2: in FP32 from one reciprocal square root
__device__ __forceinline__ void sound_speed(float c2, float &c, float &ic, float &ic2)
{
    ic = __builtin_amdgcn_rsqf(c2);
    c = c2 * ic;
    ic2 = ic * ic;
}
__device__ __forceinline__ void sound_speed(double c2, double &c, double &ic, double &ic2)
{
    c = sqrt(c2);
    ic2 = tdiv(1.0, c2);
    ic = c * ic2;
}

// Roe flux on (rho, rho u_n, rho u_t, rho E) of the two-species gas in primitive-
// jump form with Harten's entropy fix on the acoustic waves.  q = (rho, u_n, u_t,
// p, Y).  F[0..3] mass, normal and tangential momentum (less pref), energy.
template <class R> __device__ __forceinline__ void roe_flux(const R *qL, const R *qR, R pref, R *F)
{
    const R rl = qL[0], unl = qL[1], utl = qL[2], pl = qL[3], Yl = qL[4];
    const R rr = qR[0], unr = qR[1], utr = qR[2], pr = qR[3], Yr = qR[4];
    const R Hl = gas_cp(Yl) * tdiv(pl, rl * gas_R(Yl)) + gas_h0(Yl) + R(0.5) * (unl * unl + utl * utl);
    const R Hr = gas_cp(Yr) * tdiv(pr, rr * gas_R(Yr)) + gas_h0(Yr) + R(0.5) * (unr * unr + utr * utr);
    const R ml = rl * unl, mr = rr * unr;

    const R sl = fsqrt(rl), sr = fsqrt(rr);
    const R isum = tdiv(R(1), sl + sr);
    const R wl = sl * isum, wr = sr * isum;
    const R rho = sl * sr;
    const R un = wl * unl + wr * unr;
    const R ut = wl * utl + wr * utr;
    const R H = wl * Hl + wr * Hr;
    const R Y = wl * Yl + wr * Yr;
    const R q2 = un * un + ut * ut;
    const R Rm = gas_R(Y);
    const R h0 = gas_h0(Y);
    // c^2 = gamma R T with T = (H - q^2/2 - h0) / c_p and gamma = c_p / c_v
    const R c2 = Rm * tdiv(H - R(0.5) * q2 - h0, gas_cv(Y));
    R c, ic, ic2;
    sound_speed(c2, c, ic, ic2);

    const R dr = rr - rl, dun = unr - unl, dut = utr - utl, dp = pr - pl;
    const R i2c2 = R(0.5) * ic2;
    const R a1 = (dp - rho * c * dun) * i2c2;
    const R a2 = dr - dp * ic2;
    const R a3 = rho * dut;
    const R a4 = (dp + rho * c * dun) * i2c2;
    R l1 = fabs(un - c), l4 = fabs(un + c);
    const R l2 = fabs(un);
    // Harten's fix within del = c / 10: l -> (l^2 + del^2) / (2 del), with 1 / (2 del) = 5 / c
    const R del = R(0.1) * c, i2del = R(5) * ic;
    if (l1 < del) l1 = (l1 * l1 + del * del) * i2del;
    if (l4 < del) l4 = (l4 * l4 + del * del) * i2del;
    const R w1 = l1 * a1, w2 = l2 * a2, w3 = l2 * a3, w4 = l4 * a4;
    // eigenvectors: (1, un-c, ut, H-un c), (1, un, ut, q2/2 + h0), (0, 0, 1, ut), (1, un+c, ut, H+un c)
    F[0] = R(0.5) * (ml + mr) - R(0.5) * (w1 + w2 + w4);
    // a uniform reference pressure exerts no net force on a closed cell: it is taken
    // out of the momentum flux (and out of the axisymmetric pressure source), which
    // keeps the FP32 path free of cancellation between large pressure terms
    F[1] = R(0.5) * (ml * unl + (pl - pref) + mr * unr + (pr - pref)) - R(0.5) * (w1 * (un - c) + w2 * un + w4 * (un + c));
    F[2] = R(0.5) * (ml * utl + mr * utr) - R(0.5) * ((w1 + w2 + w4) * ut + w3);
    F[3] = R(0.5) * (ml * Hl + mr * Hr)
           - R(0.5) * (w1 * (H - un * c) + w2 * (R(0.5) * q2 + h0) + w3 * ut + w4 * (H + un * c));
}

}  // namespace cp
