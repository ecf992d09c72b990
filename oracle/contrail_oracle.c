/*
 * contrail_oracle.c -- plain, slow, FP64 CPU oracle for the explicit finite-volume
 * step of the non-equilibrium contrail-formation solver (Tegethoff & Wheeler,
 * "Non-Equilibrium Phase Changes in Aircraft Exhaust", arXiv 2504.20742).
 *
 * THIS FILE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  The product (the HIP library) shares
 * no code, header, table or constant generator with it.
 *
 * It follows the paper section by section:
 *   Sec. 2.2, Eq. 1          saturation ratio S and subcooling dT
 *   Sec. 2.2, Eq. 2-3        CNT barrier, critical radius
 *   Sec. 2.2, Eq. 4-7        homogeneous nucleation rate, Kantrowitz correction
 *   Sec. 2.2, Eq. 8-11       heterogeneous (soot) nucleation, contact-angle factor
 *   Sec. 2.2, Eq. 12-13      homogeneous freezing (Koop water-activity rate)
 *   Sec. 2.2, Eq. 14-15      immersion freezing (active-site density)
 *   Sec. 2.2, Eq. 16-18      Young's growth law, wetness evolution
 *   Sec. 2.2, Eq. 19-21      radius moments with the r20 closure
 *   Sec. 3.1, Eq. 22-26      conservation laws, drag, species and moment transport
 *   Sec. 3.2                 Roe-type flux + MUSCL / van Leer, central viscous
 *                            fluxes, explicit Runge-Kutta with a global CFL, source
 *                            evaluated explicitly per cell.
 * Readings where the paper is silent are documented beside the code that takes
 * them (and in the design notes of the repository).
 *
 * Parity unpinned (nothing but the paper's own statement to check them against):
 * the immersion-freezing time scale k_imm (Eq. 14-15 carry no time unit) and the
 * Kantrowitz bracket of Eq. 5 beyond its classical form.  Every other part is pinned
 * in the tests against closed forms, exact solutions, quadrature, invariants or
 * published values.
 *
 * Build:  gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC  (no fast-math).
 * Every per-cell result is independent of the thread count.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* Per-cell arrays hold NV entries: the 15 variables of the state, and four more
 * (15..18) for the homogeneously nucleated droplets when the liquid is carried as
 * two populations (Sec. 2.2); unused entries stay zero.  Arrays in memory hold
 * cx->nv planes (15 or 19).                                                    */
#define NV 19
#define NV_BASE 15

/* ---------------------------------------------------------------- constants -- */
/* Ideal-gas two-species carrier (dry air pseudo-component + water vapour),
 * reference temperature 273.15 K for the caloric laws.                          */
static const double T_REF = 273.15;
static const double RGAS_AIR = 287.0;            /* 78/21/1 % N2/O2/Ar, Sec. 4.1  */
static const double CP_AIR = 1004.5;             /* 3.5 R, diatomic              */
static const double RGAS_VAP = 461.52;
static const double CP_VAP = 1846.08;            /* 4 R, triatomic               */
static const double GAMMA_VAP = 4.0 / 3.0;
static const double C_LIQ = 4218.0, C_ICE = 2106.0;
static const double L_VAP0 = 2.5008e6;           /* h_fg at 273.15 K             */
static const double L_SUB0 = 2.8345e6;           /* h_sg at 273.15 K             */
static const double RHO_LIQ = 1000.0, RHO_ICE = 917.0;
static const double BOLTZMANN = 1.380649e-23;
static const double AVOGADRO = 6.02214076e23;
static const double MOLAR_W = 0.018015268;
static const double PRANDTL = 0.71, PRANDTL_T = 0.9, PRANDTL_V = 1.0;
static const double SCHMIDT_T = 0.7;             /* Sec. 3.1                     */
static const double SUTH_MU0 = 1.716e-5, SUTH_S = 110.4;
static const double DIFF_V0 = 2.11e-5, DIFF_V_EXP = 1.94, DIFF_P0 = 101325.0;
static const double COND_COEF = 1.0;             /* q_c                          */
static const double YOUNG_ALPHA = 11.0;          /* Sec. 2.2 growth kinetics      */
static const double N_MIN = 1.0;                 /* number floor [1/m^3]         */
static const double SUB_SAFETY = 0.2;            /* sub-step / depletion time     */
/* Pa, floor of p_v in ln S: below the ice saturation pressure at 150 K (6e-6 Pa),
 * the cold end of the property range, so a cell without vapour is subsaturated. */
static const double PV_FLOOR = 1.0e-9;
static const double R_MIN = 1.0e-10;             /* m: smaller r20 = evaporated   */
static const double PI = 3.14159265358979323846;

/* --------------------------------------------------------- public structs -- */
/* Layout of these two structs is part of the oracle's own interface.            */
typedef struct {
    int nx, nr;
    double Lx, Lr;
    double sx_ratio;     /* ratio of successive axial widths (1 = uniform)        */
    double r_cluster;    /* radius the radial cells cluster about (<=0: uniform)  */
    double beta_r;       /* clustering strength                                   */
    int geom;            /* 0 axisymmetric, 1 planar, 2 quasi-1D duct (nr = 1)    */
    int bc_xlo, bc_xhi, bc_rlo, bc_rhi;  /* 0 inflow,1 copy,2 wall,3 far field    */
} or_mesh;

typedef struct {
    double p_amb, T_amb, RH_ice, mach_amb;
    double R_core, u_core, T_core, Y_core;
    double R_fan, u_byp, T_byp, Y_byp;   /* Y_byp < 0: bypass carries ambient Y     */
    double n_soot, r_g_soot, sigma_g_soot;
    double cfl;
    double theta_deg;    /* soot contact angle                                    */
    double n_s;          /* active-site density for immersion freezing [1/m^2]    */
    double k_imm;        /* immersion-freezing rate scale [1/s]                   */
    double kappa_m, s_delta, delta0_frac;  /* mixing-length eddy viscosity        */
    int n_sub_max;
    int phase_change;
    int pad0, pad1;
} or_case;

enum { BC_INFLOW = 0, BC_COPY = 1, BC_WALL = 2, BC_FARFIELD = 3 };
enum { GEOM_AXI = 0, GEOM_PLANAR = 1, GEOM_Q1D = 2 };

typedef struct {
    or_mesh m;
    or_case c;
    int nx, nr;
    double *xf, *rf, *xc, *rc, *dx, *dr;
    double *ax;                 /* quasi-1D: duct area at the nx+1 x faces         */
    double *inflow;             /* nr x NV: Dirichlet inflow state by row          */
    double ambient[NV];
    double Y_amb, u_amb;
    double f_theta;             /* Eq. 9 at the case's contact angle               */
    double soot_area;           /* 4 pi r_g^2 exp(2 ln^2 sigma_g) per particle     */
    double delta0;
    int equilibrium;            /* 1: equilibrium phase change instead of kinetics */
    int drift;                  /* 1: droplets and crystals drift against the gas  */
    int bimodal;                /* 1: two liquid populations (soot-activated in 5..8,
                                 *    homogeneously nucleated in 15..18)           */
    int nv;                     /* variables per cell in memory: 15, or 19 bimodal */
    double *ptab;               /* water property table (null: closed forms)       */
    int ptab_n;
    double ptab_T0, ptab_h;
} or_ctx;

/* ================================================================ Sec. 2.2 == */
/* Sonntag saturation pressures (the paper's choice below the triple point),
 * natural log of the pressure in Pa.                                            */
double or_ln_psat_liq(double T)
{
    return -6096.9385 / T + 16.635794 - 2.711193e-2 * T + 1.673952e-5 * T * T
           + 2.433502 * log(T) + log(100.0);
}

double or_ln_psat_ice(double T)
{
    return -6024.5282 / T + 24.7219 + 1.0613868e-2 * T - 1.3198825e-5 * T * T
           - 0.49382577 * log(T) + log(100.0);
}

/* Saturation temperature at vapour pressure pv: Newton on x = 1/T of
 * ln p_sat(1/x) = ln pv, 4 steps from the local gas temperature.                */
static double tsat_newton(int ice, double lnpv, double T_start)
{
    double a, b, c, d, e;
    if (ice) { a = -6024.5282; b = 24.7219; c = 1.0613868e-2; d = -1.3198825e-5; e = -0.49382577; }
    else     { a = -6096.9385; b = 16.635794; c = -2.711193e-2; d = 1.673952e-5; e = 2.433502; }
    double x = 1.0 / T_start;
    for (int it = 0; it < 4; ++it) {
        /* ln p(x) = a x + b + c/x + d/x^2 - e ln x + ln 100 */
        double f = a * x + b + c / x + d / (x * x) - e * log(x) + log(100.0) - lnpv;
        double fp = a - c / (x * x) - 2.0 * d / (x * x * x) - e / x;
        x = x - f / fp;
    }
    return 1.0 / x;
}

double or_tsat_liq(double pv, double T_start) { return tsat_newton(0, log(pv), T_start); }
double or_tsat_ice(double pv, double T_start) { return tsat_newton(1, log(pv), T_start); }

/* IAPWS (1994) surface tension of water, extrapolated below 273.15 K; it vanishes
 * at the critical point and stays zero above it (no liquid surface there).      */
double or_sigma_lg(double T)
{
    double tau = 1.0 - T / 647.096;
    if (!(tau > 0.0)) return 0.0;
    return 0.2358 * pow(tau, 1.256) * (1.0 - 0.625 * tau);
}

/* ======================================= tabulated water properties (Sec. 3.2) == */
/* The paper tabulates the water properties before the run and interpolates them
 * with a second-order Taylor expansion.  Here: nodes T_k = T0 + k h on [150, 700] K
 * holding f, f' and f''/2 of ln p_sat over liquid, ln p_sat over ice and the
 * surface tension, from their closed forms and analytic derivatives; a lookup
 * expands about the nearest node (outside the range, about the end node).        */
enum { PT_LNPW = 0, PT_LNPI = 1, PT_SIGMA = 2, PT_NPROP = 3 };
static const double PT_T0 = 150.0, PT_T1 = 700.0;

static void sonntag_derivs(int ice, double T, double *f)
{
    double a, c, d, e;
    if (ice) { a = -6024.5282; c = 1.0613868e-2; d = -1.3198825e-5; e = -0.49382577; }
    else     { a = -6096.9385; c = -2.711193e-2; d = 1.673952e-5; e = 2.433502; }
    f[0] = ice ? or_ln_psat_ice(T) : or_ln_psat_liq(T);
    f[1] = -a / (T * T) + c + 2.0 * d * T + e / T;
    f[2] = 0.5 * (2.0 * a / (T * T * T) + 2.0 * d - e / (T * T));
}

static void sigma_derivs(double T, double *f)
{
    /* sigma = B (tau^m - 0.625 tau^(m+1)), tau = 1 - T/Tc */
    const double B = 0.2358, m = 1.256, Tc = 647.096;
    double tau = 1.0 - T / Tc;
    if (!(tau > 0.0)) {   /* no surface tension at and above the critical point */
        f[0] = f[1] = f[2] = 0.0;
        return;
    }
    double s1 = B * (m * pow(tau, m - 1.0) - 0.625 * (m + 1.0) * pow(tau, m));
    double s2 = B * (m * (m - 1.0) * pow(tau, m - 2.0) - 0.625 * (m + 1.0) * m * pow(tau, m - 1.0));
    f[0] = or_sigma_lg(T);
    f[1] = -s1 / Tc;
    f[2] = 0.5 * s2 / (Tc * Tc);
}

int or_set_property_table(or_ctx *cx, double h)
{
    free(cx->ptab);
    cx->ptab = NULL;
    cx->ptab_n = 0;
    if (h == 0.0) return 0;
    if (!(h > 0.0) || (PT_T1 - PT_T0) / h > 1.0e6) return -1;
    int n = (int)floor((PT_T1 - PT_T0) / h) + 1;
    cx->ptab = malloc(sizeof(double) * 3 * PT_NPROP * n);
    cx->ptab_n = n;
    cx->ptab_T0 = PT_T0;
    cx->ptab_h = h;
    for (int k = 0; k < n; ++k) {
        double T = PT_T0 + k * h;
        double *row = cx->ptab + 3 * PT_NPROP * k;
        sonntag_derivs(0, T, row + 3 * PT_LNPW);
        sonntag_derivs(1, T, row + 3 * PT_LNPI);
        sigma_derivs(T, row + 3 * PT_SIGMA);
    }
    return 0;
}

/* Taylor expansion of property q about the node nearest T; *dfdT its slope.       */
static double ptab_eval(const or_ctx *cx, int q, double T, double *dfdT)
{
    double u = (T - cx->ptab_T0) / cx->ptab_h;
    int k = (int)floor(u + 0.5);
    if (k < 0) k = 0;
    if (k > cx->ptab_n - 1) k = cx->ptab_n - 1;
    const double *c = cx->ptab + 3 * PT_NPROP * k + 3 * q;
    double d = T - (cx->ptab_T0 + k * cx->ptab_h);
    if (dfdT) *dfdT = c[1] + 2.0 * c[2] * d;
    return c[0] + d * (c[1] + d * c[2]);
}

/* The water properties the phase change reads: the table when one is set, else
 * the closed forms.                                                               */
static double prop_lnp(const or_ctx *cx, int ice, double T)
{
    if (cx->ptab) return ptab_eval(cx, ice ? PT_LNPI : PT_LNPW, T, NULL);
    return ice ? or_ln_psat_ice(T) : or_ln_psat_liq(T);
}

static double prop_sigma(const or_ctx *cx, double T)
{
    if (cx->ptab) return ptab_eval(cx, PT_SIGMA, T, NULL);
    return or_sigma_lg(T);
}

/* Saturation temperature at ln p_v: four Newton steps in x = 1/T from the gas
 * temperature, or from 373.15 K in hotter gas (the upper end of the Sonntag fits:
 * beyond it the extrapolated ln p_sat bends and the steps can settle on a spurious
 * root above the gas temperature); with a table on the expanded ln p_sat, whose
 * slope in x is -T^2 d(ln p_sat)/dT.                                              */
static const double T_SAT_START_MAX = 373.15;
static double prop_tsat(const or_ctx *cx, int ice, double lnpv, double T_start)
{
    if (T_start > T_SAT_START_MAX) T_start = T_SAT_START_MAX;
    if (!cx->ptab) return tsat_newton(ice, lnpv, T_start);
    double x = 1.0 / T_start;
    for (int it = 0; it < 4; ++it) {
        double T = 1.0 / x, g;
        double f = ptab_eval(cx, ice ? PT_LNPI : PT_LNPW, T, &g) - lnpv;
        x = x - f / (-T * T * g);
    }
    return 1.0 / x;
}

/* Property q (0 ln p_sat liquid, 1 ln p_sat ice, 2 surface tension) as the phase
 * change reads it, and the saturation temperature over liquid (ice = 0) or ice.  */
double or_property(const or_ctx *cx, int q, double T)
{
    return q == PT_SIGMA ? prop_sigma(cx, T) : prop_lnp(cx, q == PT_LNPI, T);
}

double or_property_tsat(const or_ctx *cx, int ice, double lnpv, double T_start)
{
    return prop_tsat(cx, ice, lnpv, T_start);
}

static double latent_vap(double T) { return L_VAP0 + (CP_VAP - C_LIQ) * (T - T_REF); }
static double latent_sub(double T) { return L_SUB0 + (CP_VAP - C_ICE) * (T - T_REF); }

double or_mu_sutherland(double T)
{
    double t = T / T_REF;
    return SUTH_MU0 * t * sqrt(t) * (T_REF + SUTH_S) / (T + SUTH_S);
}

/* Eq. 2: Gibbs energy of a cluster of radius r; (g_l - g_g) = -R_s T ln S.      */
double or_gibbs_cluster(double r, double T, double lnS, double sigma)
{
    return -4.0 / 3.0 * PI * r * r * r * RHO_LIQ * RGAS_VAP * T * lnS
           + 4.0 * PI * r * r * sigma;
}

/* Eq. 3: critical radius and barrier.                                          */
double or_critical_radius(double sigma, double T, double lnS)
{
    return 2.0 * sigma / (RHO_LIQ * RGAS_VAP * T * lnS);
}

double or_barrier_hom(double sigma, double rcrit)
{
    return 4.0 / 3.0 * PI * sigma * rcrit * rcrit;
}

/* Eq. 4 prefactor q_c sqrt(2 sigma N_A^3 / (pi M^3)) rho_v^2 / rho_l.            */
double or_cnt_prefactor(double sigma, double rho_v)
{
    return COND_COEF * sqrt(2.0 * sigma * AVOGADRO * AVOGADRO * AVOGADRO
                            / (PI * MOLAR_W * MOLAR_W * MOLAR_W))
           * rho_v * rho_v / RHO_LIQ;
}

/* Eq. 5, Kantrowitz correction with the free-molecular heat-transfer coefficient
 * alpha_crit = rho_g sqrt(R T / 2 pi) c_p,v (gamma+1)/(2 gamma): rho_g and the
 * thermal-speed factor cancel against the printed prefactor.                    */
double or_kantrowitz_phi(double T, double hfg)
{
    double pref = COND_COEF * 2.0 * GAMMA_VAP / ((GAMMA_VAP + 1.0) * CP_VAP);
    return pref * (hfg * hfg / (RGAS_VAP * T * T) - hfg / T);
}

/* Eq. 9 contact-angle factor.                                                   */
double or_contact_factor(double theta_rad)
{
    double c = cos(theta_rad);
    return 0.25 * (2.0 + c) * (1.0 - c) * (1.0 - c);
}

/* Eq. 12: homogeneous freezing rate of Koop et al. (2000), the water-activity
 * polynomial, converted from cm^-3 s^-1 to m^-3 s^-1.  Pure water droplets
 * (a_w = 1), so Delta a_w = 1 - p_sat,ice/p_sat,liq, clamped to the fit range.  */
static double koop_clamp(double d)
{
    if (d < 0.26) d = 0.26;
    if (d > 0.34) d = 0.34;
    return d;
}

double or_koop_delta_aw(double T)
{
    return koop_clamp(1.0 - exp(or_ln_psat_ice(T) - or_ln_psat_liq(T)));
}

double or_koop_rate(double daw)
{
    double lg = -906.7 + 8502.0 * daw - 26924.0 * daw * daw + 29180.0 * daw * daw * daw;
    return 1.0e6 * pow(10.0, lg);
}

/* Eq. 16 auxiliary parameter nu of Young's growth law.                           */
double or_young_nu(double Tsat, double h)
{
    return RGAS_VAP * Tsat / h
           * (YOUNG_ALPHA - 0.5 - (2.0 - COND_COEF) / (2.0 * COND_COEF)
              * (GAMMA_VAP + 1.0) / (2.0 * GAMMA_VAP) * CP_VAP * Tsat / h);
}

/* Eq. 16 with beta = 0: G = lambda dT_K / (rho_p h r (1 + 3.78 (1-nu) Kn/Pr)),
 * Kn = lbar / (2 r).  drive = dT (1 - r_crit/r) for droplets, dT for ice.         */
double or_young_growth(double lambda_g, double drive, double r, double rho_p,
                       double h, double nu, double lbar)
{
    double Kn = lbar / (2.0 * r);
    return lambda_g * drive / (rho_p * h * r * (1.0 + 3.78 * (1.0 - nu) * Kn / PRANDTL_V));
}

/* Eq. 24: Schiller-Naumann drag with the Cunningham slip correction.            */
double or_cunningham_ac(double Kn) { return 1.257 + 0.4 * exp(-1.1 / (2.0 * Kn)); }

double or_drag_cd(double Re, double Kn)
{
    return 24.0 / Re * (1.0 + 0.15 * pow(Re, 0.687)) / (1.0 + 2.0 * or_cunningham_ac(Kn) * Kn);
}

/* ------------------------------------------------------ gas thermodynamics -- */
static double mix_R(double Y) { return (1.0 - Y) * RGAS_AIR + Y * RGAS_VAP; }
static double mix_cp(double Y) { return (1.0 - Y) * CP_AIR + Y * CP_VAP; }
static double mix_cv(double Y) { return (1.0 - Y) * (CP_AIR - RGAS_AIR) + Y * (CP_VAP - RGAS_VAP); }
/* enthalpy offset: h = cp_mix T + h0(Y) with h_a = cp_a (T-Tref), h_v = L0 + cp_v (T-Tref) */
static double mix_h0(double Y) { return -(1.0 - Y) * CP_AIR * T_REF + Y * (L_VAP0 - CP_VAP * T_REF); }

/* Conserved -> primitive state (Eq. 23).                                         */
typedef struct {
    double rho, u, v, p, T, Y, c, gam, R, cp, phi[NV];
} prim_t;

static void cons_to_prim(const double *U, prim_t *w)
{
    w->rho = U[0];
    w->u = U[1] / U[0];
    w->v = U[2] / U[0];
    w->Y = U[4] / U[0];
    double e = U[3] / U[0] - 0.5 * (w->u * w->u + w->v * w->v);
    double Y = w->Y;
    w->T = (e + (1.0 - Y) * CP_AIR * T_REF - Y * (L_VAP0 - CP_VAP * T_REF)) / mix_cv(Y);
    w->R = mix_R(Y);
    w->cp = mix_cp(Y);
    w->p = w->rho * w->R * w->T;
    w->gam = w->cp / mix_cv(Y);
    w->c = sqrt(w->gam * w->R * w->T);
    for (int m = 4; m < NV; ++m) w->phi[m] = U[m] / U[0];
}

/* Primitive (rho,u,v,p,Y, specific scalars) -> conserved.                        */
static void prim_to_cons(double rho, double u, double v, double p, double Y,
                         const double *phi /* NV, entries 5..14 used */, double *U)
{
    double T = p / (rho * mix_R(Y));
    double e = mix_cv(Y) * T - (1.0 - Y) * CP_AIR * T_REF + Y * (L_VAP0 - CP_VAP * T_REF);
    U[0] = rho;
    U[1] = rho * u;
    U[2] = rho * v;
    U[3] = rho * (e + 0.5 * (u * u + v * v));
    U[4] = rho * Y;
    for (int m = 5; m < NV; ++m) U[m] = rho * (phi ? phi[m] : 0.0);
}

void or_prim_to_cons(const double *W /* rho,u,v,p,Y,phi5..phi14 */, double *U /* 15 */)
{
    double phi[NV] = {0}, Ul[NV];
    for (int m = 5; m < NV_BASE; ++m) phi[m] = W[m];
    prim_to_cons(W[0], W[1], W[2], W[3], W[4], phi, Ul);
    memcpy(U, Ul, sizeof(double) * NV_BASE);
}

void or_cons_to_prim(const double *U /* 15 */, double *W /* rho,u,v,p,Y,phi5..14,T,c */)
{
    double Ul[NV] = {0};
    memcpy(Ul, U, sizeof(double) * NV_BASE);
    prim_t w;
    cons_to_prim(Ul, &w);
    W[0] = w.rho; W[1] = w.u; W[2] = w.v; W[3] = w.p; W[4] = w.Y;
    for (int m = 5; m < NV_BASE; ++m) W[m] = w.phi[m];
    W[15] = w.T; W[16] = w.c;
}

/* ================================================= source: rates (Eq. 1-21) == */
/* Liquid populations: 0 holds all droplets (one population), or the soot-activated
 * ones when the liquid is carried as two populations; 1 holds the homogeneously
 * nucleated droplets (Sec. 2.2: two moment sets evolved side by side, each with its
 * own nucleation source, growth closure and freezing).                           */
static int liq_base(int pop) { return pop ? 15 : 5; }

typedef struct {
    double dM[2][4], dN[4]; /* liquid moment rates per population / ice moment rates */
    double act;             /* soot activation rate                                 */
    double F[2][4];         /* moments each liquid population loses to freezing     */
    double mdot_f;          /* liquid -> ice mass rate                              */
    double Gl[2], Gs;       /* growth rates at r20                                  */
    double Jhom, Jhet, rcrit, lnSl, lnSi;
    int stale_l[2], stale_s;/* number left without mass: evaporated population      */
} rates_t;

/* A population with particles (mu0 > N_MIN) is valid while its mean radii
 * r20 = sqrt(mu2/mu0) and r30 = (mu3/mu0)^(1/3) are at least a molecular radius;
 * below that it has evaporated (its number has no mass left).                  */
static int population_valid(const double *m)
{
    return m[0] > N_MIN && m[2] > m[0] * R_MIN * R_MIN && m[3] > m[0] * R_MIN * R_MIN * R_MIN;
}

/* One evaluation of the phase-change rates at state U (NV entries); h is the
 * sub-step length, which bounds the activation rate so that at most the
 * unactivated soot activates.                                                    */
static void phase_change_rates(const or_ctx *cx, const double *U, double h, rates_t *r)
{
    memset(r, 0, sizeof(*r));
    prim_t w;
    cons_to_prim(U, &w);
    const double T = w.T;
    const double rho_v = U[4];
    const double *N = U + 9;
    const double Ns = U[13], Na = U[14];
    const int npop = cx->bimodal ? 2 : 1;

    /* Eq. 1: driving potentials */
    double pv = rho_v * RGAS_VAP * T;
    if (pv < PV_FLOOR) pv = PV_FLOOR;
    const double lnpv = log(pv);
    const double lnpw = prop_lnp(cx, 0, T), lnpi = prop_lnp(cx, 1, T);
    const double lnSl = lnpv - lnpw, lnSi = lnpv - lnpi;
    r->lnSl = lnSl; r->lnSi = lnSi;

    const double sigma = prop_sigma(cx, T);
    const double hfg = latent_vap(T), hsg = latent_sub(T);
    const double mu = or_mu_sutherland(T);
    const double lambda_g = w.cp * mu / PRANDTL;
    const double lbar = 1.5 * mu * sqrt(w.R * T) / w.p;

    /* Eq. 3-6, 8-11: nucleation (only for a supersaturated vapour).  J[pop] is the
     * number of new droplets of population pop per m^3 and s: all of them in one
     * population, or the soot-activated ones in 0 and the homogeneous ones in 1. */
    double J[2] = {0.0, 0.0};
    if (lnSl > 0.0 && rho_v > 0.0) {
        double rc = or_critical_radius(sigma, T, lnSl);
        double x = or_barrier_hom(sigma, rc) / (BOLTZMANN * T);
        double K = or_cnt_prefactor(sigma, rho_v);
        double phi = or_kantrowitz_phi(T, hfg);
        double Jhom = K * exp(-x) / (1.0 + phi);
        double act = 0.0;
        if (Ns > Na) {
            double Jhet = K * exp(-cx->f_theta * x) / (1.0 + phi);
            double cap = (Ns - Na) / h;
            act = Jhet < cap ? Jhet : cap;
            r->Jhet = Jhet;
        }
        r->Jhom = Jhom;
        r->rcrit = rc;
        r->act = act;
        if (npop == 1) J[0] = Jhom + act;
        else { J[0] = act; J[1] = Jhom; }
    }

    const int ice = population_valid(N);
    r->stale_s = (N[0] > N_MIN && !ice);
    double Jhom_s = 0.0, Jhet_s = 0.0;
    if (T < T_REF) {
        Jhom_s = or_koop_rate(koop_clamp(1.0 - exp(lnpi - lnpw)));
        Jhet_s = cx->c.k_imm * cx->c.n_s * Ns * cx->soot_area;
    }

    for (int pop = 0; pop < npop; ++pop) {
        const double *M = U + liq_base(pop);
        const int liquid = population_valid(M);
        r->stale_l[pop] = (M[0] > N_MIN && !liquid);
        /* Eq. 16, 21: droplet growth at r20 with the Kelvin factor (1 - r_crit/r) */
        if (liquid) {
            double r20 = sqrt(M[2] / M[0]);
            double Tsat = prop_tsat(cx, 0, lnpv, T);
            double dT = Tsat - T;
            double drive;
            if (fabs(lnSl) < 1e-12)
                drive = dT - 2.0 * sigma * Tsat / (RHO_LIQ * hfg * r20);
            else
                drive = dT * (1.0 - or_critical_radius(sigma, T, lnSl) / r20);
            double nu = or_young_nu(Tsat, hfg);
            r->Gl[pop] = or_young_growth(lambda_g, drive, r20, RHO_LIQ, hfg, nu, lbar);
        }
        /* Eq. 12-15: freezing of droplets; moments above mu3 from a lognormal
         * closure.  Immersion freezing needs a soot core: homogeneously nucleated
         * droplets freeze by the homogeneous (Koop) rate alone.                   */
        if (T < T_REF && liquid) {
            double l2 = log(M[2] / M[0]), l3 = log(M[3] / M[0]);
            double s2 = 2.0 / 3.0 * l3 - l2;
            if (s2 < 0.0) s2 = 0.0;
            double lnrg = 0.5 * l2 - s2;
            double Mh[7];
            Mh[3] = M[3];
            for (int n = 4; n <= 6; ++n) Mh[n] = M[0] * exp(n * lnrg + 0.5 * n * n * s2);
            double Jf = pop == 0 ? Jhom_s + Jhet_s : Jhom_s;
            for (int k = 0; k < 4; ++k) r->F[pop][k] = Jf * (4.0 / 3.0 * PI) * Mh[k + 3];
            r->mdot_f += RHO_LIQ * (4.0 / 3.0 * PI) * r->F[pop][3];
        }
        /* Eq. 21 moment sources of the population */
        double rk = 1.0;
        for (int k = 0; k < 4; ++k) {
            double grow_l = k > 0 ? k * M[k - 1] * r->Gl[pop] : 0.0;
            r->dM[pop][k] = grow_l + J[pop] * rk - r->F[pop][k];
            rk *= r->rcrit;
        }
    }
    /* ice crystals grow analogously with ice properties, no Kelvin factor */
    if (ice) {
        double r20 = sqrt(N[2] / N[0]);
        double Tsat = prop_tsat(cx, 1, lnpv, T);
        double dT = Tsat - T;
        double nu = or_young_nu(Tsat, hsg);
        r->Gs = or_young_growth(lambda_g, dT, r20, RHO_ICE, hsg, nu, lbar);
    }
    /* frozen droplets join the crystals with radius r (rho_l/rho_s)^(1/3) */
    for (int k = 0; k < 4; ++k) {
        double grow_s = k > 0 ? k * N[k - 1] * r->Gs : 0.0;
        double Ft = r->F[0][k];
        if (npop == 2) Ft += r->F[1][k];
        r->dN[k] = grow_s + pow(RHO_LIQ / RHO_ICE, k / 3.0) * Ft;
    }
}

/* Eq. 22-26 source vector from moment rates: vapour sink keeps total water exact,
 * the gas carries the vapour's momentum, latent heats go to the gas.            */
static void exchange_terms(const double *U, const double (*dM)[4], const double *dN, int npop,
                           double act, double mdot_f, double *S)
{
    prim_t w;
    cons_to_prim(U, &w);
    const double T = w.T;
    for (int k = 0; k < 4; ++k) {
        S[5 + k] = dM[0][k];
        S[9 + k] = dN[k];
        S[15 + k] = npop == 2 ? dM[1][k] : 0.0;
    }
    S[13] = 0.0;
    S[14] = act;
    const double fpi = 4.0 / 3.0 * PI;
    double liq3 = S[8];
    if (npop == 2) liq3 += S[18];
    S[4] = -fpi * (RHO_LIQ * liq3 + RHO_ICE * S[12]);
    S[0] = S[4];
    S[1] = S[4] * w.u;
    S[2] = S[4] * w.v;
    double mdot_l = fpi * RHO_LIQ * liq3 + mdot_f;
    double mdot_s = fpi * RHO_ICE * S[12] - mdot_f;
    double hv = L_VAP0 + CP_VAP * (T - T_REF);
    double hl = hv - latent_vap(T), hi = hv - latent_sub(T);
    double ke = 0.5 * (w.u * w.u + w.v * w.v);
    S[3] = -mdot_l * (hl + ke) - mdot_s * (hi + ke) + mdot_f * (latent_sub(T) - latent_vap(T));
}

/* Instantaneous source S(U) (no sub-cycling), for pins.  U and S hold cx->nv
 * entries.                                                                       */
void or_source_rates_cell(const or_ctx *cx, const double *Uin, double h, double *Sout, double *diag)
{
    double U[NV] = {0}, S[NV];
    memcpy(U, Uin, sizeof(double) * cx->nv);
    rates_t r;
    phase_change_rates(cx, U, h, &r);
    exchange_terms(U, (const double(*)[4])r.dM, r.dN, cx->bimodal ? 2 : 1, r.act, r.mdot_f, S);
    memcpy(Sout, S, sizeof(double) * cx->nv);
    if (diag) {
        diag[0] = r.Gl[0]; diag[1] = r.Gs; diag[2] = r.Jhom; diag[3] = r.Jhet;
        diag[4] = r.rcrit; diag[5] = r.lnSl; diag[6] = r.lnSi; diag[7] = r.mdot_f;
    }
}

/* The equilibrium comparison model's rule for a cell without condensate: it
 * changes only once it is supersaturated over liquid (no ice from vapour alone),
 * judged on the closed-form saturation pressure in either property mode.          */
static int source_idle(const double *U)
{
    if (U[5] > N_MIN || U[9] > N_MIN || U[15] > N_MIN) return 0;
    if (!(U[4] > 0.0)) return 1;
    prim_t w;
    cons_to_prim(U, &w);
    double pv = U[4] * RGAS_VAP * w.T;
    if (pv < PV_FLOOR) pv = PV_FLOOR;
    return !(log(pv) - or_ln_psat_liq(w.T) > 0.0);
}

/* Components whose depletion bounds the sub-step and the positivity scaling:
 * vapour, liquid and ice moments (both liquid populations).                      */
static int depletable(int c) { return (c >= 4 && c <= 12) || (c >= 15 && c <= 18); }

/* Stiff source integration over dt (explicit sub-cycling, per-step positivity
 * scaling, complete-evaporation rule, mu1 realisability clamp). U0 and Q hold NV
 * entries. Returns Q = (U(t+dt) - U(t)) / dt and the number of sub-steps taken.   */
static int source_integrate(const or_ctx *cx, const double *U0, double dt, double *Q)
{
    double U[NV];
    memcpy(U, U0, sizeof(U));
    for (int v = 0; v < NV; ++v) Q[v] = 0.0;
    if (!cx->c.phase_change) return 0;
    const int npop = cx->bimodal ? 2 : 1;
    const double fpi = 4.0 / 3.0 * PI;
    rates_t r;
    double S[NV];
    phase_change_rates(cx, U, dt, &r);
    exchange_terms(U, (const double(*)[4])r.dM, r.dN, npop, r.act, r.mdot_f, S);
    /* rates that vanish in every component, with no population left without mass,
     * leave the state as it is, so every later evaluation vanishes too: no source
     * (e.g. a cell without particles that is not supersaturated over liquid) */
    int live = r.stale_l[0] || r.stale_l[1] || r.stale_s;
    for (int v = 0; v < NV && !live; ++v) live = S[v] != 0.0;
    if (!live) return 0;
    /* depletion time scales and positivity scaling protect the components that are
     * not negative already (transport of sharp fields can leave a moment slightly
     * negative; no scaling of the step restores it) */
    double tau = HUGE_VAL;
    for (int c = 4; c < NV; ++c)
        if (depletable(c) && U[c] >= 0.0 && S[c] < 0.0) {
            double t = U[c] / (-S[c]);
            if (t < tau) tau = t;
        }
    int nsub = 1;
    if (tau < HUGE_VAL) {
        double want = ceil(dt / (SUB_SAFETY * tau));
        if (want > (double)cx->c.n_sub_max) nsub = cx->c.n_sub_max;
        else if (want > 1.0) nsub = (int)want;
    }
    const double h = dt / nsub;
    for (int s = 0; s < nsub; ++s) {
        phase_change_rates(cx, U, h, &r);
        double dM[2][4], dN[4], act = r.act, mdf = r.mdot_f;
        for (int k = 0; k < 4; ++k) { dM[0][k] = r.dM[0][k]; dM[1][k] = r.dM[1][k]; dN[k] = r.dN[k]; }
        int evap_l[2] = {0, 0}, evap_s = 0;
        for (int pop = 0; pop < npop; ++pop) {
            const int b = liq_base(pop);
            if (r.stale_l[pop] || (r.Gl[pop] < 0.0 && U[b + 3] + h * (3.0 * U[b + 2] * r.Gl[pop]) <= 0.0)) {
                /* evaporation alone (the growth term of mu3, not the freezing sink) would
                 * empty the population within the sub-step: all droplets evaporate, none
                 * of them freezes; soot-activated ones release their soot */
                evap_l[pop] = 1;
                for (int k = 0; k < 4; ++k) dM[pop][k] = -U[b + k] / h;
                if (pop == 0) act = -U[14] / h;
            }
        }
        if (evap_l[0] || evap_l[1]) {
            /* the crystals keep their growth and the freezing of the surviving population */
            mdf = 0.0;
            for (int k = 0; k < 4; ++k) dN[k] = k > 0 ? k * U[9 + k - 1] * r.Gs : 0.0;
            for (int pop = 0; pop < npop; ++pop) {
                if (evap_l[pop]) continue;
                for (int k = 0; k < 4; ++k) dN[k] += pow(RHO_LIQ / RHO_ICE, k / 3.0) * r.F[pop][k];
                mdf += RHO_LIQ * fpi * r.F[pop][3];
            }
        }
        if (r.stale_s || (r.Gs < 0.0 && U[12] + h * dN[3] <= 0.0)) {
            evap_s = 1;
            for (int k = 0; k < 4; ++k) dN[k] = -U[9 + k] / h;
        }
        exchange_terms(U, (const double(*)[4])dM, dN, npop, act, mdf, S);
        /* positivity scaling; an evaporating population reaches zero at theta = 1 by
         * construction and is left out of the minimum.  The component that sets
         * theta < 1 (the first of equals) reaches zero: it is set to zero exactly
         * rather than left at the rounding residue of its update.                    */
        double theta = 1.0;
        int czero = -1;
        for (int c = 4; c < NV; ++c) {
            if (!depletable(c)) continue;
            if ((evap_l[0] && c >= 5 && c <= 8) || (evap_s && c >= 9 && c <= 12) || (evap_l[1] && c >= 15)) continue;
            if (U[c] >= 0.0 && S[c] < 0.0) {
                double t = U[c] / (-h * S[c]);
                if (t < theta) { theta = t; czero = c; }
            }
        }
        for (int v = 0; v < NV; ++v) U[v] = U[v] + theta * h * S[v];
        if (czero >= 0) U[czero] = 0.0;
        if (theta == 1.0) {
            if (evap_l[0]) { U[5] = U[6] = U[7] = U[8] = 0.0; U[14] = 0.0; }
            if (evap_l[1]) { U[15] = U[16] = U[17] = U[18] = 0.0; }
            if (evap_s) { U[9] = U[10] = U[11] = U[12] = 0.0; }
        }
        /* Hoelder bounds on mu1 given (mu0, mu2, mu3): mu2^2/mu3 <= mu1 <= sqrt(mu0 mu2).
         * When the interval is empty (an unrealisable (mu0, mu2, mu3) triple) mu1 takes
         * the upper bound, so the clamp is continuous where the interval degenerates
         * (monodisperse populations, e.g. freshly nucleated or frozen ones). */
        for (int set = 0; set < 3; ++set) {
            double *m = U + (set == 0 ? 5 : set == 1 ? 9 : 15);
            if (population_valid(m)) {
                double lo = m[2] * m[2] / m[3], hi = sqrt(m[0] * m[2]);
                if (lo > hi) lo = hi;
                if (m[1] < lo) m[1] = lo;
                if (m[1] > hi) m[1] = hi;
            }
        }
    }
    for (int v = 0; v < NV; ++v) Q[v] = (U[v] - U0[v]) / dt;
    return nsub;
}

/* ============================== equilibrium comparison model (Sec. 4.2) == */
/* The paper's comparison model lets vapour condense as soon as the cell is
 * supersaturated over liquid, with no nucleation barrier and no growth kinetics,
 * and lets the condensate freeze once ice is the stable phase.  Read here as an
 * instantaneous phase equilibrium of the cell's water at fixed dry air, velocity
 * and energy: the condensate is liquid when the equilibrium temperature is at or
 * above T_MELT, ice below it (at T_MELT both, split by the energy balance), and the
 * vapour sits at saturation over that phase, or all water is vapour when the cell
 * cannot saturate.  Like the kinetic model, ice never forms from vapour alone: a
 * cell without condensate changes only once it is supersaturated over liquid.
 * Energy: condensing vapour keeps its latent heat in the gas (the condensate
 * carries its enthalpy h_l or h_i at the final temperature).                     */
static const double T_MELT = 273.15;
static const double R_EQ_NEW = 1.0e-7;   /* m: radius of condensate that forms without soot */

typedef struct {
    double rho_a, rho_v, m_l, m_s, W, u, v, ke, rhoE;
} eq_cell_t;

/* End state of one phase branch at trial temperature Ts: vapour at saturation over
 * the phase (ice = 0 liquid, 1 ice; capped by the water available), the rest
 * condensed in that phase.  Returns the temperature the gas then has.           */
static double eq_branch_T(const or_ctx *cx, const eq_cell_t *e, int ice, double Ts, double *rho_v_out, double *cond_out)
{
    double rho_sat = exp(prop_lnp(cx, ice, Ts)) / (RGAS_VAP * Ts);
    double cond = e->W - rho_sat;
    if (cond < 0.0) cond = 0.0;
    double rho_v = e->W - cond;
    double hv = L_VAP0 + CP_VAP * (Ts - T_REF);
    double hl = hv - latent_vap(Ts), hi = hv - latent_sub(Ts);
    double L = ice ? 0.0 : cond, I = ice ? cond : 0.0;
    double rhoE = e->rhoE - (L - e->m_l) * (hl + e->ke) - (I - e->m_s) * (hi + e->ke);
    double rho = e->rho_a + rho_v;
    double Y = rho_v / rho;
    double eint = rhoE / rho - e->ke;
    if (rho_v_out) *rho_v_out = rho_v;
    if (cond_out) *cond_out = cond;
    return (eint - mix_h0(Y)) / mix_cv(Y);
}

/* Root of T_gas(Ts) = Ts of one branch by bisection (the gas temperature falls as
 * Ts rises: warmer saturation keeps more vapour and releases less heat).        */
static double eq_branch_root(const or_ctx *cx, const eq_cell_t *e, int ice)
{
    double a = 100.0, b = 1000.0;
    for (int it = 0; it < 64; ++it) {
        double m = 0.5 * (a + b);
        if (eq_branch_T(cx, e, ice, m, NULL, NULL) > m) a = m;
        else b = m;
    }
    return 0.5 * (a + b);
}

/* Moments of a population of mass M [kg/m^3] of material density rho_p: N
 * particles of one radius.                                                      */
static void eq_population(double M, double N, double rho_p, double *mom)
{
    if (!(M > 0.0) || !(N > 0.0)) {
        for (int k = 0; k < 4; ++k) mom[k] = 0.0;
        return;
    }
    double r = cbrt(M / (4.0 / 3.0 * PI * rho_p * N));
    mom[0] = N; mom[1] = N * r; mom[2] = N * r * r; mom[3] = N * r * r * r;
}

static int source_equilibrium(const or_ctx *cx, const double *U, double dt, double *Q)
{
    for (int v = 0; v < NV; ++v) Q[v] = 0.0;
    if (!cx->c.phase_change) return 0;
    if (source_idle(U)) return 0;   /* no condensate, not supersaturated over liquid */
    prim_t w;
    cons_to_prim(U, &w);
    const double fpi = 4.0 / 3.0 * PI;
    eq_cell_t e;
    e.rho_v = U[4];
    e.rho_a = U[0] - U[4];
    e.m_l = U[5] > N_MIN ? fpi * RHO_LIQ * U[8] : 0.0;
    e.m_s = U[9] > N_MIN ? fpi * RHO_ICE * U[12] : 0.0;
    e.W = e.rho_v + e.m_l + e.m_s;
    e.u = w.u; e.v = w.v;
    e.ke = 0.5 * (w.u * w.u + w.v * w.v);
    e.rhoE = U[3];

    /* phase of the condensate: liquid if its branch settles at or above T_MELT, ice
     * if the ice branch settles below, else both at T_MELT                          */
    double T_end, rho_v_end, L = 0.0, I = 0.0;
    double TL = eq_branch_root(cx, &e, 0), cL;
    eq_branch_T(cx, &e, 0, TL, &rho_v_end, &cL);
    if (TL >= T_MELT) {
        T_end = TL; L = cL;
    } else {
        double TI = eq_branch_root(cx, &e, 1), cI;
        eq_branch_T(cx, &e, 1, TI, &rho_v_end, &cI);
        if (TI < T_MELT) {
            T_end = TI; I = cI;
        } else {
            /* both phases at T_MELT, vapour saturated over liquid; the ice share is the
             * one that puts the gas at T_MELT (freezing releases h_sl = h_l - h_i)       */
            T_end = T_MELT;
            double rho_sat = exp(prop_lnp(cx, 0, T_MELT)) / (RGAS_VAP * T_MELT);
            double C = e.W - rho_sat;
            if (C < 0.0) C = 0.0;
            rho_v_end = e.W - C;
            double hv = L_VAP0 + CP_VAP * (T_MELT - T_REF);
            double hl = hv - latent_vap(T_MELT), hi = hv - latent_sub(T_MELT);
            double rho = e.rho_a + rho_v_end, Y = rho_v_end / rho;
            double rhoE_need = rho * (mix_h0(Y) + mix_cv(Y) * T_MELT + e.ke);
            double rhoE_liq = e.rhoE - (C - e.m_l) * (hl + e.ke) + e.m_s * (hi + e.ke);
            I = (rhoE_need - rhoE_liq) / (hl - hi);   /* each kg frozen adds h_l - h_i */
            if (I < 0.0) I = 0.0;
            if (I > C) I = C;
            L = C - I;
        }
    }
    (void)T_end;

    /* end state: dry air, velocity kept; gas mass and energy follow the exchange */
    double Un[NV];
    memcpy(Un, U, sizeof(Un));
    double rho = e.rho_a + rho_v_end;
    double hvT = L_VAP0 + CP_VAP * (T_end - T_REF);
    double hlT = hvT - latent_vap(T_end), hiT = hvT - latent_sub(T_end);
    Un[0] = rho;
    Un[1] = rho * e.u;
    Un[2] = rho * e.v;
    Un[3] = e.rhoE - (L - e.m_l) * (hlT + e.ke) - (I - e.m_s) * (hiT + e.ke);
    Un[4] = rho_v_end;
    /* particle numbers: the condensate keeps the particles it has (freezing and
     * melting move them between the phases); condensate that forms from none sits
     * on the soot, or without soot on particles of radius R_EQ_NEW               */
    double Nl = U[5] > N_MIN ? U[5] : 0.0, Ns = U[9] > N_MIN ? U[9] : 0.0;
    double N = Nl + Ns, C = L + I;
    int seeded = 0;
    if (C > 0.0 && !(N > N_MIN)) {
        if (U[13] > N_MIN) { N = U[13]; seeded = 1; }
        else N = C / (fpi * (I > 0.0 ? RHO_ICE : RHO_LIQ) * R_EQ_NEW * R_EQ_NEW * R_EQ_NEW);
    }
    double mom[4];
    eq_population(L, C > 0.0 ? N * L / C : 0.0, RHO_LIQ, mom);
    for (int k = 0; k < 4; ++k) Un[5 + k] = mom[k];
    eq_population(I, C > 0.0 ? N * I / C : 0.0, RHO_ICE, mom);
    for (int k = 0; k < 4; ++k) Un[9 + k] = mom[k];
    if (seeded) Un[14] = U[13];
    if (!(C > 0.0)) Un[14] = 0.0;
    for (int v = 0; v < NV; ++v) Q[v] = (Un[v] - U[v]) / dt;
    return 1;
}

int or_set_equilibrium(or_ctx *cx, int on)
{
    if (on && cx->bimodal) return -1;   /* the equilibrium model has one liquid population */
    cx->equilibrium = on ? 1 : 0;
    return 0;
}

/* Two liquid populations (Sec. 2.2): soot-activated droplets keep variables 5..8,
 * homogeneously nucleated ones get 15..18, and arrays in memory hold 19 planes.
 * Not with the equilibrium model or particle drift (one liquid population each). */
int or_set_bimodal(or_ctx *cx, int on)
{
    if (on && (cx->equilibrium || cx->drift)) return -1;
    cx->bimodal = on ? 1 : 0;
    cx->nv = on ? NV : NV_BASE;
    return 0;
}

int or_nvar(const or_ctx *cx) { return cx->nv; }

/* Source of one cell; U and Q hold cx->nv entries.                               */
int or_source_cell(const or_ctx *cx, const double *Uin, double dt, double *Qout)
{
    double U[NV] = {0}, Q[NV];
    memcpy(U, Uin, sizeof(double) * cx->nv);
    int n = cx->equilibrium ? source_equilibrium(cx, U, dt, Q) : source_integrate(cx, U, dt, Q);
    memcpy(Qout, Q, sizeof(double) * cx->nv);
    return n;
}

/* ========================================================== mesh (Sec. 4.1) == */
static void build_mesh(or_ctx *cx)
{
    const or_mesh *m = &cx->m;
    int nx = m->nx, nr = m->nr;
    cx->xf = malloc(sizeof(double) * (nx + 1));
    cx->rf = malloc(sizeof(double) * (nr + 1));
    cx->xc = malloc(sizeof(double) * (nx + 4));
    cx->rc = malloc(sizeof(double) * (nr + 4));
    cx->dx = malloc(sizeof(double) * nx);
    cx->dr = malloc(sizeof(double) * nr);
    /* axial: geometric stretching from x = 0 */
    for (int i = 0; i <= nx; ++i) {
        if (m->sx_ratio == 1.0) cx->xf[i] = m->Lx * i / nx;
        else cx->xf[i] = m->Lx * (pow(m->sx_ratio, i) - 1.0) / (pow(m->sx_ratio, nx) - 1.0);
    }
    cx->xf[nx] = m->Lx;
    /* radial: interior-point sinh clustering about r_cluster */
    if (m->r_cluster > 0.0) {
        double b = m->beta_r, D = m->r_cluster, H = m->Lr;
        double A = 0.5 / b * log((1.0 + (exp(b) - 1.0) * D / H) / (1.0 + (exp(-b) - 1.0) * D / H));
        for (int j = 0; j <= nr; ++j) {
            double eta = (double)j / nr;
            cx->rf[j] = D * (1.0 + sinh(b * (eta - A)) / sinh(b * A));
        }
    } else {
        for (int j = 0; j <= nr; ++j) cx->rf[j] = m->Lr * j / nr;
    }
    cx->rf[0] = 0.0;
    cx->rf[nr] = m->Lr;
    for (int i = 0; i < nx; ++i) {
        cx->dx[i] = cx->xf[i + 1] - cx->xf[i];
        cx->xc[i + 2] = 0.5 * (cx->xf[i] + cx->xf[i + 1]);
    }
    for (int j = 0; j < nr; ++j) {
        cx->dr[j] = cx->rf[j + 1] - cx->rf[j];
        cx->rc[j + 2] = 0.5 * (cx->rf[j] + cx->rf[j + 1]);
    }
    /* ghost centres mirrored about the boundary faces */
    for (int g = 0; g < 2; ++g) {
        cx->xc[1 - g] = 2.0 * cx->xf[0] - cx->xc[2 + g];
        cx->xc[nx + 2 + g] = 2.0 * cx->xf[nx] - cx->xc[nx + 1 - g];
        cx->rc[1 - g] = 2.0 * cx->rf[0] - cx->rc[2 + g];
        cx->rc[nr + 2 + g] = 2.0 * cx->rf[nr] - cx->rc[nr + 1 - g];
    }
}

#define XC(i) (cx->xc[(i) + 2])
#define RC(j) (cx->rc[(j) + 2])

/* ============================================= case, inflow, initial state == */
static void stream_state(double p, double T, double u, double Y, double nsoot, double *U)
{
    double rho = p / (mix_R(Y) * T);
    double phi[NV] = {0};
    phi[13] = nsoot / rho;
    prim_to_cons(rho, u, 0.0, p, Y, phi, U);
}

or_ctx *or_create(const or_mesh *m, const or_case *c)
{
    or_ctx *cx = calloc(1, sizeof(or_ctx));
    cx->m = *m;
    cx->c = *c;
    cx->nx = m->nx;
    cx->nr = m->nr;
    cx->nv = NV_BASE;
    build_mesh(cx);
    if (m->geom == GEOM_Q1D) {
        cx->ax = malloc(sizeof(double) * (m->nx + 1));
        for (int i = 0; i <= m->nx; ++i) cx->ax[i] = 1.0;   /* a straight duct until set */
    }
    /* ambient: vapour partial pressure from the ice relative humidity */
    double pv = c->RH_ice * exp(or_ln_psat_ice(c->T_amb));
    double rho_v = pv / (RGAS_VAP * c->T_amb);
    double rho_a = (c->p_amb - pv) / (RGAS_AIR * c->T_amb);
    cx->Y_amb = rho_v / (rho_a + rho_v);
    double Ra = mix_R(cx->Y_amb), cpa = mix_cp(cx->Y_amb);
    cx->u_amb = c->mach_amb * sqrt(cpa / (cpa - Ra) * Ra * c->T_amb);
    stream_state(c->p_amb, c->T_amb, cx->u_amb, cx->Y_amb, 0.0, cx->ambient);
    double Yb = c->Y_byp < 0.0 ? cx->Y_amb : c->Y_byp;
    cx->inflow = malloc(sizeof(double) * NV * m->nr);
    for (int j = 0; j < m->nr; ++j) {
        double r = RC(j);
        double *U = cx->inflow + NV * j;
        if (r < c->R_core) stream_state(c->p_amb, c->T_core, c->u_core, c->Y_core, c->n_soot, U);
        else if (r < c->R_fan) stream_state(c->p_amb, c->T_byp, c->u_byp, Yb, 0.0, U);
        else memcpy(U, cx->ambient, sizeof(double) * NV);
    }
    cx->f_theta = or_contact_factor(c->theta_deg * PI / 180.0);
    double ls = log(c->sigma_g_soot);
    cx->soot_area = 4.0 * PI * c->r_g_soot * c->r_g_soot * exp(2.0 * ls * ls);
    cx->delta0 = c->delta0_frac * c->R_core;
    return cx;
}

void or_destroy(or_ctx *cx)
{
    if (!cx) return;
    free(cx->xf); free(cx->rf); free(cx->xc); free(cx->rc); free(cx->dx); free(cx->dr);
    free(cx->inflow);
    free(cx->ax);
    free(cx->ptab);
    free(cx);
}

/* Quasi-1D duct: the cross-section area at the nx+1 x faces (all > 0).  The
 * duct has one row of cells; walls close it in r.  Returns -1 for other
 * geometries or a non-positive area.                                            */
int or_set_area(or_ctx *cx, const double *area)
{
    if (cx->m.geom != GEOM_Q1D || cx->nr != 1) return -1;
    for (int i = 0; i <= cx->nx; ++i)
        if (!(area[i] > 0.0)) return -1;
    memcpy(cx->ax, area, sizeof(double) * (cx->nx + 1));
    return 0;
}

void or_mesh_faces(const or_ctx *cx, double *xf, double *rf)
{
    memcpy(xf, cx->xf, sizeof(double) * (cx->nx + 1));
    memcpy(rf, cx->rf, sizeof(double) * (cx->nr + 1));
}

void or_case_derived(const or_ctx *cx, double *out /* Y_amb, u_amb, f_theta, soot_area */)
{
    out[0] = cx->Y_amb; out[1] = cx->u_amb; out[2] = cx->f_theta; out[3] = cx->soot_area;
}

int or_init(const or_ctx *cx, double *U)
{
    const int nx = cx->nx, nr = cx->nr;
    const size_t plane = (size_t)nx * nr;
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i)
            for (int v = 0; v < cx->nv; ++v) U[v * plane + (size_t)j * nx + i] = cx->inflow[NV * j + v];
    return 0;
}

/* ================================================================ BCs ====== */
/* State of cell (i, j) for i in [-2, nx+1], j in [-2, nr+1]: interior cells are
 * read from U; ghost cells follow the boundary treatment of each side.           */
static void cell_state(const or_ctx *cx, const double *U, int i, int j, double *out)
{
    const int nx = cx->nx, nr = cx->nr;
    const size_t plane = (size_t)nx * nr;
    int flip_u = 0, flip_v = 0;
    /* repeated mirroring handles meshes thinner than the ghost depth */
    while (j < 0 || j >= nr) {
        if (j < 0) {                         /* axis or wall: mirror, v odd          */
            j = -1 - j;
            flip_v ^= 1;
        } else {
            if (cx->m.bc_rhi == BC_FARFIELD) { memcpy(out, cx->ambient, sizeof(double) * NV); return; }
            if (cx->m.bc_rhi == BC_WALL) { j = 2 * nr - 1 - j; flip_v ^= 1; }
            else j = nr - 1;
        }
    }
    const double *src = NULL;
    while (!src && (i < 0 || i >= nx)) {
        if (i < 0) {
            if (cx->m.bc_xlo == BC_INFLOW) src = cx->inflow + NV * j;
            else if (cx->m.bc_xlo == BC_WALL) { i = -1 - i; flip_u ^= 1; }
            else i = 0;
        } else {
            if (cx->m.bc_xhi == BC_WALL) { i = 2 * nx - 1 - i; flip_u ^= 1; }
            else i = nx - 1;
        }
    }
    if (src) memcpy(out, src, sizeof(double) * NV);
    else
        for (int v = 0; v < NV; ++v) out[v] = v < cx->nv ? U[v * plane + (size_t)j * nx + i] : 0.0;
    if (flip_u) out[1] = -out[1];
    if (flip_v) out[2] = -out[2];
}

/* ======================================================= numerics: Sec. 3.2 == */
/* Extended field of primitives over [-2, nx+1] x [-2, nr+1].                    */
typedef struct {
    int nx, nr, ex;              /* ex = nx + 4                                    */
    prim_t *w;
    double *mu, *mut, *Dv;       /* molecular viscosity, eddy viscosity, vapour D  */
} field_t;

#define FW(f, i, j) ((f)->w[((j) + 2) * (f)->ex + (i) + 2])
#define FS(f, a, i, j) ((f)->a[((j) + 2) * (f)->ex + (i) + 2])

static double mixing_length(const or_ctx *cx, double x)
{
    return cx->c.kappa_m * (cx->delta0 + cx->c.s_delta * x);
}

static void build_field(const or_ctx *cx, const double *U, field_t *f)
{
    const int nx = cx->nx, nr = cx->nr;
    f->nx = nx; f->nr = nr; f->ex = nx + 4;
    size_t n = (size_t)(nx + 4) * (nr + 4);
    f->w = malloc(sizeof(prim_t) * n);
    f->mu = calloc(n, sizeof(double));
    f->mut = calloc(n, sizeof(double));
    f->Dv = calloc(n, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = -2; j < nr + 2; ++j)
        for (int i = -2; i < nx + 2; ++i) {
            double Uc[NV];
            cell_state(cx, U, i, j, Uc);
            prim_t *w = &FW(f, i, j);
            cons_to_prim(Uc, w);
            FS(f, mu, i, j) = or_mu_sutherland(w->T);
            FS(f, Dv, i, j) = DIFF_V0 * pow(w->T / T_REF, DIFF_V_EXP) * (DIFF_P0 / w->p);
        }
    /* algebraic eddy viscosity (stands in for Spalart-Allmaras):
     * mu_t = rho l_m^2 |du/dr + dv/dx| with central differences at the cell      */
#pragma omp parallel for schedule(static)
    for (int j = -1; j < nr + 1; ++j)
        for (int i = -1; i < nx + 1; ++i) {
            double dudr = (FW(f, i, j + 1).u - FW(f, i, j - 1).u) / (RC(j + 1) - RC(j - 1));
            double dvdx = (FW(f, i + 1, j).v - FW(f, i - 1, j).v) / (XC(i + 1) - XC(i - 1));
            double lm = mixing_length(cx, XC(i));
            FS(f, mut, i, j) = FW(f, i, j).rho * lm * lm * fabs(dudr + dvdx);
        }
}

static void free_field(field_t *f)
{
    free(f->w); free(f->mu); free(f->mut); free(f->Dv);
}

/* MUSCL with the van Leer limiter in harmonic form, index space.                 */
static double van_leer(double a, double b)
{
    return (a * b > 0.0) ? 2.0 * a * b / (a + b) : 0.0;
}

/* reconstructed variables: rho, u_n, u_t, p, Y, phi5..phi14                     */
static void recon_vars(const prim_t *w, int dir, double *q)
{
    q[0] = w->rho;
    q[1] = dir == 0 ? w->u : w->v;
    q[2] = dir == 0 ? w->v : w->u;
    q[3] = w->p;
    q[4] = w->Y;
    for (int m = 5; m < NV; ++m) q[m] = w->phi[m];
}

/* Roe flux (primitive-jump form, Harten entropy fix on the acoustic waves) for
 * (rho, rho u_n, rho u_t, rho E); per-mass scalars take the upwinded mass flux.
 * Output F in the rotated frame: F[1] normal momentum, F[2] tangential.          */
static void roe_flux(const double *L, const double *R, double *F)
{
    double rl = L[0], unl = L[1], utl = L[2], pl = L[3], Yl = L[4];
    double rr = R[0], unr = R[1], utr = R[2], pr = R[3], Yr = R[4];
    double Hl = mix_cp(Yl) * (pl / (rl * mix_R(Yl))) + mix_h0(Yl) + 0.5 * (unl * unl + utl * utl);
    double Hr = mix_cp(Yr) * (pr / (rr * mix_R(Yr))) + mix_h0(Yr) + 0.5 * (unr * unr + utr * utr);
    double ml = rl * unl, mr = rr * unr;
    double FL[4] = {ml, ml * unl + pl, ml * utl, ml * Hl};
    double FR[4] = {mr, mr * unr + pr, mr * utr, mr * Hr};

    double sl = sqrt(rl), sr = sqrt(rr);
    double wl = sl / (sl + sr), wr = sr / (sl + sr);
    double rho = sl * sr;
    double un = wl * unl + wr * unr;
    double ut = wl * utl + wr * utr;
    double H = wl * Hl + wr * Hr;
    double Y = wl * Yl + wr * Yr;
    double q2 = un * un + ut * ut;
    double cp = mix_cp(Y), Rm = mix_R(Y);
    double gam = cp / (cp - Rm);
    double T = (H - 0.5 * q2 - mix_h0(Y)) / cp;
    double c = sqrt(gam * Rm * T);

    double drho = rr - rl, dun = unr - unl, dut = utr - utl, dp = pr - pl;
    double a1 = (dp - rho * c * dun) / (2.0 * c * c);
    double a2 = drho - dp / (c * c);
    double a3 = rho * dut;
    double a4 = (dp + rho * c * dun) / (2.0 * c * c);
    double l1 = fabs(un - c), l2 = fabs(un), l4 = fabs(un + c);
    double del = 0.1 * c;
    if (l1 < del) l1 = (l1 * l1 + del * del) / (2.0 * del);
    if (l4 < del) l4 = (l4 * l4 + del * del) / (2.0 * del);
    double K1[4] = {1.0, un - c, ut, H - un * c};
    /* entropy wave: d(rho E) at fixed p, u and Y is (q^2/2 + h0(Y)) d rho, because
     * rho e = p/(gamma-1) + rho h0(Y) for the offset caloric law                   */
    double K2[4] = {1.0, un, ut, 0.5 * q2 + mix_h0(Y)};
    double K3[4] = {0.0, 0.0, 1.0, ut};
    double K4[4] = {1.0, un + c, ut, H + un * c};
    for (int k = 0; k < 4; ++k) {
        double diss = l1 * a1 * K1[k] + l2 * a2 * K2[k] + l2 * a3 * K3[k] + l4 * a4 * K4[k];
        F[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * diss;
    }
    /* species and moment scalars: upwind with the Roe mass flux */
    for (int m = 4; m < NV; ++m) F[m] = F[0] * (F[0] >= 0.0 ? L[m] : R[m]);
}

/* ================================================ drift of the particles (Eq. 24) == */
/* The drag law (Eq. 24) read as a drift flux: droplets and crystals lag the gas's
 * pressure-driven acceleration, so relative to the gas a particle of radius r moves
 * with the terminal slip at which the drag of Eq. 24 balances the pressure-gradient
 * force.  In the Stokes limit that is w_St(r) = (2 rho_p r^2 Cc(r) / (9 mu))
 * (1 - rho/rho_p) (dp/dn) / rho, with the Cunningham factor Cc = 1 + 2 A_C Kn,
 * Kn = lbar / (2 r); the Schiller-Naumann factor 1 + 0.15 Re^0.687 divides it,
 * Re = rho |w| 2 r / mu on the diameter (the Reynolds number with which C_D Re -> 24
 * is Stokes's law), so w solves w (1 + 0.15 Re(w)^0.687) = w_St: six fixed-point
 * steps from w_St (converged to about 1e-8 at Re = 1).  Each population drifts as a
 * whole with the slip of its mean radius r20, so all its moments cross a face with
 * the same velocity (upwind in its sign), which keeps the moment set realisable.
 * Face values: means of the two cells; lbar = 1.5 mu sqrt(R T) / p.  Soot stays
 * with the gas (its response time is negligible).                               */
double or_sn_slip(double w_st, double rho, double r, double mu)
{
    double w = w_st;
    for (int it = 0; it < 6; ++it) {
        double Re = rho * fabs(w) * 2.0 * r / mu;
        w = w_st / (1.0 + 0.15 * pow(Re, 0.687));
    }
    return w;
}

static void drift_add(const prim_t *a, const prim_t *b, double mu_a, double mu_b, double dn, double *F)
{
    double rho = 0.5 * (a->rho + b->rho), mu = 0.5 * (mu_a + mu_b);
    double p = 0.5 * (a->p + b->p), T = 0.5 * (a->T + b->T), R = 0.5 * (a->R + b->R);
    double lbar = 1.5 * mu * sqrt(R * T) / p;
    double dpdn = (b->p - a->p) / dn;
    for (int pop = 0; pop < 2; ++pop) {
        int base = pop ? 9 : 5;
        double rho_p = pop ? RHO_ICE : RHO_LIQ;
        double c = 2.0 * rho_p * (1.0 - rho / rho_p) * dpdn / (9.0 * mu * rho);
        const prim_t *w = c > 0.0 ? a : b;
        double M[4];
        for (int k = 0; k < 4; ++k) M[k] = w->rho * w->phi[base + k];
        if (!population_valid(M)) continue;
        double r20 = sqrt(M[2] / M[0]);
        double Kn = lbar / (2.0 * r20);
        double W = or_sn_slip(c * r20 * r20 * (1.0 + 2.0 * or_cunningham_ac(Kn) * Kn), rho, r20, mu);
        for (int k = 0; k < 4; ++k) F[base + k] += W * M[k];
    }
}

int or_set_drift(or_ctx *cx, int on)
{
    if (on && cx->bimodal) return -1;   /* drift is defined for one liquid population */
    cx->drift = on ? 1 : 0;
    return 0;
}

/* Convective minus viscous flux through one face, in global components.
 * dir 0: face between (i,j) and (i+1,j); dir 1: between (i,j) and (i,j+1).       */
static void face_flux(const or_ctx *cx, const field_t *f, int dir, int i, int j, double *Fout)
{
    const int di = dir == 0 ? 1 : 0, dj = dir == 0 ? 0 : 1;
    /* MUSCL: four cells along the normal */
    double qm[NV], q0[NV], q1[NV], q2[NV], L[NV], R[NV];
    recon_vars(&FW(f, i - di, j - dj), dir, qm);
    recon_vars(&FW(f, i, j), dir, q0);
    recon_vars(&FW(f, i + di, j + dj), dir, q1);
    recon_vars(&FW(f, i + 2 * di, j + 2 * dj), dir, q2);
    for (int m = 0; m < NV; ++m) {
        double s0 = van_leer(q0[m] - qm[m], q1[m] - q0[m]);
        double s1 = van_leer(q1[m] - q0[m], q2[m] - q1[m]);
        L[m] = q0[m] + 0.5 * s0;
        R[m] = q1[m] - 0.5 * s1;
    }
    double Fc[NV];
    roe_flux(L, R, Fc);

    /* central viscous / eddy flux */
    const prim_t *a = &FW(f, i, j), *b = &FW(f, i + di, j + dj);
    double dn = dir == 0 ? XC(i + 1) - XC(i) : RC(j + 1) - RC(j);
    double mu = 0.5 * (FS(f, mu, i, j) + FS(f, mu, i + di, j + dj));
    double mut = 0.5 * (FS(f, mut, i, j) + FS(f, mut, i + di, j + dj));
    double rho = 0.5 * (a->rho + b->rho);
    double cp = 0.5 * (a->cp + b->cp);
    double Dv = 0.5 * (FS(f, Dv, i, j) + FS(f, Dv, i + di, j + dj));
    double dh = 0.5 * ((L_VAP0 + CP_VAP * (a->T - T_REF) - CP_AIR * (a->T - T_REF))
                       + (L_VAP0 + CP_VAP * (b->T - T_REF) - CP_AIR * (b->T - T_REF)));
    double uf = 0.5 * (a->u + b->u), vf = 0.5 * (a->v + b->v);
    double un_n = ((dir == 0 ? b->u : b->v) - (dir == 0 ? a->u : a->v)) / dn; /* normal velocity along n */
    double ut_n = ((dir == 0 ? b->v : b->u) - (dir == 0 ? a->v : a->u)) / dn; /* tangential velocity along n */
    double dT_n = (b->T - a->T) / dn;
    double dY_n = (b->Y - a->Y) / dn;
    /* tangential derivatives: mean of the two cells' central differences */
    double dut_t, dun_t;   /* d(u_t)/dt and d(u_n)/dt along the tangential direction */
    if (dir == 0) {
        double h = RC(j + 1) - RC(j - 1);
        double dv_a = (FW(f, i, j + 1).v - FW(f, i, j - 1).v) / h;
        double dv_b = (FW(f, i + 1, j + 1).v - FW(f, i + 1, j - 1).v) / h;
        double du_a = (FW(f, i, j + 1).u - FW(f, i, j - 1).u) / h;
        double du_b = (FW(f, i + 1, j + 1).u - FW(f, i + 1, j - 1).u) / h;
        dut_t = 0.5 * (dv_a + dv_b);   /* dv/dr */
        dun_t = 0.5 * (du_a + du_b);   /* du/dr */
    } else {
        double h = XC(i + 1) - XC(i - 1);
        double du_a = (FW(f, i + 1, j).u - FW(f, i - 1, j).u) / h;
        double du_b = (FW(f, i + 1, j + 1).u - FW(f, i - 1, j + 1).u) / h;
        double dv_a = (FW(f, i + 1, j).v - FW(f, i - 1, j).v) / h;
        double dv_b = (FW(f, i + 1, j + 1).v - FW(f, i - 1, j + 1).v) / h;
        dut_t = 0.5 * (du_a + du_b);   /* du/dx */
        dun_t = 0.5 * (dv_a + dv_b);   /* dv/dx */
    }
    double hoop = 0.0;
    if (cx->m.geom == 0) hoop = dir == 0 ? vf / RC(j) : vf / cx->rf[j + 1];
    double div = un_n + dut_t + hoop;         /* du/dx + dv/dr + v/r              */
    double mue = mu + mut;
    double tau_nn = mue * (2.0 * un_n - 2.0 / 3.0 * div);
    double tau_nt = mue * (ut_n + dun_t);     /* du/dr + dv/dx                      */
    double diffY = rho * Dv + mut / SCHMIDT_T;
    double Jv = -diffY * dY_n;
    double qn = -(cp * mu / PRANDTL + cp * mut / PRANDTL_T) * dT_n + dh * Jv;
    double Fv[NV];
    Fv[0] = 0.0;
    if (dir == 0) {
        Fv[1] = tau_nn; Fv[2] = tau_nt;
        Fv[3] = uf * tau_nn + vf * tau_nt - qn;
    } else {
        Fv[1] = tau_nt; Fv[2] = tau_nn;
        Fv[3] = uf * tau_nt + vf * tau_nn - qn;
    }
    Fv[4] = -Jv;
    for (int m = 5; m < NV; ++m) Fv[m] = mut / SCHMIDT_T * (b->phi[m] - a->phi[m]) / dn;

    /* convective flux back to global components */
    double Fg[NV];
    Fg[0] = Fc[0];
    Fg[1] = dir == 0 ? Fc[1] : Fc[2];
    Fg[2] = dir == 0 ? Fc[2] : Fc[1];
    for (int m = 3; m < NV; ++m) Fg[m] = Fc[m];
    if (cx->drift) drift_add(a, b, FS(f, mu, i, j), FS(f, mu, i + di, j + dj), dn, Fg);
    for (int m = 0; m < NV; ++m) Fout[m] = Fg[m] - Fv[m];
}

/* Cell volume: per radian (axisymmetric), per unit depth (planar), or the
 * trapezoidal duct volume 0.5 (A_w + A_e) dx (quasi-1D).                        */
static double cell_volume(const or_ctx *cx, int i, int j)
{
    if (cx->m.geom == GEOM_Q1D) return 0.5 * (cx->ax[i] + cx->ax[i + 1]) * cx->dx[i];
    if (cx->m.geom == GEOM_AXI) return RC(j) * cx->dr[j] * cx->dx[i];
    return cx->dr[j] * cx->dx[i];
}

/* Transport residual per unit volume: -(1/V) sum_faces (Fc - Fv).A plus the
 * axisymmetric pressure / hoop-stress source on radial momentum.  In the
 * quasi-1D duct the x faces carry the duct areas, there are no r faces, and the
 * walls push on the gas with p (A_e - A_w) along x: the textbook quasi-1D Euler
 * equations, d(rho u A)/dx = 0, d((rho u^2 + p) A)/dx = p dA/dx, in finite-volume
 * form.                                                                         */
static void transport_residual(const or_ctx *cx, const double *U, double *Rout)
{
    const int nx = cx->nx, nr = cx->nr;
    const size_t plane = (size_t)nx * nr;
    field_t f;
    build_field(cx, U, &f);
    double *Fx = malloc(sizeof(double) * NV * (size_t)(nx + 1) * nr);
    double *Fr = calloc((size_t)NV * nx * (nr + 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nr; ++j)
        for (int i = -1; i < nx; ++i) face_flux(cx, &f, 0, i, j, Fx + NV * ((size_t)j * (nx + 1) + i + 1));
#pragma omp parallel for schedule(static)
    for (int j = -1; j < nr; ++j)
        for (int i = 0; i < nx; ++i) {
            double *F = Fr + NV * ((size_t)(j + 1) * nx + i);
            if (cx->m.geom == 0 && j == -1) continue;       /* axis face: zero area */
            if (cx->m.geom == GEOM_Q1D) continue;           /* duct: no r faces     */
            face_flux(cx, &f, 1, i, j, F);
        }
    const int axi = cx->m.geom == 0;
    const int q1d = cx->m.geom == GEOM_Q1D;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i) {
            double Ax = axi ? RC(j) * cx->dr[j] : cx->dr[j];
            double As = axi ? cx->rf[j] * cx->dx[i] : cx->dx[i];
            double An = axi ? cx->rf[j + 1] * cx->dx[i] : cx->dx[i];
            double V = axi ? RC(j) * cx->dr[j] * cx->dx[i] : cx->dr[j] * cx->dx[i];
            const double *Fw = Fx + NV * ((size_t)j * (nx + 1) + i);
            const double *Fe = Fx + NV * ((size_t)j * (nx + 1) + i + 1);
            const double *Fs = Fr + NV * ((size_t)j * nx + i);
            const double *Fn = Fr + NV * ((size_t)(j + 1) * nx + i);
            double Sax = 0.0;
            if (axi) {
                const prim_t *w = &FW(&f, i, j);
                double dudx = (FW(&f, i + 1, j).u - FW(&f, i - 1, j).u) / (XC(i + 1) - XC(i - 1));
                double dvdr = (FW(&f, i, j + 1).v - FW(&f, i, j - 1).v) / (RC(j + 1) - RC(j - 1));
                double vr = w->v / RC(j);
                double div = dudx + dvdr + vr;
                double mue = FS(&f, mu, i, j) + FS(&f, mut, i, j);
                double tau_tt = mue * (2.0 * vr - 2.0 / 3.0 * div);
                Sax = (w->p - tau_tt) * cx->dx[i] * cx->dr[j];
            }
            if (q1d) {
                double Aw = cx->ax[i], Ae = cx->ax[i + 1];
                double Vq = cell_volume(cx, i, j);
                for (int v = 0; v < cx->nv; ++v) {
                    double Rv = -(Fe[v] * Ae - Fw[v] * Aw);
                    if (v == 1) Rv += FW(&f, i, j).p * (Ae - Aw);
                    Rout[v * plane + (size_t)j * nx + i] = Rv / Vq;
                }
                continue;
            }
            for (int v = 0; v < cx->nv; ++v) {
                double net = (Fe[v] - Fw[v]) * Ax + (Fn[v] * An - Fs[v] * As);
                double Rv = -net;
                if (v == 2) Rv += Sax;
                Rout[v * plane + (size_t)j * nx + i] = Rv / V;
            }
        }
    free(Fx);
    free(Fr);
    free_field(&f);
}

int or_residual(const or_ctx *cx, const double *U, double *R)
{
    transport_residual(cx, U, R);
    return 0;
}

/* Source Q(U, dt) on the whole mesh; returns the total number of sub-steps.      */
long or_source(const or_ctx *cx, const double *U, double dt, double *Q)
{
    const int nx = cx->nx, nr = cx->nr;
    const size_t plane = (size_t)nx * nr;
    long total = 0;
#pragma omp parallel for schedule(static) reduction(+ : total)
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i) {
            double Uc[NV] = {0}, Qc[NV];
            for (int v = 0; v < cx->nv; ++v) Uc[v] = U[v * plane + (size_t)j * nx + i];
            total += cx->equilibrium ? source_equilibrium(cx, Uc, dt, Qc) : source_integrate(cx, Uc, dt, Qc);
            for (int v = 0; v < cx->nv; ++v) Q[v * plane + (size_t)j * nx + i] = Qc[v];
        }
    return total;
}

/* Global CFL time step: dt = CFL min 1/((|u|+c)/dx + (|v|+c)/dr + 2 nu_eff (1/dx^2+1/dr^2)). */
int or_cfl_dt(const or_ctx *cx, const double *U, double *dt_out)
{
    const int nx = cx->nx, nr = cx->nr;
    field_t f;
    build_field(cx, U, &f);
    double best = HUGE_VAL;
#pragma omp parallel for schedule(static) reduction(min : best)
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i) {
            const prim_t *w = &FW(&f, i, j);
            /* the quasi-1D duct has no r direction: its r terms vanish */
            double idx = 1.0 / cx->dx[i], idr = cx->m.geom == GEOM_Q1D ? 0.0 : 1.0 / cx->dr[j];
            double fac = w->gam / PRANDTL;
            if (fac < 4.0 / 3.0) fac = 4.0 / 3.0;
            double nu = (FS(&f, mu, i, j) + FS(&f, mut, i, j)) / w->rho * fac;
            double rate = (fabs(w->u) + w->c) * idx + (fabs(w->v) + w->c) * idr
                          + 2.0 * nu * (idx * idx + idr * idr);
            double d = 1.0 / rate;
            if (d < best) best = d;
        }
    free_field(&f);
    *dt_out = cx->c.cfl * best;
    return 0;
}

/* One SSP-RK3 (Shu-Osher) step with L(U) = R(U)/V + Q(U, dt).                     */
int or_step(const or_ctx *cx, double *U, double dt)
{
    const size_t n = (size_t)cx->nv * cx->nx * cx->nr;
    double *R = malloc(sizeof(double) * n), *Q = malloc(sizeof(double) * n);
    double *U1 = malloc(sizeof(double) * n), *U2 = malloc(sizeof(double) * n);
    transport_residual(cx, U, R);
    or_source(cx, U, dt, Q);
    for (size_t k = 0; k < n; ++k) U1[k] = U[k] + dt * (R[k] + Q[k]);
    transport_residual(cx, U1, R);
    or_source(cx, U1, dt, Q);
    for (size_t k = 0; k < n; ++k) U2[k] = 0.75 * U[k] + 0.25 * (U1[k] + dt * (R[k] + Q[k]));
    transport_residual(cx, U2, R);
    or_source(cx, U2, dt, Q);
    for (size_t k = 0; k < n; ++k) U[k] = (1.0 / 3.0) * U[k] + (2.0 / 3.0) * (U2[k] + dt * (R[k] + Q[k]));
    free(R); free(Q); free(U1); free(U2);
    return 0;
}

/* n steps, each with its own global CFL dt; returns the simulated time.          */
double or_run(const or_ctx *cx, double *U, int nsteps)
{
    double t = 0.0;
    for (int s = 0; s < nsteps; ++s) {
        double dt;
        or_cfl_dt(cx, U, &dt);
        or_step(cx, U, dt);
        t += dt;
    }
    return t;
}

/* Diagnostics: total water mass per radian, max ln S_l, total ice number.          */
/* O7.8 diagnostics of the drag law (Eq. 24): the response time of each particle
 * population at its mean radius r20, tau_p = rho_p (2 r20)^2 Cc / (18 mu) (the
 * particle mass over its Stokes friction coefficient 6 pi mu r / Cc; zero slip, so
 * the Schiller-Naumann factor is 1), and the Stokes number St = tau_p |u| / dx_i.
 * tau and St hold 2 planes (droplets, crystals) of nr x nx; zero where the
 * population is empty or has evaporated.                                        */
void or_particle_times(const or_ctx *cx, const double *U, double *tau, double *St)
{
    const int nx = cx->nx, nr = cx->nr;
    const size_t plane = (size_t)nx * nr;
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t c = (size_t)j * nx + i;
            double Uc[NV] = {0};
            for (int v = 0; v < cx->nv; ++v) Uc[v] = U[v * plane + c];
            prim_t w;
            cons_to_prim(Uc, &w);
            const double mu = or_mu_sutherland(w.T);
            const double lbar = 1.5 * mu * sqrt(w.R * w.T) / w.p;
            const double speed = sqrt(w.u * w.u + w.v * w.v);
            for (int pop = 0; pop < 2; ++pop) {
                const double *M = Uc + (pop ? 9 : 5);
                const double rho_p = pop ? RHO_ICE : RHO_LIQ;
                double t = 0.0;
                if (population_valid(M)) {
                    const double r20 = sqrt(M[2] / M[0]);
                    const double Kn = lbar / (2.0 * r20);
                    const double Cc = 1.0 + 2.0 * or_cunningham_ac(Kn) * Kn;
                    t = rho_p * (2.0 * r20) * (2.0 * r20) * Cc / (18.0 * mu);
                }
                tau[pop * plane + c] = t;
                St[pop * plane + c] = t * speed / cx->dx[i];
            }
        }
}

void or_diag(const or_ctx *cx, const double *U, double *out)
{
    const int nx = cx->nx, nr = cx->nr;
    const size_t plane = (size_t)nx * nr;
    double water = 0.0, lnS = -HUGE_VAL, nice = 0.0, gas = 0.0;
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t k = (size_t)j * nx + i;
            double V = cell_volume(cx, i, j);
            double liq = U[8 * plane + k];
            if (cx->bimodal) liq += U[18 * plane + k];
            water += V * (U[4 * plane + k] + 4.0 / 3.0 * PI * (RHO_LIQ * liq + RHO_ICE * U[12 * plane + k]));
            nice += V * U[9 * plane + k];
            gas += V * U[k];
            double Uc[NV] = {0};
            for (int v = 0; v < cx->nv; ++v) Uc[v] = U[v * plane + k];
            prim_t w;
            cons_to_prim(Uc, &w);
            double pv = Uc[4] * RGAS_VAP * w.T;
            if (pv < PV_FLOOR) pv = PV_FLOOR;
            double l = log(pv) - or_ln_psat_liq(w.T);
            if (l > lnS) lnS = l;
        }
    out[0] = water; out[1] = lnS; out[2] = nice; out[3] = gas;
}
