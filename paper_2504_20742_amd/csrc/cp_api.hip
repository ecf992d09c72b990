// cp_api.hip -- host runtime and C ABI of the contrail finite-volume step.
//
// Owns the per-case state: mesh metrics (Sec. 4.1 axisymmetric mesh, tensor
// product of a geometrically stretched axial and a sinh-clustered radial
// distribution), inflow / far-field states, stage buffers, the device-resident
// time step, the captured step graph and the tile-shape autotuner.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/contrail.h"
#include "cp_internal.hpp"

using namespace cp;

enum { M_XC, M_RC, M_INV_DXF, M_INV_DRF, M_INV_D2X, M_INV_D2R, M_LM2, M_INV_DX, M_RFA, M_INVV_R, M_INV_RC,
       M_INV_RF, M_AXF, M_INVVX, M_COUNT };

struct cp_ctx {
    int precision = CP_FP64;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    cp_mesh mesh{};
    cp_case cs{};
    int nx = 0, nr = 0;
    long plane = 0;
    std::vector<double> xf, rf, xc, rc, dx, dr;     // host mesh
    std::vector<double> ax;                         // quasi-1D duct areas at the x faces
    double *ptab = nullptr;                         // water property table (device), or null
    bool drift = false;                             // particles drift against the gas
    int nv = NVAR;                                  // variables per cell: NVAR, or NVAR_BI (two liquid populations)
    double *rfa_d = nullptr, *invVr_d = nullptr;    // double r-face areas and 1/(r_c dr) for the drift
    std::vector<void *> allocs;                     // device memory owned by the context
    double *inflow = nullptr, *ambient = nullptr, *vol = nullptr;
    double *xc_d = nullptr, *rc_d = nullptr, *inv_dx_d = nullptr, *inv_dr_d = nullptr;
    void *met[M_COUNT] = {};                        // metric arrays in the storage precision
    void *Ua = nullptr, *Ub = nullptr;
    double *dt_d = nullptr, *t_d = nullptr, *diag_d = nullptr, *Qsur = nullptr;
    unsigned long long *acc_d = nullptr, *nsub_d = nullptr;
    double *cfl_bm = nullptr;   // per-workgroup minima of the CFL kernel
    int cfl_nb = 0;
    int *flag_d = nullptr;
    int *act_count = nullptr, *act_list = nullptr;  // source-active cells per stage
    unsigned *tmask[3] = {};                        // tile masks of U, Ua, Ub (non-zero scalars)
    unsigned ghost_bits = 0;                        // non-zero scalars of the inflow / far-field states
    bool masks_off = false;                         // cp_set_tile_masks(ctx, 0)
    bool sur_ready = false;                         // a network snapshot is attached
    SurNorm nm{};
    int *sur_cnt = nullptr, *sur_cells = nullptr, *fb_list = nullptr;
    unsigned long long *sur_tot = nullptr;   // running totals of network / fallback cells
    int *src_cnt = nullptr, *src_list = nullptr;   // active cells of a cp_source call
    float *sur_Y = nullptr;      // network outputs of the gated rows
    uint16_t *sur_w = nullptr;   // packed snapshot of the attached network's weights
    float *sur_b = nullptr;
    SourceParams sp{};
    int qmode = CP_Q_EXACT;
    int tx = 0, ty = 0;                             // 0: autotune on first use
    hipGraphExec_t graph = nullptr, graph_m = nullptr, graph_k = nullptr;   // 1, kStepsMid, kStepsPerGraph steps
    void *graph_U = nullptr;
    double Y_amb = 0, u_amb = 0;
    std::string err;
};

namespace {

constexpr int kStepsPerGraph = 32, kStepsMid = 8;

// Release the captured step graphs (after any change of what a step launches).
void drop_graphs(cp_ctx *c)
{
    if (c->graph) hipGraphExecDestroy(c->graph);
    if (c->graph_m) hipGraphExecDestroy(c->graph_m);
    if (c->graph_k) hipGraphExecDestroy(c->graph_k);
    c->graph = c->graph_m = c->graph_k = nullptr;
}

int fail(cp_ctx *c, int code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(c, x)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (x);                                                                           \
        if (e_ != hipSuccess) return fail((c), CP_EHIP, std::string(#x ": ") + hipGetErrorString(e_)); \
    } while (0)

template <class T> T *dalloc(cp_ctx *c, size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    c->allocs.push_back(p);
    return (T *)p;
}

// ---------------------------------------------------------------- gas model (host side)
constexpr double hRa = 287.0, hCpa = 1004.5, hRv = 461.52, hCpv = 1846.08, hTref = 273.15, hLv0 = 2.5008e6;
double h_R(double Y) { return (1.0 - Y) * hRa + Y * hRv; }
double h_cp(double Y) { return (1.0 - Y) * hCpa + Y * hCpv; }
double h_cv(double Y) { return h_cp(Y) - h_R(Y); }
double h_ln_psat_ice(double T)
{
    return -6024.5282 / T + 24.7219 + 1.0613868e-2 * T - 1.3198825e-5 * T * T - 0.49382577 * log(T) + log(100.0);
}

// Water property table: on nodes T0 + k h the value, slope and half curvature of
// ln p_sat over liquid and over ice (Sonntag) and of the IAPWS surface tension
// (zero at and above the critical point), from the closed forms' analytic
// derivatives.
constexpr double kTabT0 = 150.0, kTabT1 = 700.0;

void sonntag_taylor(const double *k, double T, double *f)   // k: a, b, c, d, e
{
    f[0] = k[0] / T + k[1] + k[2] * T + k[3] * T * T + k[4] * log(T) + log(100.0);
    f[1] = -k[0] / (T * T) + k[2] + 2.0 * k[3] * T + k[4] / T;
    f[2] = k[0] / (T * T * T) + k[3] - 0.5 * k[4] / (T * T);
}

void sigma_taylor(double T, double *f)
{
    const double B = 0.2358, m = 1.256, Tc = 647.096, t = 1.0 - T / Tc;
    if (!(t > 0.0)) {
        f[0] = f[1] = f[2] = 0.0;
        return;
    }
    // sigma(t) = B (t^m - 0.625 t^(m+1)); d/dT = -(1/Tc) d/dt
    f[0] = B * pow(t, m) * (1.0 - 0.625 * t);
    f[1] = -B * (m * pow(t, m - 1.0) - 0.625 * (m + 1.0) * pow(t, m)) / Tc;
    f[2] = 0.5 * B * (m * (m - 1.0) * pow(t, m - 2.0) - 0.625 * (m + 1.0) * m * pow(t, m - 1.0)) / (Tc * Tc);
}

std::vector<double> property_table(double h, int n)
{
    static const double liq[5] = {-6096.9385, 16.635794, -2.711193e-2, 1.673952e-5, 2.433502};
    static const double ice[5] = {-6024.5282, 24.7219, 1.0613868e-2, -1.3198825e-5, -0.49382577};
    std::vector<double> t((size_t)n * 9);
    for (int k = 0; k < n; ++k) {
        const double T = kTabT0 + k * h;
        sonntag_taylor(liq, T, &t[9 * (size_t)k]);
        sonntag_taylor(ice, T, &t[9 * (size_t)k + 3]);
        sigma_taylor(T, &t[9 * (size_t)k + 6]);
    }
    return t;
}

// Conserved state of a jet or of the free stream: pressure-matched, no radial
// velocity, no condensate; soot number n_soot.
void stream_cons(double p, double T, double u, double Y, double nsoot, double *U)
{
    const double rho = p / (h_R(Y) * T);
    const double e = h_cv(Y) * T - (1.0 - Y) * hCpa * hTref + Y * (hLv0 - hCpv * hTref);
    for (int v = 0; v < NVAR; ++v) U[v] = 0.0;
    U[0] = rho;
    U[1] = rho * u;
    U[3] = rho * (e + 0.5 * u * u);
    U[4] = rho * Y;
    U[13] = nsoot;
}

void build_mesh(cp_ctx *c)
{
    const cp_mesh &m = c->mesh;
    const int nx = m.nx, nr = m.nr;
    c->xf.assign(nx + 1, 0.0);
    c->rf.assign(nr + 1, 0.0);
    for (int i = 0; i <= nx; ++i)
        c->xf[i] = m.sx_ratio == 1.0 ? m.Lx * i / nx
                                     : m.Lx * (pow(m.sx_ratio, i) - 1.0) / (pow(m.sx_ratio, nx) - 1.0);
    c->xf[nx] = m.Lx;
    if (m.r_cluster > 0.0) {
        // interior-point clustering: r = D (1 + sinh(b (eta - A)) / sinh(b A))
        const double b = m.beta_r, D = m.r_cluster, H = m.Lr;
        const double A = 0.5 / b * log((1.0 + (exp(b) - 1.0) * D / H) / (1.0 + (exp(-b) - 1.0) * D / H));
        for (int j = 0; j <= nr; ++j) {
            const double eta = (double)j / nr;
            c->rf[j] = D * (1.0 + sinh(b * (eta - A)) / sinh(b * A));
        }
    } else {
        for (int j = 0; j <= nr; ++j) c->rf[j] = m.Lr * j / nr;
    }
    c->rf[0] = 0.0;
    c->rf[nr] = m.Lr;
    c->xc.assign(nx + 4, 0.0);
    c->rc.assign(nr + 4, 0.0);
    c->dx.assign(nx, 0.0);
    c->dr.assign(nr, 0.0);
    for (int i = 0; i < nx; ++i) {
        c->dx[i] = c->xf[i + 1] - c->xf[i];
        c->xc[i + 2] = 0.5 * (c->xf[i] + c->xf[i + 1]);
    }
    for (int j = 0; j < nr; ++j) {
        c->dr[j] = c->rf[j + 1] - c->rf[j];
        c->rc[j + 2] = 0.5 * (c->rf[j] + c->rf[j + 1]);
    }
    for (int g = 0; g < 2; ++g) {   // ghost centres mirrored about the boundary faces
        c->xc[1 - g] = 2.0 * c->xf[0] - c->xc[2 + g];
        c->xc[nx + 2 + g] = 2.0 * c->xf[nx] - c->xc[nx + 1 - g];
        c->rc[1 - g] = 2.0 * c->rf[0] - c->rc[2 + g];
        c->rc[nr + 2 + g] = 2.0 * c->rf[nr] - c->rc[nr + 1 - g];
    }
}

template <class T> int upload_as(cp_ctx *c, const std::vector<double> &h, void **slot)
{
    std::vector<T> t(h.begin(), h.end());
    T *d = dalloc<T>(c, t.size());
    if (!d) return fail(c, CP_ENOMEM, "metric allocation");
    HIPCHK(c, hipMemcpy(d, t.data(), t.size() * sizeof(T), hipMemcpyHostToDevice));
    *slot = d;
    return CP_OK;
}

template <class R> int upload_metrics(cp_ctx *c)
{
    const int nx = c->nx, nr = c->nr;
    const bool axi = c->mesh.geom == CP_GEOM_AXI;
    const bool q1d = c->mesh.geom == CP_GEOM_QUASI1D;
    auto XC = [&](int i) { return c->xc[i + 2]; };
    auto RC = [&](int j) { return c->rc[j + 2]; };
    std::vector<double> inv_dxf(nx + 1), inv_drf(nr + 1), inv_d2x(nx + 2), inv_d2r(nr + 2), lm2(nx + 2),
        inv_dx(nx), rfa(nr + 1), invV_r(nr), inv_rc(nr + 2), inv_rf(nr + 1);
    for (int i = 0; i <= nx; ++i) inv_dxf[i] = 1.0 / (XC(i) - XC(i - 1));
    for (int j = 0; j <= nr; ++j) inv_drf[j] = 1.0 / (RC(j) - RC(j - 1));
    const double delta0 = c->cs.delta0_frac * c->cs.R_core;
    for (int i = -1; i <= nx; ++i) {
        inv_d2x[i + 1] = 1.0 / (XC(i + 1) - XC(i - 1));
        const double lm = c->cs.kappa_m * (delta0 + c->cs.s_delta * XC(i));
        lm2[i + 1] = lm * lm;
    }
    for (int j = -1; j <= nr; ++j) {
        inv_d2r[j + 1] = 1.0 / (RC(j + 1) - RC(j - 1));
        inv_rc[j + 1] = axi ? 1.0 / RC(j) : 0.0;
    }
    for (int i = 0; i < nx; ++i) inv_dx[i] = 1.0 / c->dx[i];
    for (int j = 0; j <= nr; ++j) {
        rfa[j] = axi ? c->rf[j] : (q1d ? 0.0 : 1.0);   // the duct has no r faces
        inv_rf[j] = (axi && c->rf[j] > 0.0) ? 1.0 / c->rf[j] : 0.0;
    }
    for (int j = 0; j < nr; ++j) invV_r[j] = axi ? 1.0 / (RC(j) * c->dr[j]) : 1.0 / c->dr[j];
    // duct: x-face areas and 1 / V_i with V_i = 0.5 (A_w + A_e) dx (unit areas and
    // 1/dx elsewhere; the stage kernel reads them only for the duct)
    std::vector<double> axf(nx + 1, 1.0), invVx(inv_dx);
    if (q1d) {
        axf = c->ax;
        for (int i = 0; i < nx; ++i) invVx[i] = 1.0 / (0.5 * (c->ax[i] + c->ax[i + 1]) * c->dx[i]);
    }
    const std::vector<double> *src[M_COUNT] = {&c->xc, &c->rc, &inv_dxf, &inv_drf, &inv_d2x, &inv_d2r, &lm2,
                                               &inv_dx, &rfa, &invV_r, &inv_rc, &inv_rf, &axf, &invVx};
    for (int k = 0; k < M_COUNT; ++k) {
        int r = upload_as<R>(c, *src[k], &c->met[k]);
        if (r) return r;
    }
    // double copies for the CFL reduction and the diagnostics
    void *p;
    int r;
    if ((r = upload_as<double>(c, c->xc, &p))) return r;
    c->xc_d = (double *)p;
    if ((r = upload_as<double>(c, c->rc, &p))) return r;
    c->rc_d = (double *)p;
    std::vector<double> idx(nx), idr(nr), vol((size_t)nx * nr);
    for (int i = 0; i < nx; ++i) idx[i] = 1.0 / c->dx[i];
    for (int j = 0; j < nr; ++j) idr[j] = q1d ? 0.0 : 1.0 / c->dr[j];   // the duct has no r direction
    for (int j = 0; j < nr; ++j)
        for (int i = 0; i < nx; ++i)
            vol[(size_t)j * nx + i] = q1d ? 0.5 * (c->ax[i] + c->ax[i + 1]) * c->dx[i]
                                          : (axi ? RC(j) : 1.0) * c->dr[j] * c->dx[i];
    if ((r = upload_as<double>(c, idx, &p))) return r;
    c->inv_dx_d = (double *)p;
    if ((r = upload_as<double>(c, idr, &p))) return r;
    c->inv_dr_d = (double *)p;
    if ((r = upload_as<double>(c, vol, &p))) return r;
    c->vol = (double *)p;
    if ((r = upload_as<double>(c, rfa, &p))) return r;
    c->rfa_d = (double *)p;
    if ((r = upload_as<double>(c, invV_r, &p))) return r;
    c->invVr_d = (double *)p;
    return CP_OK;
}

template <class R> Metrics<R> metrics(const cp_ctx *c)
{
    Metrics<R> m;
    m.xc = (const R *)c->met[M_XC];
    m.rc = (const R *)c->met[M_RC];
    m.inv_dxf = (const R *)c->met[M_INV_DXF];
    m.inv_drf = (const R *)c->met[M_INV_DRF];
    m.inv_d2x = (const R *)c->met[M_INV_D2X];
    m.inv_d2r = (const R *)c->met[M_INV_D2R];
    m.lm2 = (const R *)c->met[M_LM2];
    m.inv_dx = (const R *)c->met[M_INV_DX];
    m.rfa = (const R *)c->met[M_RFA];
    m.invV_r = (const R *)c->met[M_INVV_R];
    m.inv_rc = (const R *)c->met[M_INV_RC];
    m.inv_rf = (const R *)c->met[M_INV_RF];
    m.axf = (const R *)c->met[M_AXF];
    m.invVx = (const R *)c->met[M_INVVX];
    return m;
}

BcInfo bcinfo(const cp_ctx *c)
{
    BcInfo b;
    b.nx = c->nx;
    b.nr = c->nr;
    b.geom = c->mesh.geom;
    b.bc_xlo = c->mesh.bc_xlo;
    b.bc_xhi = c->mesh.bc_xhi;
    b.bc_rlo = c->mesh.bc_rlo;
    b.bc_rhi = c->mesh.bc_rhi;
    b.inflow = c->inflow;
    b.ambient = c->ambient;
    return b;
}

// Tile masks of the passive scalars: one per state buffer (the caller's U, and the
// two stage buffers), for the current tile shape.  Off with the drift, whose pass
// moves particles after the stage kernel without widening the masks.
bool masks_on(const cp_ctx *c) { return !c->drift && !c->masks_off && c->tx > 0 && c->tmask[0]; }
unsigned *mask_of(const cp_ctx *c, const void *p)
{
    return p == c->Ua ? c->tmask[1] : (p == c->Ub ? c->tmask[2] : c->tmask[0]);
}
TileMask tile_mask(const cp_ctx *c, const void *Uin, const void *Uout, int stage, const void *Un = nullptr)
{
    TileMask m{};
    if (!masks_on(c)) return m;
    m.in = Uin ? mask_of(c, Uin) : nullptr;
    m.un = stage > 0 && Un ? mask_of(c, Un) : nullptr;
    m.out = stage >= 0 && Uout ? mask_of(c, Uout) : nullptr;
    m.tx = c->tx;
    m.ty = c->ty;
    m.gx = (c->nx + c->tx - 1) / c->tx;
    m.gy = (c->nr + c->ty - 1) / c->ty;
    m.nx = c->nx;
    m.ghost = c->ghost_bits;
    return m;
}
// Masks of the caller's state U (its contents may have changed since the last call),
// and all-ones masks of the two stage buffers: a stage skips the store of a zero scalar
// where its output buffer's mask says that the tile already holds zero, and the stage
// buffers may have been written since under another tile shape or with the masks off.
int mask_seed(cp_ctx *c, const void *U, hipStream_t s)
{
    if (!masks_on(c)) return CP_OK;
    hipError_t e = c->precision == CP_FP64
                       ? launch_tile_mask<double>((const double *)U, c->plane, c->nx, c->nr, c->nv, c->tx, c->ty,
                                                  c->tmask[0], c->tmask[1], c->tmask[2], s)
                       : launch_tile_mask<float>((const float *)U, c->plane, c->nx, c->nr, c->nv, c->tx, c->ty,
                                                 c->tmask[0], c->tmask[1], c->tmask[2], s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("tile mask: ") + hipGetErrorString(e));
    return CP_OK;
}

template <class R>
StageArgs<R> stage_args(const cp_ctx *c, const void *Uin, const void *Un, void *Uout, int stage, double dt,
                        const double *dt_dev)
{
    StageArgs<R> a;
    a.Uin = (const R *)Uin;
    a.Un = (const R *)Un;
    a.Uout = (R *)Uout;
    a.dt_dev = dt_dev;
    a.dt = dt;
    a.plane = c->plane;
    a.stage = stage;
    a.qmode = c->qmode;
    a.bc = bcinfo(c);
    a.m = metrics<R>(c);
    a.sp = c->sp;
    a.sp.enabled = (c->cs.phase_change != 0 && c->qmode != CP_Q_OFF) ? 1 : 0;
    a.flag = c->flag_d;
    a.pref = c->cs.p_amb;
    a.active_count = c->act_count + (stage < 0 ? 0 : stage);
    a.active_list = c->act_list;
    const bool sur = c->qmode == CP_Q_SURROGATE && c->sur_ready && stage >= 0;
    a.sur_cnt = sur ? c->sur_cnt : nullptr;
    a.sur_tot = c->sur_tot;
    a.mask = tile_mask(c, Uin, Uout, stage, Un);
    return a;
}

template <class R>
SourceFixArgs<R> fix_args(const cp_ctx *c, const void *Uin, void *Uout, int stage, double dt, const double *dt_dev)
{
    SourceFixArgs<R> a;
    a.Uin = (const R *)Uin;
    a.Uout = (R *)Uout;
    a.dt_dev = dt_dev;
    a.dt = dt;
    a.plane = c->plane;
    a.stage = stage;
    a.count = c->act_count + stage;
    a.list = c->act_list;
    a.next_count = c->act_count + (stage + 1) % 3;
    a.sp = c->sp;
    a.sp.enabled = 1;
    a.flag = c->flag_d;
    a.nsub = c->nsub_d;
    a.mask = tile_mask(c, nullptr, Uout, stage);
    return a;
}

template <class R>
SurArgs<R> sur_args(const cp_ctx *c, const void *Uin, void *Uout, int stage, double dt, const double *dt_dev)
{
    SurArgs<R> a;
    a.Uin = (const R *)Uin;
    a.Uout = (R *)Uout;
    a.dt_dev = dt_dev;
    a.dt = dt;
    a.plane = c->plane;
    a.stage = stage;
    a.count = c->act_count + stage;
    a.list = c->act_list;
    a.cnt = c->sur_cnt;
    a.mlp_cells = c->sur_cells;
    a.fb_list = c->fb_list;
    a.Y = c->sur_Y;
    a.nm = c->nm;
    a.flag = c->flag_d;
    a.q_only = 0;
    a.mask = tile_mask(c, nullptr, Uout, stage);
    return a;
}

FusedNet sur_net(const cp_ctx *c)
{
    return FusedNet{c->sur_w, c->sur_w + kFusedW1, c->sur_w + kFusedW1 + kFusedW2, c->sur_b, c->sur_b + 256,
                    c->sur_b + 512};
}

// Learned source for the active cells of a stage: split them (network / exact) and run
// the network on its rows in one launch, then decode + project + apply, exact source
// for the rest.
template <class R>
int surrogate_stage(cp_ctx *c, const void *Uin, void *Uout, int stage, double dt, const double *dt_dev, hipStream_t s)
{
    // the stage kernel has already folded and cleared the counters
    SurArgs<R> a = sur_args<R>(c, Uin, Uout, stage, dt, dt_dev);
    hipError_t e = launch_sur_gate_net<R>(a, sur_net(c), c->sur_Y, c->plane, s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("surrogate gate and network: ") + hipGetErrorString(e));
    const SourceFixArgs<R> f = fix_args<R>(c, Uin, Uout, stage, dt, dt_dev);
    e = launch_sur_finish<R>(a, f.sp, f.next_count, c->nsub_d, c->plane, s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("surrogate finish: ") + hipGetErrorString(e));
    return CP_OK;
}

// cp_source in surrogate mode: Q already holds the exact source of every cell; the
// network's (closed) source replaces it in the cells the gate hands to the network.
template <class R> int surrogate_source(cp_ctx *c, const void *U, double dt, void *Q)
{
    hipStream_t s = c->stream;
    HIPCHK(c, hipMemsetAsync(c->src_cnt, 0, sizeof(int), s));
    hipError_t e = launch_active_list<R>((const R *)U, c->plane, c->src_cnt, c->src_list, s);
    SurArgs<R> a = sur_args<R>(c, U, Q, 0, dt, nullptr);
    a.count = c->src_cnt;
    a.list = c->src_list;
    a.q_only = 1;
    a.mask = TileMask{};
    if (e == hipSuccess) e = launch_sur_reset(c->sur_cnt, c->sur_tot, s);
    if (e == hipSuccess) e = launch_sur_gate_net<R>(a, sur_net(c), c->sur_Y, c->plane, s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("surrogate gate and network: ") + hipGetErrorString(e));
    SourceParams sp = c->sp;
    sp.enabled = 1;
    e = launch_sur_finish<R>(a, sp, nullptr, nullptr, c->plane, s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("surrogate finish: ") + hipGetErrorString(e));
    return CP_OK;
}

int surrogate_any(cp_ctx *c, const void *Uin, void *Uout, int stage, double dt, const double *dt_dev, hipStream_t s)
{
    return c->precision == CP_FP64 ? surrogate_stage<double>(c, Uin, Uout, stage, dt, dt_dev, s)
                                   : surrogate_stage<float>(c, Uin, Uout, stage, dt, dt_dev, s);
}

int stage_any(cp_ctx *c, const void *Uin, const void *Un, void *Uout, int stage, double dt, const double *dt_dev,
              hipStream_t s)
{
    hipError_t e;
    if (c->precision == CP_FP64)
        e = launch_stage<double>(stage_args<double>(c, Uin, Un, Uout, stage, dt, dt_dev), c->tx, c->ty, c->nv, s);
    else
        e = launch_stage<float>(stage_args<float>(c, Uin, Un, Uout, stage, dt, dt_dev), c->tx, c->ty, c->nv, s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("stage launch: ") + hipGetErrorString(e));
    if (c->drift) {
        auto drift = [&](auto *tag) {
            using R = std::remove_pointer_t<decltype(tag)>;
            DriftArgs<R> d;
            d.Uin = (const R *)Uin;
            d.Uout = (R *)Uout;
            d.dt_dev = dt_dev;
            d.dt = dt;
            d.plane = c->plane;
            d.stage = stage;
            d.bc = bcinfo(c);
            d.xc = c->xc_d;
            d.rc = c->rc_d;
            d.inv_dx = c->inv_dx_d;
            d.rfa = c->rfa_d;
            d.invV_r = c->invVr_d;
            d.flag = c->flag_d;
            return launch_drift<R>(d, s);
        };
        e = c->precision == CP_FP64 ? drift((double *)nullptr) : drift((float *)nullptr);
        if (e != hipSuccess) return fail(c, CP_EHIP, std::string("drift launch: ") + hipGetErrorString(e));
    }
    const bool src = stage >= 0 && c->cs.phase_change != 0 && c->qmode != CP_Q_OFF;
    if (!src) return CP_OK;
    if (c->qmode == CP_Q_SURROGATE) return surrogate_any(c, Uin, Uout, stage, dt, dt_dev, s);
    if (c->precision == CP_FP64)
        e = launch_source_fix<double>(fix_args<double>(c, Uin, Uout, stage, dt, dt_dev), c->plane, c->nv, s);
    else
        e = launch_source_fix<float>(fix_args<float>(c, Uin, Uout, stage, dt, dt_dev), c->plane, c->nv, s);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("source launch: ") + hipGetErrorString(e));
    return CP_OK;
}

// Arguments of the CFL reduction over U for context c (the running minimum and
// the per-workgroup array are the caller's).
template <class R> CflArgs<R> cfl_args(const cp_ctx *c, const void *U)
{
    CflArgs<R> a;
    a.U = (const R *)U;
    a.plane = c->plane;
    a.bc = bcinfo(c);
    a.xc = c->xc_d;
    a.rc = c->rc_d;
    a.inv_dx = c->inv_dx_d;
    a.inv_dr = c->inv_dr_d;
    const bool f32 = sizeof(R) == 4;
    a.f_d2x = f32 ? (const float *)c->met[M_INV_D2X] : nullptr;
    a.f_d2r = f32 ? (const float *)c->met[M_INV_D2R] : nullptr;
    a.f_lm2 = f32 ? (const float *)c->met[M_LM2] : nullptr;
    a.f_idx = f32 ? (const float *)c->met[M_INV_DX] : nullptr;
    a.kappa_m = c->cs.kappa_m;
    a.delta0 = c->cs.delta0_frac * c->cs.R_core;
    a.s_delta = c->cs.s_delta;
    a.acc = nullptr;
    a.block_min = nullptr;
    return a;
}

int cfl_any(cp_ctx *c, const void *U, hipStream_t s)
{
    hipError_t e;
    auto fill = [&](auto *tag) {
        using R = std::remove_pointer_t<decltype(tag)>;
        CflArgs<R> a = cfl_args<R>(c, U);
        a.acc = c->acc_d;
        a.block_min = c->cfl_bm;
        return launch_cfl<R>(a, s);
    };
    e = c->precision == CP_FP64 ? fill((double *)nullptr) : fill((float *)nullptr);
    if (e != hipSuccess) return fail(c, CP_EHIP, std::string("cfl launch: ") + hipGetErrorString(e));
    return CP_OK;
}

int check_flag(cp_ctx *c)
{
    int flag = 0;
    HIPCHK(c, hipMemcpyAsync(&flag, c->flag_d, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (flag & 1) return fail(c, CP_ENONFINITE, "a stage wrote a non-finite value");
    return CP_OK;
}

// Pick the fastest tile shape for this mesh and precision: time the transport
// residual (reads U, writes a private buffer) for every built shape.  All shapes give bit-identical
// results, so the choice only affects speed.
int autotune(cp_ctx *c, const void *U)
{
    if (c->tx) return CP_OK;
    if (c->nv == NVAR_BI) {   // two liquid populations: the one built shape
        c->tx = 32;
        c->ty = 8;
        return CP_OK;
    }
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    // Shapes are tried in the built order; a later shape must beat the best so far by
    // more than 5% to replace it, so that run-to-run noise does not flip the choice.
    float best = 1e30f;
    int btx = 32, bty = 8;
    for (auto &sh : tile_list()) {
        c->tx = sh.first;
        c->ty = sh.second;
        int r = mask_seed(c, U, c->stream);
        if (r) return r;
        r = stage_any(c, U, U, c->Ua, -1, 0.0, nullptr, c->stream);
        if (r) return r;
        HIPCHK(c, hipEventRecord(e0, c->stream));
        for (int k = 0; k < 6; ++k) {
            r = stage_any(c, U, U, c->Ua, -1, 0.0, nullptr, c->stream);
            if (r) return r;
        }
        HIPCHK(c, hipEventRecord(e1, c->stream));
        HIPCHK(c, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
        if (ms < 0.95f * best) {
            best = ms;
            btx = sh.first;
            bty = sh.second;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c->tx = btx;
    c->ty = bty;
    int zero = 0;
    HIPCHK(c, hipMemcpyAsync(c->flag_d, &zero, sizeof(int), hipMemcpyHostToDevice, c->stream));
    return CP_OK;
}

int enqueue_step(cp_ctx *c, void *U, double dt, const double *dt_dev, hipStream_t s)
{
    int r;
    if ((r = stage_any(c, U, U, c->Ua, 0, dt, dt_dev, s))) return r;
    if ((r = stage_any(c, c->Ua, U, c->Ub, 1, dt, dt_dev, s))) return r;
    return stage_any(c, c->Ub, U, U, 2, dt, dt_dev, s);
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

int cp_create(const cp_mesh *mesh, const cp_case *cs, int precision, void *hip_stream, cp_ctx **out)
{
    if (!mesh || !cs || !out) return CP_EINVAL;
    *out = nullptr;
    const bool q1d = mesh->geom == CP_GEOM_QUASI1D;
    if (mesh->nx < 2 || (q1d ? mesh->nr != 1 : mesh->nr < 2) || !(mesh->Lx > 0) || !(mesh->Lr > 0))
        return CP_EINVAL;
    if ((long)mesh->nx * mesh->nr > kMaxCells) return CP_EINVAL;   // a state plane must stay below 2 GiB
    if (precision != CP_FP64 && precision != CP_MIXED) return CP_EINVAL;
    if (mesh->geom != CP_GEOM_AXI && mesh->geom != CP_GEOM_PLANAR && !q1d) return CP_EINVAL;
    if (mesh->bc_rhi == CP_BC_INFLOW || mesh->bc_xhi == CP_BC_INFLOW || mesh->bc_rlo != CP_BC_WALL) return CP_EINVAL;
    if (q1d) {
        if (!mesh->area_x || mesh->bc_rhi != CP_BC_WALL) return CP_EINVAL;
        for (int i = 0; i <= mesh->nx; ++i)
            if (!std::isfinite(mesh->area_x[i]) || !(mesh->area_x[i] > 0.0)) return CP_EINVAL;
    }
    if (!(mesh->sx_ratio > 0) || cs->n_sub_max < 1 || !(cs->cfl > 0)) return CP_EINVAL;
    cp_ctx *c = new cp_ctx();
    c->precision = precision;
    c->stream = (hipStream_t)hip_stream;
    c->mesh = *mesh;
    c->mesh.area_x = nullptr;   // the areas are copied; the caller's array is not kept
    if (q1d) c->ax.assign(mesh->area_x, mesh->area_x + mesh->nx + 1);
    c->cs = *cs;
    c->nx = mesh->nx;
    c->nr = mesh->nr;
    c->plane = (long)mesh->nx * mesh->nr;
    build_mesh(c);

    // ambient and inflow states (Sec. 4.1 streams)
    const double pv = cs->RH_ice * exp(h_ln_psat_ice(cs->T_amb));
    const double rho_v = pv / (hRv * cs->T_amb), rho_a = (cs->p_amb - pv) / (hRa * cs->T_amb);
    c->Y_amb = rho_v / (rho_a + rho_v);
    const double cpA = h_cp(c->Y_amb), RA = h_R(c->Y_amb);
    c->u_amb = cs->mach_amb * sqrt(cpA / (cpA - RA) * RA * cs->T_amb);
    std::vector<double> amb(NVAR), inflow((size_t)NVAR * c->nr);
    stream_cons(cs->p_amb, cs->T_amb, c->u_amb, c->Y_amb, 0.0, amb.data());
    const double Yb = cs->Y_byp < 0.0 ? c->Y_amb : cs->Y_byp;
    for (int j = 0; j < c->nr; ++j) {
        const double r = c->rc[j + 2];
        double *U = inflow.data() + (size_t)NVAR * j;
        if (r < cs->R_core) stream_cons(cs->p_amb, cs->T_core, cs->u_core, cs->Y_core, cs->n_soot, U);
        else if (r < cs->R_fan) stream_cons(cs->p_amb, cs->T_byp, cs->u_byp, Yb, 0.0, U);
        else for (int v = 0; v < NVAR; ++v) U[v] = amb[v];
    }
    for (int v = 5; v < NVAR; ++v) {   // scalars a ghost cell can take from a boundary state
        if (amb[v] != 0.0) c->ghost_bits |= 1u << v;
        for (int j = 0; j < c->nr; ++j)
            if (inflow[(size_t)NVAR * j + v] != 0.0) c->ghost_bits |= 1u << v;
    }

    // phase-change constants evaluated once on the host
    const double ct = cos(cs->theta_deg * M_PI / 180.0);
    c->sp.f_theta = 0.25 * (2.0 + ct) * (1.0 - ct) * (1.0 - ct);
    const double lsg = log(cs->sigma_g_soot);
    c->sp.het_freeze = cs->k_imm * cs->n_s * (4.0 * M_PI * cs->r_g_soot * cs->r_g_soot * exp(2.0 * lsg * lsg));
    const double NA = 6.02214076e23, Mw = 0.018015268;
    c->sp.cnt_const = 1.0 * sqrt(2.0 * NA * NA * NA / (M_PI * Mw * Mw * Mw)) / 1000.0;
    for (int k = 0; k < 4; ++k) c->sp.ice_ratio[k] = pow(1000.0 / 917.0, k / 3.0);
    c->sp.n_sub_max = cs->n_sub_max;
    c->sp.enabled = cs->phase_change ? 1 : 0;

    int r = CP_OK;
    auto bail = [&](int code) {
        std::string msg = c->err;
        cp_destroy(c);
        return code;
    };
    if (!c->stream) {
        // graph capture needs a non-null stream; the context still launches on the
        // caller's stream
    }
    if (hipStreamCreate(&c->cap_stream) != hipSuccess) return bail(CP_EHIP);
    const size_t esz = precision == CP_FP64 ? sizeof(double) : sizeof(float);
    c->inflow = dalloc<double>(c, inflow.size());
    c->ambient = dalloc<double>(c, NVAR);
    // stage buffers sized for two liquid populations, so that cp_set_bimodal needs no allocation
    c->Ua = dalloc<char>(c, esz * NVAR_BI * c->plane);
    c->Ub = dalloc<char>(c, esz * NVAR_BI * c->plane);
    c->dt_d = dalloc<double>(c, 1);
    c->t_d = dalloc<double>(c, 1);
    c->diag_d = dalloc<double>(c, 8);
    c->acc_d = dalloc<unsigned long long>(c, 1);
    c->cfl_nb = ((c->nx + kCflBX - 1) / kCflBX) * ((c->nr + kCflBY * kCflRows - 1) / (kCflBY * kCflRows));
    c->cfl_bm = dalloc<double>(c, c->cfl_nb);
    c->nsub_d = dalloc<unsigned long long>(c, 1);
    c->flag_d = dalloc<int>(c, 1);
    c->act_count = dalloc<int>(c, 4);
    c->act_list = dalloc<int>(c, c->plane);
    // tile masks: enough words for the smallest built tile (16 x 4 cells)
    const size_t mwords = (size_t)((c->nx + 15) / 16) * ((c->nr + 3) / 4);
    for (int k = 0; k < 3; ++k) c->tmask[k] = dalloc<unsigned>(c, mwords);
    if (!c->tmask[0] || !c->tmask[1] || !c->tmask[2] || !c->act_count || !c->act_list || !c->inflow || !c->ambient || !c->Ua || !c->Ub || !c->dt_d || !c->t_d || !c->diag_d || !c->acc_d || !c->cfl_bm ||
        !c->nsub_d || !c->flag_d)
        return bail(CP_ENOMEM);
    if (hipMemcpy(c->inflow, inflow.data(), inflow.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->ambient, amb.data(), NVAR * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return bail(CP_EHIP);
    r = precision == CP_FP64 ? upload_metrics<double>(c) : upload_metrics<float>(c);
    if (r) return bail(r);
    if (hipMemset(c->flag_d, 0, sizeof(int)) != hipSuccess || hipMemset(c->t_d, 0, sizeof(double)) != hipSuccess ||
        hipMemset(c->nsub_d, 0, sizeof(unsigned long long)) != hipSuccess ||
        hipMemset(c->act_count, 0, 4 * sizeof(int)) != hipSuccess)
        return bail(CP_EHIP);
    if (launch_acc_reset(c->acc_d, c->stream) != hipSuccess) return bail(CP_EHIP);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(CP_EHIP);
    *out = c;
    return CP_OK;
}

void cp_destroy(cp_ctx *c)
{
    if (!c) return;
    if (c->stream) hipStreamSynchronize(c->stream);
    else hipDeviceSynchronize();
    drop_graphs(c);
    for (void *p : c->allocs)
        if (p) hipFree(p);
    if (c->ptab) hipFree(c->ptab);
    if (c->cap_stream) hipStreamDestroy(c->cap_stream);
    delete c;
}

int cp_init(cp_ctx *c, void *U)
{
    if (!c || !U) return fail(c, CP_EINVAL, "null argument");
    hipError_t e = c->precision == CP_FP64
                       ? launch_init<double>((double *)U, c->inflow, c->nx, c->nr, c->nv, c->stream)
                       : launch_init<float>((float *)U, c->inflow, c->nx, c->nr, c->nv, c->stream);
    if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
    return CP_OK;
}

int cp_residual(cp_ctx *c, const void *U, void *R)
{
    if (!c || !U || !R) return fail(c, CP_EINVAL, "null argument");
    if (U == R) return fail(c, CP_EINVAL, "U and R must not alias");
    if (!c->tx) {
        c->tx = 32;
        c->ty = 8;
    }
    int r = mask_seed(c, U, c->stream);
    if (r) return r;
    return stage_any(c, U, U, R, -1, 0.0, nullptr, c->stream);
}

int cp_source(cp_ctx *c, const void *U, double dt, void *Q)
{
    if (!c || !U || !Q) return fail(c, CP_EINVAL, "null argument");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, CP_EDT, "dt must be positive and finite");
    SourceParams sp = c->sp;
    sp.enabled = (c->cs.phase_change != 0 && c->qmode != CP_Q_OFF) ? 1 : 0;
    HIPCHK(c, hipMemsetAsync(c->nsub_d, 0, sizeof(unsigned long long), c->stream));
    hipError_t e = c->precision == CP_FP64
                       ? launch_source<double>((const double *)U, (double *)Q, c->plane, c->plane, dt, sp, c->nsub_d,
                                               c->nv, c->stream)
                       : launch_source<float>((const float *)U, (float *)Q, c->plane, c->plane, dt, sp, c->nsub_d,
                                              c->nv, c->stream);
    if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
    if (c->qmode == CP_Q_SURROGATE && sp.enabled)
        return c->precision == CP_FP64 ? surrogate_source<double>(c, U, dt, Q) : surrogate_source<float>(c, U, dt, Q);
    return CP_OK;
}

int cp_step(cp_ctx *c, void *U, double dt)
{
    if (!c || !U) return fail(c, CP_EINVAL, "null argument");
    if (!(dt > 0.0) || !isfinite(dt)) return fail(c, CP_EDT, "dt must be positive and finite");
    int r = autotune(c, U);
    if (r) return r;
    if ((r = mask_seed(c, U, c->stream))) return r;
    return enqueue_step(c, U, dt, nullptr, c->stream);
}

int cp_cfl_dt(cp_ctx *c, const void *U, double *dt_host)
{
    if (!c || !U || !dt_host) return fail(c, CP_EINVAL, "null argument");
    int r = cfl_any(c, U, c->stream);
    if (r) return r;
    hipError_t e = launch_cfl_finalize_blocks(c->cfl_bm, c->cfl_nb, c->cs.cfl, c->dt_d, nullptr, c->stream);
    if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
    HIPCHK(c, hipMemcpyAsync(dt_host, c->dt_d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if ((r = check_flag(c))) return r;
    if (!(*dt_host > 0.0) || !isfinite(*dt_host)) return fail(c, CP_EDT, "CFL time step not positive");
    return CP_OK;
}

// Capture `steps` consecutive steps (CFL reduction, dt, three stages each) into one
// executable graph.
int capture_steps(cp_ctx *c, void *U, int steps, hipGraphExec_t *out)
{
    hipGraph_t g;
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int r = mask_seed(c, U, c->cap_stream);   // U may have changed between replays
    for (int k = 0; k < steps && !r; ++k) {
        r = cfl_any(c, U, c->cap_stream);
        if (!r && launch_cfl_finalize_blocks(c->cfl_bm, c->cfl_nb, c->cs.cfl, c->dt_d, c->t_d, c->cap_stream) !=
                      hipSuccess)
            r = fail(c, CP_EHIP, "finalize launch");
        if (!r) r = enqueue_step(c, U, 0.0, c->dt_d, c->cap_stream);
    }
    hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    if (r) return r;
    if (ec != hipSuccess) return fail(c, CP_EHIP, std::string("capture: ") + hipGetErrorString(ec));
    hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(c, CP_EHIP, std::string("graph instantiate: ") + hipGetErrorString(ei));
    return CP_OK;
}

int cp_step_n(cp_ctx *c, void *U, int n, double *t_host)
{
    if (!c || !U || n < 0) return fail(c, CP_EINVAL, "bad argument");
    int r = autotune(c, U);
    if (r) return r;
    if (!c->graph || c->graph_U != U) {
        drop_graphs(c);
        if ((r = capture_steps(c, U, 1, &c->graph)) || (r = capture_steps(c, U, kStepsMid, &c->graph_m)) ||
            (r = capture_steps(c, U, kStepsPerGraph, &c->graph_k))) {
            drop_graphs(c);
            return r;
        }
        c->graph_U = U;
    }
    HIPCHK(c, hipMemsetAsync(c->t_d, 0, sizeof(double), c->stream));
    // whole groups of steps per replay (fewer graph boundaries), then smaller groups and
    // single steps
    for (int k = 0; k < n / kStepsPerGraph; ++k) HIPCHK(c, hipGraphLaunch(c->graph_k, c->stream));
    for (int k = 0; k < n % kStepsPerGraph / kStepsMid; ++k) HIPCHK(c, hipGraphLaunch(c->graph_m, c->stream));
    for (int k = 0; k < n % kStepsMid; ++k) HIPCHK(c, hipGraphLaunch(c->graph, c->stream));
    double t = 0.0;
    HIPCHK(c, hipMemcpyAsync(&t, c->t_d, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if ((r = check_flag(c))) return r;
    if (t_host) *t_host = t;
    return CP_OK;
}

int cp_sur_set(cp_ctx *c, cp_mlp *mlp, const float *norm, int n_norm)
{
    if (!c || !mlp || !norm) return fail(c, CP_EINVAL, "null argument");
    if (n_norm != (int)(sizeof(SurNorm) / sizeof(float))) return fail(c, CP_EINVAL, "normalisation size");
    int ni, no;
    mlp_dims(mlp, &ni, &no);
    if (ni != 17 || no != 15) return fail(c, CP_EINVAL, "network must map 17 features to 15 sources");
    // the captured step refers to the previous network and buffers: drop it first
    drop_graphs(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->sur_ready = false;
    if (c->qmode == CP_Q_SURROGATE) c->qmode = CP_Q_EXACT;   // select it again after a new network
    memcpy(&c->nm, norm, sizeof(SurNorm));
    if (!c->sur_cnt) {
        c->sur_cnt = dalloc<int>(c, 3);
        if (!c->sur_cnt) return fail(c, CP_ENOMEM, "surrogate counters");
        HIPCHK(c, hipMemset(c->sur_cnt, 0, 3 * sizeof(int)));
    }
    if (!c->sur_tot) {
        c->sur_tot = dalloc<unsigned long long>(c, 2);
        if (!c->sur_tot) return fail(c, CP_ENOMEM, "surrogate counters");
        HIPCHK(c, hipMemset(c->sur_tot, 0, 2 * sizeof(unsigned long long)));
    }
    if (!c->src_cnt && !(c->src_cnt = dalloc<int>(c, 1))) return fail(c, CP_ENOMEM, "surrogate lists");
    if (!c->sur_cells && !(c->sur_cells = dalloc<int>(c, c->plane))) return fail(c, CP_ENOMEM, "surrogate lists");
    if (!c->fb_list && !(c->fb_list = dalloc<int>(c, c->plane))) return fail(c, CP_ENOMEM, "surrogate lists");
    if (!c->src_list && !(c->src_list = dalloc<int>(c, c->plane))) return fail(c, CP_ENOMEM, "surrogate lists");
    if (!mlp_fusable(mlp)) return fail(c, CP_EUNSUPPORTED, "in-step inference needs 256 hidden units");
    if (!c->sur_Y && !(c->sur_Y = dalloc<float>(c, (size_t)c->plane * 15))) return fail(c, CP_ENOMEM, "output rows");
    if (!c->sur_w && !(c->sur_w = dalloc<uint16_t>(c, kFusedW1 + kFusedW2 + kFusedW3)))
        return fail(c, CP_ENOMEM, "packed weights");
    if (!c->sur_b && !(c->sur_b = dalloc<float>(c, 528))) return fail(c, CP_ENOMEM, "packed biases");
    // the context keeps its own copy: later training of the network does not change it
    int r = mlp_snapshot(mlp, c->sur_w, c->sur_b, c->stream);
    if (r) return fail(c, r, "weight snapshot");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->sur_ready = true;
    return CP_OK;
}

int cp_set_qmode(cp_ctx *c, int qmode)
{
    if (!c) return CP_EINVAL;
    if (qmode != CP_Q_EXACT && qmode != CP_Q_OFF && qmode != CP_Q_SURROGATE && qmode != CP_Q_EQUILIBRIUM)
        return fail(c, CP_EINVAL, "bad qmode");
    if (c->nv == NVAR_BI && (qmode == CP_Q_SURROGATE || qmode == CP_Q_EQUILIBRIUM))
        return fail(c, CP_EUNSUPPORTED, "the surrogate and the equilibrium model have one liquid population");
    if (qmode == CP_Q_SURROGATE && !c->sur_ready) return fail(c, CP_ESTATE, "no surrogate attached (cp_sur_set)");
    c->qmode = qmode;
    c->sp.equilibrium = qmode == CP_Q_EQUILIBRIUM ? 1 : 0;
    drop_graphs(c);
    return CP_OK;
}

int cp_diag(cp_ctx *c, const void *U, double out[8])
{
    if (!c || !U || !out) return fail(c, CP_EINVAL, "null argument");
    HIPCHK(c, hipMemsetAsync(c->diag_d, 0, 8 * sizeof(double), c->stream));
    hipError_t e = c->precision == CP_FP64
                       ? launch_diag<double>((const double *)U, c->plane, c->nx, c->nr, c->vol, c->diag_d, c->nv,
                                             c->stream)
                       : launch_diag<float>((const float *)U, c->plane, c->nx, c->nr, c->vol, c->diag_d, c->nv,
                                            c->stream);
    if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
    double h[8];
    unsigned long long ns = 0;
    HIPCHK(c, hipMemcpyAsync(h, c->diag_d, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&ns, c->nsub_d, sizeof(ns), hipMemcpyDeviceToHost, c->stream));
    int r = check_flag(c);
    if (r) return r;
    unsigned long long key;
    memcpy(&key, &h[1], 8);
    unsigned long long bits = (key & 0x8000000000000000ull) ? (key & 0x7FFFFFFFFFFFFFFFull) : ~key;
    memcpy(&h[1], &bits, 8);
    for (int k = 0; k < 5; ++k) out[k] = h[k];
    out[5] = (double)ns;
    int sc[3] = {0, 0, 0};
    unsigned long long st[2] = {0, 0};
    if (c->sur_cnt) {
        HIPCHK(c, hipMemcpyAsync(sc, c->sur_cnt, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipMemcpyAsync(st, c->sur_tot, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    out[6] = (double)(st[0] + (unsigned long long)(sc[0] - sc[2]));
    out[7] = (double)(st[1] + (unsigned long long)(sc[1] + sc[2]));
    return CP_OK;
}

int cp_particle_times(cp_ctx *c, const void *U, double *tau_p, double *St)
{
    if (!c || !U || !tau_p || !St) return fail(c, CP_EINVAL, "null argument");
    if (c->nv != NVAR) return fail(c, CP_EUNSUPPORTED, "particle times: one liquid population only");
    hipError_t e = c->precision == CP_FP64
                       ? launch_particle_times<double>((const double *)U, c->plane, c->nx, c->inv_dx_d, tau_p, St,
                                                       c->stream)
                       : launch_particle_times<float>((const float *)U, c->plane, c->nx, c->inv_dx_d, tau_p, St,
                                                      c->stream);
    if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
    return CP_OK;
}

int cp_sur_features(cp_ctx *c, const void *U, double dt, const float *s_in, float *F)
{
    if (!c || !U || !s_in || !F) return fail(c, CP_EINVAL, "null argument");
    if (!(dt > 0.0)) return fail(c, CP_EDT, "dt must be positive");
    if (c->nv != NVAR) return fail(c, CP_EUNSUPPORTED, "the surrogate's features have one liquid population");
    for (int v = 0; v < NVAR; ++v)
        if (!(s_in[v] > 0.f)) return fail(c, CP_EINVAL, "feature scales must be positive");
    SurNorm nm{};
    memcpy(nm.s_in, s_in, sizeof(nm.s_in));
    hipError_t e = c->precision == CP_FP64
                       ? launch_sur_features<double>((const double *)U, c->plane, dt, nm, F, c->stream)
                       : launch_sur_features<float>((const float *)U, c->plane, dt, nm, F, c->stream);
    if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
    return CP_OK;
}

int cp_set_tile(cp_ctx *c, int tx, int ty)
{
    if (!c) return CP_EINVAL;
    if (tx == 0 && ty == 0) {
        c->tx = c->ty = 0;
    } else if (!tile_supported(tx, ty) || (c->nv == NVAR_BI && (tx != 32 || ty != 8))) {
        return fail(c, CP_EUNSUPPORTED, "tile shape not built");
    } else {
        c->tx = tx;
        c->ty = ty;
    }
    drop_graphs(c);
    return CP_OK;
}

int cp_set_tile_masks(cp_ctx *c, int on)
{
    if (!c) return CP_EINVAL;
    c->masks_off = on == 0;
    drop_graphs(c);
    return CP_OK;
}

int cp_set_drift(cp_ctx *c, int on)
{
    if (!c) return CP_EINVAL;
    if (on && c->mesh.geom == CP_GEOM_QUASI1D) return fail(c, CP_EUNSUPPORTED, "no drift in the quasi-1D duct");
    if (on && c->nv == NVAR_BI) return fail(c, CP_EUNSUPPORTED, "drift is defined for one liquid population");
    c->drift = on != 0;
    drop_graphs(c);
    return CP_OK;
}

int cp_set_bimodal(cp_ctx *c, int on)
{
    if (!c) return CP_EINVAL;
    if (on) {
        if (c->mesh.geom == CP_GEOM_QUASI1D) return fail(c, CP_EUNSUPPORTED, "no particles in the quasi-1D duct");
        if (c->drift) return fail(c, CP_EUNSUPPORTED, "drift is defined for one liquid population");
        if (c->qmode == CP_Q_SURROGATE || c->qmode == CP_Q_EQUILIBRIUM)
            return fail(c, CP_EUNSUPPORTED, "the surrogate and the equilibrium model have one liquid population");
    }
    const int nv = on ? NVAR_BI : NVAR;
    if (nv != c->nv) {
        c->nv = nv;
        c->tx = c->ty = 0;   // the tile is chosen again for the new variable count
        drop_graphs(c);
    }
    return CP_OK;
}

int cp_nvar(const cp_ctx *c) { return c ? c->nv : CP_EINVAL; }

int cp_set_property_table(cp_ctx *c, double h)
{
    if (!c) return CP_EINVAL;
    if (!(h >= 0.0) || (h > 0.0 && (kTabT1 - kTabT0) / h > 1.0e6)) return fail(c, CP_EINVAL, "table spacing");
    // captured steps carry the old table pointer: drop them, and let queued work finish
    drop_graphs(c);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (c->ptab) hipFree(c->ptab);
    c->ptab = nullptr;
    c->sp.ptab = nullptr;
    c->sp.ptab_n = 0;
    if (h == 0.0) return CP_OK;
    const int n = (int)floor((kTabT1 - kTabT0) / h) + 1;
    const std::vector<double> t = property_table(h, n);
    void *p = nullptr;
    if (hipMalloc(&p, t.size() * sizeof(double)) != hipSuccess) return fail(c, CP_ENOMEM, "property table");
    c->ptab = (double *)p;
    HIPCHK(c, hipMemcpy(c->ptab, t.data(), t.size() * sizeof(double), hipMemcpyHostToDevice));
    c->sp.ptab = c->ptab;
    c->sp.ptab_T0 = kTabT0;
    c->sp.ptab_h = h;
    c->sp.ptab_n = n;
    return CP_OK;
}

int cp_get_tile(const cp_ctx *c, int *tx, int *ty)
{
    if (!c || !tx || !ty) return CP_EINVAL;
    *tx = c->tx;
    *ty = c->ty;
    return CP_OK;
}

int cp_time_stage(cp_ctx *c, void *U, int reps, double *ms)
{
    if (!c || !U || !ms || reps < 1) return fail(c, CP_EINVAL, "bad argument");
    int r = autotune(c, U);
    if (r) return r;
    // the three stages of a step, U -> Ua -> Ub -> Ua (U is only read), source off
    const double dt = 1e-12;
    const void *in[3] = {U, c->Ua, c->Ub};
    void *out[3] = {c->Ua, c->Ub, c->Ua};
    if ((r = mask_seed(c, U, c->stream))) return r;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k)
        for (int st = 0; st < 3; ++st) {
            hipError_t e;
            if (c->precision == CP_FP64) {
                StageArgs<double> a = stage_args<double>(c, in[st], U, out[st], st, dt, nullptr);
                a.sp.enabled = 0;   // keep the active list untouched
                e = launch_stage<double>(a, c->tx, c->ty, c->nv, c->stream);
            } else {
                StageArgs<float> a = stage_args<float>(c, in[st], U, out[st], st, dt, nullptr);
                a.sp.enabled = 0;
                e = launch_stage<float>(a, c->tx, c->ty, c->nv, c->stream);
            }
            if (e != hipSuccess) return fail(c, CP_EHIP, hipGetErrorString(e));
        }
    HIPCHK(c, hipEventRecord(e1, c->stream));
    HIPCHK(c, hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, e0, e1));
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms = (double)t / (3.0 * reps);
    return check_flag(c);
}

int cp_mesh_faces(const cp_ctx *c, double *xf, double *rf)
{
    if (!c || !xf || !rf) return CP_EINVAL;
    memcpy(xf, c->xf.data(), sizeof(double) * (c->nx + 1));
    memcpy(rf, c->rf.data(), sizeof(double) * (c->nr + 1));
    return CP_OK;
}

const char *cp_error_string(const cp_ctx *c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"

// ====================================================================== batch
// Many operating points, each a full context (mesh, metrics, BC states, stage
// buffers, active list), advanced together: one stage launch per RK stage covers a
// work list of (plume, tile) pairs, the CFL reduction keeps one time step per
// plume on the device, and the step is captured once in a HIP graph.
struct cp_batch {
    int n = 0, precision = CP_FP64;
    hipStream_t stream = nullptr, cap_stream = nullptr;
    std::vector<cp_ctx *> plumes;
    int tx = 32, ty = 8;
    bool tuned = false;        // tile shape picked by the autotuner
    long max_cells = 0;
    int max_cfl_tiles = 0;     // CFL tiles of the largest plume
    int nwork = 0, cap_work = 0;
    int *work_plume = nullptr, *work_tile = nullptr;
    void *stage_args[3] = {}, *fix_args[3] = {}, *cfl_args = nullptr;
    unsigned long long *acc = nullptr;
    double *cfl = nullptr, *dt = nullptr, *t = nullptr;
    std::vector<void *> allocs;
    hipGraphExec_t graph = nullptr, graph_k = nullptr;   // one step, kStepsMid steps
    std::vector<void *> graph_U;
    std::string err;
};

namespace {

int bfail(cp_batch *b, int code, const std::string &msg)
{
    if (b) b->err = msg;
    return code;
}

template <class T> T *balloc(cp_batch *b, size_t n)
{
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
    b->allocs.push_back(p);
    return (T *)p;
}

template <class R> int batch_upload_args(cp_batch *b, void *const *U)
{
    const int n = b->n;
    std::vector<StageArgs<R>> sa[3];
    std::vector<SourceFixArgs<R>> fa[3];
    std::vector<CflArgs<R>> ca(n);
    for (int p = 0; p < n; ++p) {
        cp_ctx *c = b->plumes[p];
        const void *in[3] = {U[p], c->Ua, c->Ub};
        void *out[3] = {c->Ua, c->Ub, U[p]};
        for (int s = 0; s < 3; ++s) {
            // each plume keeps its own tile masks of U, Ua, Ub (seeded by cp_batch_step_n)
            sa[s].push_back(stage_args<R>(c, in[s], U[p], out[s], s, 0.0, b->dt + p));
            fa[s].push_back(fix_args<R>(c, in[s], out[s], s, 0.0, b->dt + p));
        }
        CflArgs<R> &a = ca[p];
        a = cfl_args<R>(c, U[p]);
        a.acc = b->acc + p;
        a.block_min = nullptr;   // the batch merges into per-plume running minima
    }
    for (int s = 0; s < 3; ++s) {
        if (!b->stage_args[s]) b->stage_args[s] = balloc<StageArgs<R>>(b, n);
        if (!b->fix_args[s]) b->fix_args[s] = balloc<SourceFixArgs<R>>(b, n);
        if (!b->stage_args[s] || !b->fix_args[s]) return bfail(b, CP_ENOMEM, "batch argument tables");
        if (hipMemcpy(b->stage_args[s], sa[s].data(), n * sizeof(StageArgs<R>), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(b->fix_args[s], fa[s].data(), n * sizeof(SourceFixArgs<R>), hipMemcpyHostToDevice) != hipSuccess)
            return bfail(b, CP_EHIP, "batch argument upload");
    }
    if (!b->cfl_args) b->cfl_args = balloc<CflArgs<R>>(b, n);
    if (!b->cfl_args) return bfail(b, CP_ENOMEM, "batch argument tables");
    if (hipMemcpy(b->cfl_args, ca.data(), n * sizeof(CflArgs<R>), hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, CP_EHIP, "batch argument upload");
    return CP_OK;
}

// (plume, tile) work list of one tile shape, uploaded to the batch's work arrays.
int batch_worklist(cp_batch *b, int tx, int ty)
{
    std::vector<int> wp, wt;
    for (int p = 0; p < b->n; ++p) {
        const int gx = (b->plumes[p]->nx + tx - 1) / tx, gy = (b->plumes[p]->nr + ty - 1) / ty;
        for (int k = 0; k < gx * gy; ++k) {
            wp.push_back(p);
            wt.push_back(k);
        }
    }
    if ((int)wp.size() > b->cap_work) return bfail(b, CP_EINVAL, "work list larger than its arrays");
    if (hipMemcpy(b->work_plume, wp.data(), wp.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->work_tile, wt.data(), wt.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, CP_EHIP, "work list upload");
    b->nwork = (int)wp.size();
    b->tx = tx;
    b->ty = ty;
    for (cp_ctx *c : b->plumes) {
        c->tx = tx;
        c->ty = ty;
    }
    return CP_OK;
}

// Pick the batch's tile shape: time the first stage of every plume (U -> its first
// stage buffer, phase-change source off so that no active list is touched, dt = 0,
// with the plumes' tile masks of that shape) for each built shape; an earlier shape
// is kept unless a later one is more than 5 % faster.  All shapes give identical
// results.
template <class R> int batch_autotune(cp_batch *b, void *const *U)
{
    StageArgs<R> *d = balloc<StageArgs<R>>(b, b->n);
    if (!d) return bfail(b, CP_ENOMEM, "autotune arguments");
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return bfail(b, CP_EHIP, "events");
    float best = 1e30f;
    int btx = 32, bty = 8, r = CP_OK;
    for (auto &sh : tile_list()) {
        if ((r = batch_worklist(b, sh.first, sh.second))) break;
        std::vector<StageArgs<R>> sa;
        for (int p = 0; p < b->n && !r; ++p) {
            cp_ctx *c = b->plumes[p];
            if ((r = mask_seed(c, U[p], b->stream))) r = bfail(b, r, c->err);
            sa.push_back(stage_args<R>(c, U[p], U[p], c->Ua, 0, 0.0, nullptr));
            sa.back().sp.enabled = 0;
            sa.back().sur_cnt = nullptr;
        }
        if (r) break;
        if (hipMemcpyAsync(d, sa.data(), b->n * sizeof(StageArgs<R>), hipMemcpyHostToDevice, b->stream) != hipSuccess ||
            hipStreamSynchronize(b->stream) != hipSuccess) {
            r = bfail(b, CP_EHIP, "autotune upload");
            break;
        }
        hipError_t e = launch_stage_batch<R>(d, b->work_plume, b->work_tile, b->nwork, b->tx, b->ty, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
        for (int k = 0; k < 4 && e == hipSuccess; ++k)
            e = launch_stage_batch<R>(d, b->work_plume, b->work_tile, b->nwork, b->tx, b->ty, b->stream);
        if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            r = bfail(b, CP_EHIP, std::string("batch autotune: ") + hipGetErrorString(e));
            break;
        }
        if (ms < 0.95f * best) {
            best = ms;
            btx = sh.first;
            bty = sh.second;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (r) return r;
    if ((r = batch_worklist(b, btx, bty))) return r;
    b->tuned = true;
    return CP_OK;
}

template <class R> int batch_enqueue_step(cp_batch *b, hipStream_t s)
{
    hipError_t e = launch_cfl_batch<R>((const CflArgs<R> *)b->cfl_args, b->n, b->max_cfl_tiles, s);
    if (e == hipSuccess) e = launch_cfl_finalize_batch(b->acc, b->cfl, b->dt, b->t, b->n, s);
    for (int st = 0; st < 3 && e == hipSuccess; ++st) {
        e = launch_stage_batch<R>((const StageArgs<R> *)b->stage_args[st], b->work_plume, b->work_tile, b->nwork,
                                  b->tx, b->ty, s);
        if (e == hipSuccess)
            e = launch_source_fix_batch<R>((const SourceFixArgs<R> *)b->fix_args[st], b->n, b->max_cells, s);
    }
    return e == hipSuccess ? CP_OK : bfail(b, CP_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
}

}  // namespace

extern "C" {

int cp_batch_create(int n, const cp_mesh *meshes, const cp_case *cases, int precision, void *hip_stream,
                    cp_batch **out)
{
    if (!out || n < 1 || !meshes || !cases) return CP_EINVAL;
    *out = nullptr;
    for (int p = 0; p < n; ++p)
        if (meshes[p].geom == CP_GEOM_QUASI1D) return CP_EUNSUPPORTED;   // the batch kernel is axisymmetric/planar
    cp_batch *b = new cp_batch();
    b->n = n;
    b->precision = precision;
    b->stream = (hipStream_t)hip_stream;
    for (int p = 0; p < n; ++p) {
        cp_ctx *c = nullptr;
        int r = cp_create(meshes + p, cases + p, precision, hip_stream, &c);
        if (r) {
            cp_batch_destroy(b);
            return r;
        }
        c->tx = b->tx;
        c->ty = b->ty;
        b->plumes.push_back(c);
        b->max_cells = std::max(b->max_cells, c->plane);
        b->max_cfl_tiles = std::max(b->max_cfl_tiles, cfl_batch_tiles(c->nx, c->nr));
    }
    // work arrays large enough for the smallest built tile (16 x 4 cells)
    for (int p = 0; p < n; ++p) b->cap_work += ((b->plumes[p]->nx + 15) / 16) * ((b->plumes[p]->nr + 3) / 4);
    b->work_plume = balloc<int>(b, b->cap_work);
    b->work_tile = balloc<int>(b, b->cap_work);
    b->acc = balloc<unsigned long long>(b, n);
    b->cfl = balloc<double>(b, n);
    b->dt = balloc<double>(b, n);
    b->t = balloc<double>(b, n);
    if (!b->work_plume || !b->work_tile || !b->acc || !b->cfl || !b->dt || !b->t ||
        hipStreamCreate(&b->cap_stream) != hipSuccess) {
        cp_batch_destroy(b);
        return CP_ENOMEM;
    }
    std::vector<unsigned long long> inf(n, 0x7FF0000000000000ull);
    std::vector<double> cfl(n), zero(n, 0.0);
    for (int p = 0; p < n; ++p) cfl[p] = cases[p].cfl;
    if (batch_worklist(b, b->tx, b->ty) != CP_OK ||
        hipMemcpy(b->acc, inf.data(), n * sizeof(unsigned long long), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->cfl, cfl.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->dt, zero.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->t, zero.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        cp_batch_destroy(b);
        return CP_EHIP;
    }
    *out = b;
    return CP_OK;
}

void cp_batch_destroy(cp_batch *b)
{
    if (!b) return;
    if (b->stream) hipStreamSynchronize(b->stream);
    else hipDeviceSynchronize();
    if (b->graph) hipGraphExecDestroy(b->graph);
    if (b->graph_k) hipGraphExecDestroy(b->graph_k);
    for (cp_ctx *c : b->plumes) cp_destroy(c);
    for (void *p : b->allocs)
        if (p) hipFree(p);
    if (b->cap_stream) hipStreamDestroy(b->cap_stream);
    delete b;
}

int cp_batch_init(cp_batch *b, void *const *U)
{
    if (!b || !U) return CP_EINVAL;
    for (int p = 0; p < b->n; ++p) {
        int r = cp_init(b->plumes[p], U[p]);
        if (r) return bfail(b, r, b->plumes[p]->err);
    }
    return CP_OK;
}

int cp_batch_step_n(cp_batch *b, void *const *U, int nsteps, double *t_host)
{
    if (!b || !U || nsteps < 0) return CP_EINVAL;
    for (int p = 0; p < b->n; ++p)
        if (!U[p]) return bfail(b, CP_EINVAL, "null plume array");
    const bool same = b->graph && b->graph_k && b->graph_U.size() == (size_t)b->n &&
                      std::equal(b->graph_U.begin(), b->graph_U.end(), U);
    if (!same) {
        if (b->graph) hipGraphExecDestroy(b->graph);
        if (b->graph_k) hipGraphExecDestroy(b->graph_k);
        b->graph = b->graph_k = nullptr;
        b->graph_U.clear();
        int r = CP_OK;
        if (!b->tuned)
            r = b->precision == CP_FP64 ? batch_autotune<double>(b, U) : batch_autotune<float>(b, U);
        if (r) return r;
        r = b->precision == CP_FP64 ? batch_upload_args<double>(b, U) : batch_upload_args<float>(b, U);
        if (r) return r;
        // one step and kStepsMid steps per graph
        for (int g = 0; g < 2 && !r; ++g) {
            hipGraph_t gr;
            if (hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return bfail(b, CP_EHIP, "begin capture");
            for (int k = 0; k < (g ? kStepsMid : 1) && !r; ++k)
                r = b->precision == CP_FP64 ? batch_enqueue_step<double>(b, b->cap_stream)
                                            : batch_enqueue_step<float>(b, b->cap_stream);
            hipError_t ec = hipStreamEndCapture(b->cap_stream, &gr);
            if (r) return r;
            if (ec != hipSuccess) return bfail(b, CP_EHIP, std::string("capture: ") + hipGetErrorString(ec));
            hipGraphExec_t *dst = g ? &b->graph_k : &b->graph;
            if (hipGraphInstantiate(dst, gr, nullptr, nullptr, 0) != hipSuccess) {
                hipGraphDestroy(gr);
                return bfail(b, CP_EHIP, "graph instantiate");
            }
            hipGraphDestroy(gr);
        }
        b->graph_U.assign(U, U + b->n);
    }
    if (hipMemsetAsync(b->t, 0, b->n * sizeof(double), b->stream) != hipSuccess) return bfail(b, CP_EHIP, "memset");
    // the plumes' states may have changed since the last call: their tile masks first
    // (the replays keep them current)
    for (int p = 0; p < b->n && nsteps > 0; ++p) {
        int r = mask_seed(b->plumes[p], U[p], b->stream);
        if (r) return bfail(b, r, "plume " + std::to_string(p) + ": " + b->plumes[p]->err);
    }
    for (int k = 0; k < nsteps / kStepsMid; ++k)
        if (hipGraphLaunch(b->graph_k, b->stream) != hipSuccess) return bfail(b, CP_EHIP, "graph launch");
    for (int k = 0; k < nsteps % kStepsMid; ++k)
        if (hipGraphLaunch(b->graph, b->stream) != hipSuccess) return bfail(b, CP_EHIP, "graph launch");
    std::vector<double> t(b->n);
    if (hipMemcpyAsync(t.data(), b->t, b->n * sizeof(double), hipMemcpyDeviceToHost, b->stream) != hipSuccess)
        return bfail(b, CP_EHIP, "time copy");
    for (int p = 0; p < b->n; ++p) {
        int r = check_flag(b->plumes[p]);
        if (r) return bfail(b, r, "plume " + std::to_string(p) + ": " + b->plumes[p]->err);
    }
    if (t_host)
        for (int p = 0; p < b->n; ++p) t_host[p] = t[p];
    return CP_OK;
}

const char *cp_batch_error_string(const cp_batch *b) { return b ? b->err.c_str() : "null batch"; }

}  // extern "C"
