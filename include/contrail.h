/*
 * contrail.h -- C ABI of the MI355X (gfx950) finite-volume step of the
 * non-equilibrium contrail-formation solver of Tegethoff & Wheeler,
 * "Non-Equilibrium Phase Changes in Aircraft Exhaust" (arXiv 2504.20742).
 *
 * The method (Sec. 3.1, Eq. 22-26): dU/dt + div(F^c - F^v) = Q on a 2-D
 * axisymmetric (x, r) structured mesh, U the 15-component conservation vector
 * below, F^c a Roe-type flux with MUSCL / van Leer reconstruction, F^v central
 * viscous + eddy fluxes, Q the per-cell non-equilibrium phase-change source
 * (Sec. 2.2, Eq. 1-21), advanced by explicit Runge-Kutta with a globally
 * controlled CFL number and the source evaluated explicitly in every cell at
 * every stage (Sec. 3.2).
 *
 * Conventions for every call
 *  - Arrays are caller-owned DEVICE pointers (hipMalloc'ed memory or torch CUDA
 *    tensors), contiguous structure-of-arrays U[15][nr][nx] (x index fastest),
 *    or U[19][nr][nx] once cp_set_bimodal has split the liquid (cp_nvar).
 *    Element type: double for CP_FP64 contexts, float for CP_MIXED contexts.
 *    The library never frees caller memory.
 *  - Component order of U (per m^3):
 *      0 rho        gas density (dry air + vapour)          Eq. 23
 *      1 rho u      axial momentum                          Eq. 23
 *      2 rho v      radial momentum                         Eq. 23
 *      3 rho E      gas total energy                        Eq. 23
 *      4 rho Y_v    vapour partial density                  Eq. 25
 *      5..8         rho mu_k of the droplets, k = 0..3      Eq. 19, 26
 *      9..12        rho mu_k of the ice crystals, k = 0..3  Eq. 19, 26
 *      13           soot number density                     Sec. 2.2 (soot at the inflow)
 *      14           activated soot number density           Sec. 2.2 (heterogeneous nucleation)
 *      15..18       rho mu_k of the homogeneously nucleated droplets, k = 0..3, with
 *                   two liquid populations (cp_set_bimodal; 5..8 then hold the
 *                   soot-activated droplets)                 Sec. 2.2
 *  - Every call is ordered on the HIP stream given to cp_create and returns
 *    without synchronising unless stated.  Status codes are returned, never
 *    exceptions; cp_error_string gives the last message of a context.
 *  - Device-side failures (non-finite values written by a stage) are latched in
 *    a device flag and reported as CP_ENONFINITE by the next synchronising call
 *    (cp_cfl_dt, cp_step_n, cp_diag).
 *  - One context per host thread.  Contexts own their workspace (two stage
 *    buffers, mesh metrics, reduction scalars).
 */
#ifndef CONTRAIL_H
#define CONTRAIL_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cp_ctx cp_ctx;

enum cp_status {
    CP_OK = 0,
    CP_EINVAL = -1,        /* bad argument (null pointer, size, dt <= 0, ...)       */
    CP_EHIP = -2,          /* a HIP runtime call failed                             */
    CP_ENONFINITE = -3,    /* a stage produced a NaN / Inf                          */
    CP_EDT = -4,           /* time step not positive / not finite                   */
    CP_ESTATE = -5,        /* call not valid in the context's state                 */
    CP_ENOMEM = -6,        /* device allocation failed                              */
    CP_EUNSUPPORTED = -7   /* option not supported                                  */
};

enum cp_precision {
    CP_FP64 = 0,           /* FP64 storage and arithmetic                           */
    CP_MIXED = 1           /* FP32 storage, fluxes and RK update; source in FP64    */
};

enum cp_qmode {
    CP_Q_EXACT = 0,        /* sub-cycled exact source (Sec. 2.2, Sec. 3.2)          */
    CP_Q_SURROGATE = 1,    /* learned MLP source with exact fallback                */
    CP_Q_OFF = 2,          /* no phase change                                       */
    CP_Q_EQUILIBRIUM = 3   /* the paper's equilibrium comparison model (Sec. 4.2):
                              instantaneous phase equilibrium of each cell's water  */
};

/* AXI: r-weighted axisymmetric cells (Sec. 4.1).  PLANAR: unit-depth cells.
 * QUASI1D: a duct of one cell row (nr = 1) whose x faces have the areas area_x;
 * the cell volume is 0.5 (A_w + A_e) dx, there are no r faces, and the walls push
 * on the gas with p (A_e - A_w) along x (the quasi-1D Euler equations in
 * finite-volume form; a verification geometry for the transport scheme).       */
enum cp_geom { CP_GEOM_AXI = 0, CP_GEOM_PLANAR = 1, CP_GEOM_QUASI1D = 2 };

/* Boundary treatment per side (Sec. 4.1: inflow streams, far field).
 *  INFLOW   (x = 0 only): Dirichlet core / bypass / ambient state by radius
 *  COPY     zero-gradient extrapolation
 *  WALL     mirror (axis at r = 0, or a slip wall): normal velocity odd
 *  FARFIELD (r = L_r only): Dirichlet ambient state                             */
enum cp_bc { CP_BC_INFLOW = 0, CP_BC_COPY = 1, CP_BC_WALL = 2, CP_BC_FARFIELD = 3 };

typedef struct {
    int nx, nr;            /* cells: both >= 2 (nr = 1 for CP_GEOM_QUASI1D), and
                              nx * nr <= 2^28                                       */
    double Lx, Lr;         /* domain [0, Lx] x [0, Lr] in metres                    */
    double sx_ratio;       /* ratio of successive axial widths (1 = uniform)        */
    double r_cluster;      /* radius the radial cells cluster about (<= 0: uniform) */
    double beta_r;         /* sinh clustering strength                              */
    int geom;              /* cp_geom                                               */
    int bc_xlo, bc_xhi, bc_rlo, bc_rhi;   /* cp_bc per side                         */
    const double *area_x;  /* CP_GEOM_QUASI1D: host array of the nx+1 duct areas at
                              the x faces, each finite and > 0; copied by cp_create
                              (the caller keeps ownership).  Ignored otherwise.    */
} cp_mesh;

typedef struct {
    double p_amb, T_amb, RH_ice, mach_amb;  /* ambient: pressure, T, ice RH, flight Ma */
    double R_core, u_core, T_core, Y_core;  /* core jet (pressure-matched)          */
    double R_fan, u_byp, T_byp, Y_byp;      /* bypass jet; Y_byp < 0: ambient Y     */
    double n_soot, r_g_soot, sigma_g_soot;  /* core soot: number, lognormal r_g, s_g */
    double cfl;                             /* CFL number of the global time step   */
    double theta_deg;                       /* soot contact angle (Eq. 9)           */
    double n_s;                             /* active-site density (Eq. 14) [1/m^2] */
    double k_imm;                           /* immersion-freezing rate scale [1/s]  */
    double kappa_m, s_delta, delta0_frac;   /* mixing-length eddy viscosity         */
    int n_sub_max;                          /* cap on source sub-steps (>= 1)       */
    int phase_change;                       /* 0: Q = 0                             */
    int pad0, pad1;
} cp_case;

/* Create a context for one mesh + operating point.  precision: cp_precision.
 * hip_stream: a hipStream_t (NULL = default stream).  On success *out owns the
 * workspace; release with cp_destroy.  Errors: CP_EINVAL (sizes, an unknown
 * geometry or boundary, bc_rlo other than WALL, INFLOW at x = Lx or r = Lr; for
 * CP_GEOM_QUASI1D also nr != 1, bc_rhi other than WALL, a null area_x or an area
 * that is not finite and > 0), CP_ENOMEM, CP_EHIP.                              */
int cp_create(const cp_mesh *mesh, const cp_case *cs, int precision, void *hip_stream, cp_ctx **out);
void cp_destroy(cp_ctx *ctx);

/* Initial state (Sec. 4.1 streams): the inflow profile (core for r < R_core,
 * bypass for r < R_fan, ambient beyond) extended uniformly in x, at rest radially.  */
int cp_init(cp_ctx *ctx, void *U);

/* Transport residual per unit volume (Eq. 22 without Q):
 *   R = -(1/V) sum_faces (F^c - F^v) . A  +  (p - tau_thetatheta) dx dr / V  on rho v
 * (axisymmetric), or + p (A_e - A_w) / V on rho u (quasi-1D duct).              */
int cp_residual(cp_ctx *ctx, const void *U, void *R);

/* Phase-change source integrated over dt (Sec. 2.2 rates, evaluated explicitly per
 * cell, Sec. 3.2): Q(U, dt) = (Phi_dt(U) - U) / dt, computed in FP64 for both
 * precisions.  dt > 0, else CP_EDT.  With CP_Q_SURROGATE selected, the cells the
 * surrogate gate hands to the network get the network's closed source instead
 * (exactly as a step would use it); every other cell keeps the exact source.       */
int cp_source(cp_ctx *ctx, const void *U, double dt, void *Q);

/* One SSP-RK3 step of size dt, in place: L(U) = R(U) + Q(U, dt).                 */
int cp_step(cp_ctx *ctx, void *U, double dt);

/* Global CFL time step (Sec. 3.2 "globally controlled CFL number"):
 *   dt = CFL min_cells 1 / ((|u|+c)/dx + (|v|+c)/dr + 2 nu_eff (1/dx^2 + 1/dr^2)),
 * without the 1/dr terms in the quasi-1D duct.
 * Evaluated in IEEE FP64 for CP_FP64 contexts and in FP32 for CP_MIXED contexts.
 * Synchronises the stream and writes *dt_host.                                   */
int cp_cfl_dt(cp_ctx *ctx, const void *U, double *dt_host);

/* n steps, each with its own CFL time step computed and kept on the device; the
 * step sequence is a captured HIP graph replayed n times.  Synchronises; writes the
 * simulated time to *t_host (may be NULL).                                        */
int cp_step_n(cp_ctx *ctx, void *U, int n, double *t_host);

/* Select how Q is evaluated (cp_qmode).  CP_Q_SURROGATE needs cp_sur_set first.
 * CP_Q_EQUILIBRIUM: Q = (Phi_eq(U) - U)/dt, Phi_eq the cell's water brought to phase
 * equilibrium at fixed dry air, velocity and energy bookkeeping: liquid at or above
 * 273.15 K, ice below, both at 273.15 K where neither branch alone is consistent;
 * vapour at saturation over that phase, or all water evaporated.  A cell without
 * condensate changes only once supersaturated over liquid.  Particle numbers are
 * kept (new condensate sits on the soot, or on 0.1 um particles without soot), each
 * population monodisperse at its mean-mass radius.  Computed in FP64 for both
 * precisions.  Errors: CP_EINVAL for an unknown mode, CP_ESTATE (see above),
 * CP_EUNSUPPORTED for CP_Q_SURROGATE or CP_Q_EQUILIBRIUM with two liquid
 * populations (cp_set_bimodal).                                                  */
int cp_set_qmode(cp_ctx *ctx, int qmode);

/* Diagnostics (synchronises): out[0] total water mass per radian
 * (vapour + 4pi/3 (rho_l M3 + rho_s N3), Eq. 25-26, both liquid populations with
 * cp_set_bimodal), out[1] max ln S_l (Eq. 1),
 * out[2] total ice number, out[3] gas mass, out[4] cells with an active source,
 * out[5] sub-steps of the exact source since the last cp_source call (that call
 * and every later step included), out[6] and out[7] running
 * totals of the active cells the surrogate (CP_Q_SURROGATE) sent to the network and
 * to the exact fallback, summed over every stage since cp_sur_set.              */
int cp_diag(cp_ctx *ctx, const void *U, double out[8]);

/* Drag-law diagnostics (Eq. 24): the response time of the droplets and of the ice
 * crystals at their mean radius r20 = sqrt(mu2/mu0),
 *   tau_p = rho_p (2 r20)^2 Cc / (18 mu),  Cc = 1 + 2 A_C Kn, Kn = lbar / (2 r20)
 * (the particle mass over its Stokes friction; zero slip in the one-velocity model,
 * so the Schiller-Naumann factor is 1), and the Stokes number St = tau_p |u| / dx_i.
 * tau_p and St: caller-owned DEVICE double arrays [2][nr][nx] (plane 0 droplets,
 * plane 1 crystals), zero where a population is empty or has evaporated.
 * Stream-ordered, no synchronisation.  Errors: CP_EINVAL (null argument),
 * CP_EUNSUPPORTED with two liquid populations, CP_EHIP.                          */
int cp_particle_times(cp_ctx *ctx, const void *U, double *tau_p, double *St);

/* Drift of droplets and crystals against the gas (on != 0), the drag law (Eq. 24)
 * read as a drift flux in this one-velocity solver: particles lag the gas's
 * pressure-driven acceleration with their terminal slip, at which the drag of
 * Eq. 24 balances that force: w (1 + 0.15 Re^0.687) = w_St with the
 * Stokes-Cunningham slip
 *   w_St(r) = 2 rho_p r^2 Cc(r) (1 - rho/rho_p) (dp/dn) / (9 mu rho),
 *   Cc = 1 + 2 A_C Kn, Kn = lbar / (2 r), lbar = 1.5 mu sqrt(R T) / p,
 * and Re = rho |w| 2 r / mu (six fixed-point steps from w_St),
 * and each population drifts as a whole with the slip of its mean radius r20:
 * moment k crosses a face with w(r20) M_k, upwind in its sign (the moment set
 * stays realisable).  Soot stays with the gas.  Applied
 * in every stage (and cp_residual) by a pass after the stage kernel, in FP64.
 * Off by default.  Errors: CP_EUNSUPPORTED in the quasi-1D duct and with two
 * liquid populations (cp_set_bimodal).                                           */
int cp_set_drift(cp_ctx *ctx, int on);

/* Water properties of the phase-change source (ln p_sat over liquid and ice, the
 * surface tension) from a table instead of the closed forms, as the paper reads its
 * pre-tabulated properties (Sec. 3.2): nodes every h kelvin on [150, 700] K, each
 * holding value, slope and half curvature; a lookup expands to second order about
 * the nearest node (about the end node outside the range), so the error falls as
 * h^3 (about 2e-8 in ln p_sat at h = 0.25 K).  Saturation temperatures invert the
 * expanded ln p_sat.  Whether a cell's source can be non-zero is still decided on
 * the closed form.  h = 0 returns to the closed forms.  The context keeps its own
 * device copy; the call synchronises the stream.  Errors: CP_EINVAL (h < 0, or
 * more than 1e6 nodes), CP_ENOMEM, CP_EHIP.                                       */
int cp_set_property_table(cp_ctx *ctx, double h);

/* Two liquid populations (on != 0), the bimodal moment approach of Sec. 2.2: the
 * soot-activated droplets keep variables 5..8 and the homogeneously nucleated ones
 * take 15..18, so every state, residual and source array of the context then has
 * 19 planes.  Each population has its own nucleation source (the activation rate,
 * or the homogeneous rate, at the critical radius), r20 growth closure and
 * lognormal freezing closure; immersion freezing acts on the soot-activated
 * droplets only (it needs a soot core), and only their complete evaporation
 * releases the activated soot; frozen droplets of both join the one crystal
 * population.  The inflow and far field carry no homogeneous droplets.  The stage
 * kernel uses the 32 x 8 tile.  Off by default; switching drops the captured
 * steps.  Errors: CP_EUNSUPPORTED in the quasi-1D duct, with drift, with the
 * surrogate or the equilibrium model selected (each has one liquid population;
 * cp_set_qmode and cp_set_drift refuse them in turn).                            */
int cp_set_bimodal(cp_ctx *ctx, int on);

/* Variables per cell of the context's arrays: 15, or 19 with two liquid
 * populations.  CP_EINVAL for a null context.                                     */
int cp_nvar(const cp_ctx *ctx);

/* Tile shape of the stage kernel: (tx, ty) from the built set, or (0, 0) to run the
 * built-in autotuner on the next step.  CP_EUNSUPPORTED for shapes not built (with
 * two liquid populations only 32 x 8 is built).                                  */
int cp_set_tile(cp_ctx *ctx, int tx, int ty);

/* Per-tile masks of the non-zero passive scalars (on by default): the stage kernel
 * loads and transports only the scalars that can be non-zero on a tile's stencil,
 * skips the RK loads of planes that are zero on the whole tile, and does not store
 * a zero scalar where the output buffer already holds zero on the tile.  The
 * results are the same with and without them, bit for bit up to the sign of a zero
 * (a scalar outside a tile's mask is zero on its whole stencil).  on = 0 turns them
 * off, for comparison.  The drift pass (cp_set_drift) runs without them.
 * CP_EINVAL for a null context.                                                    */
int cp_set_tile_masks(cp_ctx *ctx, int on);
int cp_get_tile(const cp_ctx *ctx, int *tx, int *ty);

/* Measurement entry point: launch the three SSP-RK3 stages of the fused stage kernel
 * `reps` times (U -> stage buffer -> stage buffer -> stage buffer; U is only read,
 * the phase-change source is left out) between two HIP events on the context
 * stream; synchronises and writes the mean duration of one stage launch in
 * milliseconds.  Uses the current tile (autotuned first if unset).                 */
int cp_time_stage(cp_ctx *ctx, void *U, int reps, double *ms_per_launch);

/* Mesh faces (host copies): xf[nx+1], rf[nr+1].                                   */
int cp_mesh_faces(const cp_ctx *ctx, double *xf, double *rf);

const char *cp_error_string(const cp_ctx *ctx);

/* ---------------------------------------------------------------------- batch
 * Many operating points (plumes), each with its own mesh and case, advanced
 * together: every RK stage is one launch over a work list of (plume, tile) pairs
 * (the tile shape picked by timing every built shape before the first step), each
 * plume with its own tile masks of non-zero passive scalars (seeded at every
 * cp_batch_step_n call), the CFL limit over (plume, tile) pairs with one time step
 * per plume kept on the device, and the whole step is a captured HIP graph.
 * Per-plume results are identical to running that plume alone.
 * Arrays: U[p] is plume p's U[15][nr_p][nx_p] (caller-owned device memory).         */
typedef struct cp_batch cp_batch;

/* n plumes with meshes[p], cases[p] (host arrays of n structs), all in one precision,
 * launched on hip_stream.  Errors as cp_create; CP_EUNSUPPORTED for a quasi-1D duct
 * (the batch runs axisymmetric and planar plumes).                                */
int cp_batch_create(int n, const cp_mesh *meshes, const cp_case *cases, int precision, void *hip_stream,
                    cp_batch **out);
void cp_batch_destroy(cp_batch *b);
/* Initial state of every plume (as cp_init).  U: host array of n device pointers.    */
int cp_batch_init(cp_batch *b, void *const *U);
/* nsteps steps of every plume; synchronises; t_host (n entries, may be NULL) receives
 * each plume's simulated time.  CP_ENONFINITE names the plume in the message.      */
int cp_batch_step_n(cp_batch *b, void *const *U, int nsteps, double *t_host);
const char *cp_batch_error_string(const cp_batch *b);

/* -------------------------------------------------------------- learned source
 * Multilayer perceptron n_in -> n_hidden -> n_hidden -> n_out with GELU (tanh form)
 * after each hidden layer, used as a surrogate of the stiff phase-change source.
 * bfloat16 weights and activations, FP32 accumulation on the matrix cores, FP32
 * master weights and Adam moments, mean-squared-error loss.  Parameters are flat
 * FP32 in the order W1[n_in][n_hidden], b1, W2[n_hidden][n_hidden], b2,
 * W3[n_hidden][n_out], b3 (row-major).  X, T, Y are caller-owned DEVICE arrays,
 * row-major [rows][features].                                                      */
typedef struct cp_mlp cp_mlp;

int cp_mlp_create(int n_in, int n_hidden, int n_out, void *hip_stream, cp_mlp **out);
void cp_mlp_destroy(cp_mlp *mlp);
long cp_mlp_num_params(const cp_mlp *mlp);
/* Host FP32 parameters in / out (set also resets the Adam moments).             */
int cp_mlp_set_params(cp_mlp *mlp, const float *host_params);
int cp_mlp_get_params(cp_mlp *mlp, float *host_params);
/* Y[rows][n_out] = network(X[rows][n_in]); X is rounded to bfloat16.  Networks with
 * n_in <= 32, n_hidden = 256, n_out <= 16 run all three layers in one fused kernel
 * (activations in LDS); others run layer by layer.                                */
int cp_mlp_forward(cp_mlp *mlp, const float *X, int rows, float *Y);
/* cp_mlp_forward for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same result as
 * cp_mlp_forward, with no allocation by the library at any call.  The bf16 input rows,
 * the packed weights and the biases of a call live in a static device array of
 * 4.3 MB that each GPU holds until the process ends; every call on a GPU shares it
 * (each call packs its network's weights again), so calls that overlap on one GPU
 * race.  Only the fused inference shape (n_in <= 32, 256 hidden units,
 * n_out <= 16) and at most 65536 rows per call.  Stream-ordered on the network's
 * stream, no synchronisation.  Errors: CP_EINVAL (null argument, rows outside
 * [1, 65536]), CP_EUNSUPPORTED (another network shape), CP_EHIP.                  */
int cp_mlp_forward_static(cp_mlp *mlp, const float *X, int rows, float *Y);
/* Forward + backward of the MSE loss mean((Y - T)^2) over rows and outputs; the
 * gradient is kept for cp_mlp_adam; *loss_host (nullable) gets the loss,
 * grad_host (nullable, cp_mlp_num_params floats) a host copy of the gradient.
 * Synchronises the stream.                                                      */
int cp_mlp_loss_grad(cp_mlp *mlp, const float *X, const float *T, int rows, double *loss_host, float *grad_host);
/* One Adam step with the last gradient (bias-corrected moments).               */
int cp_mlp_adam(cp_mlp *mlp, double lr, double beta1, double beta2, double eps);
const char *cp_mlp_error_string(const cp_mlp *mlp);

/* Attach a trained 17 -> 256 -> 256 -> 15 network as the source of a context
 * (CP_Q_SURROGATE).  The context takes a copy of the weights at this call, packed for
 * its fused inference kernel: later training or destruction of the network does not
 * affect it (attach again to update).  norm: n_norm = 118 host floats in the order
 *   s_in[15], mu_in[17], sd_in[17], lo[17], hi[17], mu_out[15], sd_out[15],
 *   lnS_gate, lnS_lo, lnS_hi, df_max, df_max_ice
 * Features of an active cell: f_v = asinh(U_v / s_in[v]) for the 15 state variables,
 * ln dt, log10 max(N_soot, 1), standardised with (mu_in, sd_in).  The network takes
 * the cell when every standardised feature lies in [lo, hi] and ln S_l in
 * [lnS_lo, lnS_hi] (the training envelope), |ln S_l| >= lnS_gate (away from
 * nucleation onset) and its droplets cannot freeze (no droplets, or the gas at or
 * above 273.15 K: freezing, Eq. 12-15, always takes the exact source); otherwise
 * the exact sub-cycled source is used (Sec. 3.2).
 * Output v (v = 5..12 particle moments, 14 activated soot) is the standardised
 * increment of f_v over dt: U'_v = s_in[v] sinh(max(f_v + y_v sd_out[v] + mu_out[v], 0)),
 * Q_v = (U'_v - U_v) / dt.  The remaining sources are closed exactly: vapour sink
 * -(4 pi/3)(rho_l Q_M3 + rho_s Q_N3) (water conserved, Eq. 25-26), gas mass and
 * momentum follow the vapour, the gas energy loses the condensate enthalpy, the soot
 * number is unchanged.  A network cell falls back to the exact source when any
 * predicted increment exceeds df_max in magnitude (df_max_ice for the crystal
 * moments 9..12: freezing is what the network reproduces least well, its rate
 * changing by orders of magnitude per kelvin), when a particle population is not
 * realizable after the update (neither empty nor positive, log-convex moments with a
 * mean radius in [0.1 nm, 1 mm]) or when its vapour would turn negative.
 * The context allocates 17 bf16 feature values and 15 floats of network output per
 * cell plus the packed weights (150 KB); the hidden activations never leave the
 * workgroup.  Attaching drops the captured step and leaves a context that was in
 * CP_Q_SURROGATE in CP_Q_EXACT: select CP_Q_SURROGATE again afterwards.
 * Errors: CP_EINVAL (null, n_norm != 118, network not 17 -> 15), CP_EUNSUPPORTED
 * (hidden width other than 256), CP_ENOMEM, CP_EHIP.                               */
int cp_sur_set(cp_ctx *ctx, cp_mlp *mlp, const float *norm, int n_norm);

/* Training-set features of every cell of U (the gate's own computation): F is a
 * caller-owned DEVICE float array [nr*nx][19], row j*nx+i holding
 *   asinh(U_v / s_in[v]) (v = 0..14), ln dt, log10 max(N_soot, 1), ln S_l, T
 * (unstandardised; T the gas temperature in kelvin, which decides the freezing
 * regime).  s_in: 15 positive host floats.  Stream-ordered, no sync.
 * Errors: CP_EINVAL, CP_EDT (dt <= 0), CP_EHIP.                                    */
int cp_sur_features(cp_ctx *ctx, const void *U, double dt, const float *s_in, float *F);

#ifdef __cplusplus
}
#endif
#endif /* CONTRAIL_H */
