// cp_internal.hpp -- library-internal types shared by the kernels and the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#include <vector>

#include "cp_physics.hpp"

namespace cp {

// Mesh metrics as 1-D device arrays (tensor-product mesh).  Ghost-bearing arrays
// are offset so that index i (or j) = -2 .. n+1 maps to element i+2.
template <class R> struct Metrics {
    const R *xc, *rc;          // n+4 centres (mirrored ghosts)
    const R *inv_dxf;          // nx+1: 1/(xc[i] - xc[i-1]) for the face i-1/2, i = 0..nx
    const R *inv_drf;          // nr+1
    const R *inv_d2x;          // nx+2: 1/(xc[i+1] - xc[i-1]) for i = -1..nx   (index i+1)
    const R *inv_d2r;          // nr+2
    const R *lm2;              // nx+2: mixing length squared at xc[i], i = -1..nx
    const R *inv_dx;           // nx
    const R *rfa;              // nr+1: r-face area per unit axial length (r_f, or 1 planar)
    const R *invV_r;           // nr: 1 / (r_c dr)  (1/dr planar)
    const R *inv_rc;           // nr+2: 1 / r_c for j = -1..nr (0 planar)  (index j+1)
    const R *inv_rf;           // nr+1: 1 / r_f (0 at the axis and for planar)
    const R *axf;              // nx+1: duct area at the x faces (quasi-1D only)
    const R *invVx;            // nx: 1 / (0.5 (A_w + A_e) dx) (quasi-1D only)
};

constexpr int kGeomAxi = 0, kGeomQuasi1D = 2;   // BcInfo::geom (cp_geom)
constexpr long kMaxCells = 1L << 28;             // cells per context: one FP64 plane below 2 GiB

struct BcInfo {
    int nx, nr, geom, bc_xlo, bc_xhi, bc_rlo, bc_rhi;
    const double *inflow;      // nr x 15
    const double *ambient;     // 15
};

// Which passive scalars can be non-zero, per stage tile of the current tile shape:
// bit v of word (tj * gx + ti) is set when variable v (v >= 5) may be non-zero
// somewhere in tile (ti, tj).  A stage reads the mask of its input and writes the
// mask of its output; the kernels that change a stage output afterwards (the
// phase-change source, the learned source) add the bits of the cells they change.
// A bit may be set for a variable that is zero (the masks only ever widen), never
// the other way round.  Null `in`: every scalar may be non-zero.
struct TileMask {
    const unsigned *in;
    const unsigned *un;        // mask of U^n (stages 2, 3), or null
    unsigned *out;
    int tx, ty, gx, gy;        // tile shape, tiles per row and per column
    int nx;                    // cells per row
    unsigned ghost;            // scalars the boundary states (inflow, far field) can hold
};

template <class R> struct StageArgs {
    const R *Uin;              // stencil input U^(s-1)
    const R *Un;               // U^n for the RK combination (stages 2, 3)
    R *Uout;
    const double *dt_dev;      // device time step (graph path) or null
    double dt;
    long plane;
    int stage;                 // 0, 1, 2: SSP-RK3 stage; -1: write R/V only
    int qmode;
    BcInfo bc;
    Metrics<R> m;
    SourceParams sp;
    int *flag;                 // bit 0: non-finite output
    double pref;               // reference pressure removed from the momentum fluxes
    int *active_count;         // cells appended to active_list by this stage
    int *active_list;          // cells whose phase-change source may be non-zero
    int *sur_cnt;              // surrogate counters folded into sur_tot at launch (or null)
    unsigned long long *sur_tot;
    TileMask mask;             // non-zero passive scalars of the input / output tiles
};

// Drift of droplets and crystals (drift-flux reading of the drag law, Eq. 24): a
// separate pass after a stage adds b dt R_drift(U^(s-1)) to the stage output (or
// R_drift to a residual), computed in FP64.
template <class R> struct DriftArgs {
    const R *Uin;              // state the drift is evaluated on
    R *Uout;                   // stage output or residual, updated in place
    const double *dt_dev;
    double dt;
    long plane;
    int stage;                 // 0, 1, 2: weight 1, 1/4, 2/3 of dt; -1: residual (weight 1, no dt)
    BcInfo bc;
    const double *xc, *rc;     // centres, ghost-offset by 2
    const double *inv_dx;      // nx
    const double *rfa;         // nr+1: r-face area per unit axial length
    const double *invV_r;      // nr
    int *flag;
};

template <class R> struct SourceFixArgs {
    const R *Uin;              // stage input U^(s-1): the source is evaluated here
    R *Uout;                   // stage output, updated in place
    const double *dt_dev;
    double dt;
    long plane;
    int stage;
    const int *count, *list;   // active cells of this stage
    int *next_count;           // counter of the next stage, cleared here (or null)
    SourceParams sp;
    int *flag;
    unsigned long long *nsub;  // running total of sub-steps (or null)
    TileMask mask;             // mask.out: tile mask of Uout, widened by the cells changed here
};

template <class R> struct CflArgs {
    const R *U;
    long plane;
    BcInfo bc;
    const double *xc, *rc;     // double centres (offset 2)
    const double *inv_dx, *inv_dr;
    // FP32 contexts: the mesh factors of the limit in the storage precision, indexed as
    // in Metrics (1/(x_{i+1} - x_{i-1}) and l_m^2 at i + 1, 1/(r_{j+1} - r_{j-1}) at
    // j + 1, 1/dx at i); null for FP64 contexts, whose limit uses the centres above
    const float *f_d2x, *f_d2r, *f_lm2, *f_idx;
    double kappa_m, delta0, s_delta;
    unsigned long long *acc;   // running min of the per-cell limit (bits of a positive double)
    double *block_min;         // tiled kernels: one minimum per workgroup (or null: use acc)
};
constexpr int kCflBX = 64, kCflBY = 4, kCflRows = 2;   // CFL kernels: 64 x 4 threads, 2 rows each

struct Ctx;   // host context (cp_api.hip)
}  // namespace cp

struct cp_mlp;
namespace cp {
// Network weights for the fused inference kernel: bf16 weights in MFMA B-fragment
// order for 32-deep k blocks (w1: 1 x 16 fragments, w2: 8 x 16, w3: 8 x 1; 512 bf16
// each) and FP32 biases (b1, b2: 256, b3: 16, zero-padded).
struct FusedNet {
    const uint16_t *w1, *w2, *w3;
    const float *b1, *b2, *b3;
};
constexpr long kFusedW1 = 1L * 16 * 512, kFusedW2 = 8L * 16 * 512, kFusedW3 = 8L * 1 * 512;

// network hooks used by the solver (cp_mlp.hip).  The solver keeps its own packed
// snapshot of the weights (taken by mlp_snapshot) and its own input/output rows.
bool mlp_fusable(const cp_mlp *n);
int mlp_snapshot(cp_mlp *n, uint16_t *w /* kFusedW1 + kFusedW2 + kFusedW3 */, float *b /* 528 */, hipStream_t s);
hipError_t mlp_fused_forward(const FusedNet &w, const uint16_t *X, int n_in, int n_out, const int *rows_dev,
                             int max_rows, float *Y, hipStream_t s);
void mlp_dims(const cp_mlp *n, int *n_in, int *n_out);

// launchers (cp_kernels.hip); nv: variables per cell (NVAR, or NVAR_BI with two
// liquid populations, which has the 32 x 8 stage tile only)
template <class R> hipError_t launch_stage(const StageArgs<R> &a, int tx, int ty, int nv, hipStream_t s);
template <class R> hipError_t launch_cfl(const CflArgs<R> &a, hipStream_t s);
template <class R> hipError_t launch_source_fix(const SourceFixArgs<R> &a, long max_cells, int nv, hipStream_t s);
template <class R> hipError_t launch_drift(const DriftArgs<R> &a, hipStream_t s);
// dt = cfl * min(block_min[0..n)), t += dt (t nullable)
hipError_t launch_cfl_finalize_blocks(const double *block_min, int n, double cfl, double *dt, double *t, hipStream_t s);
template <class R>
hipError_t launch_stage_batch(const StageArgs<R> *args, const int *wp, const int *wt, int nwork, int tx, int ty,
                              hipStream_t s);
template <class R>
hipError_t launch_source_fix_batch(const SourceFixArgs<R> *args, int nplumes, long max_cells, hipStream_t s);
template <class R> hipError_t launch_cfl_batch(const CflArgs<R> *args, int nplumes, int max_tiles, hipStream_t s);
int cfl_batch_tiles(int nx, int nr);   // CFL tiles of one plume's mesh
hipError_t launch_cfl_finalize_batch(unsigned long long *acc, const double *cfl, double *dt, double *t, int n,
                                     hipStream_t s);
hipError_t launch_acc_reset(unsigned long long *acc, hipStream_t s);
template <class R> hipError_t launch_source(const R *U, R *Q, long n, long plane, double dt, const SourceParams &sp,
                                            unsigned long long *nsub, int nv, hipStream_t s);
template <class R> hipError_t launch_init(R *U, const double *inflow, int nx, int nr, int nv, hipStream_t s);
template <class R> hipError_t launch_diag(const R *U, long plane, int nx, int nr, const double *vol,
                                          double *out, int nv, hipStream_t s);
// normalisation of the learned source (feature / target transforms, envelope)
struct SurNorm {
    float s_in[15];            // feature v = asinh(U_v / s_in[v]) for the 15 state variables
    float mu_in[17], sd_in[17];
    float lo[17], hi[17];      // envelope of the standardised training features
    float mu_out[15], sd_out[15];  // output v = standardised increment of feature v over dt
    float lnS_gate;            // exact source where |ln S_l| < lnS_gate (nucleation onset)
    float lnS_lo, lnS_hi;      // ln S_l range of the training set (part of the envelope)
    float df_max;              // trust bound on every predicted feature increment
    float df_max_ice;          // tighter bound on the crystal moments' increments
};

template <class R> struct SurArgs {
    const R *Uin;
    R *Uout;
    const double *dt_dev;
    double dt;
    long plane;
    int stage;
    const int *count, *list;   // active cells of the stage
    int *cnt;                  // [0] cells gated to the network, [1] gate fallback cells,
                               // [2] network cells rejected at decode (exact source)
    int *mlp_cells, *fb_list;
    const float *Y;            // network output [rows][15] (written by the gate's launch)
    SurNorm nm;
    int *flag;
    int q_only;                // write Q itself to Uout (cp_source) instead of adding b dt Q
    TileMask mask;             // mask.out: tile mask of Uout, widened by the cells changed here
};
template <class R>
hipError_t launch_sur_gate_net(const SurArgs<R> &a, const FusedNet &w, float *Y, long max_cells, hipStream_t s);
template <class R>
hipError_t launch_sur_finish(const SurArgs<R> &a, const SourceParams &sp, int *next_count, unsigned long long *nsub,
                             long max_cells, hipStream_t s);
hipError_t launch_sur_reset(int *cnt, unsigned long long *tot, hipStream_t s);
template <class R> hipError_t launch_active_list(const R *U, long plane, int *count, int *list, hipStream_t s);
// Tile masks of a state: bit v of a tile's word set when variable v >= 5 is non-zero
// in one of the tile's cells.
// Drag-law diagnostics: tau_p and Stokes number of droplets and crystals, [2][plane].
template <class R>
hipError_t launch_particle_times(const R *U, long plane, int nx, const double *inv_dx, double *tau, double *St,
                                 hipStream_t s);
template <class R>
hipError_t launch_tile_mask(const R *U, long plane, int nx, int nr, int nv, int tx, int ty, unsigned *mask,
                            unsigned *unknown_a, unsigned *unknown_b, hipStream_t s);
template <class R>
hipError_t launch_sur_features(const R *U, long plane, double dt, const SurNorm &nm, float *F, hipStream_t s);

bool tile_supported(int tx, int ty);
const std::vector<std::pair<int, int>> &tile_list();

}  // namespace cp
