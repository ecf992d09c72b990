// cp_kernels.hip -- HIP kernels of the contrail finite-volume step for gfx950.
//
// k_stage: one fused SSP-RK3 stage per launch.  A block owns a TX x TY tile of
// cells; the tile plus a 2-cell halo is staged in LDS as gas primitives (the
// MUSCL stencil of Sec. 3.2 is 2 cells wide), so every primitive, viscosity and
// eddy viscosity is computed once per tile cell.  The ten per-mass scalars
// (moments and soot numbers; the vapour travels with the gas; fourteen with two
// liquid populations) then go through the freed primitive arrays five at a time,
// upwinded with the Roe mass flux; a scalar that is zero on the whole tile is
// skipped.  The RK combination is fused into the epilogue, so a stage
// reads U^(s-1) (+ U^n) and writes U^(s) once: a coalesced structure-of-arrays
// stream.  Cells where the phase-change source (Sec. 2.2) can act are appended to
// a compacted list; k_source_fix integrates the stiff source for those cells
// only, which keeps the register footprint of the stencil kernel small.
#include "cp_fused_net.hpp"
#include "cp_internal.hpp"

namespace cp {

constexpr int kAmbient = INT32_MIN;

// Source location of cell (i, j), i in [-2, nx+1], j in [-2, nr+1]:
//   code >= 0          interior element j*nx + i
//   code == kAmbient   far-field ambient state
//   code <  0          inflow state of row (-1 - code)
// fu / fv: negate the axial / radial momentum (mirror boundaries).
struct CellSrc {
    int code;
    bool fu, fv;
};

__device__ __forceinline__ CellSrc map_cell(int i, int j, const BcInfo &b)
{
    CellSrc s{0, false, false};
    while (j < 0 || j >= b.nr) {
        if (j < 0) {
            j = -1 - j;
            s.fv = !s.fv;
        } else if (b.bc_rhi == 3) {
            s.code = kAmbient;
            return s;
        } else if (b.bc_rhi == 2) {
            j = 2 * b.nr - 1 - j;
            s.fv = !s.fv;
        } else {
            j = b.nr - 1;
        }
    }
    while (i < 0 || i >= b.nx) {
        if (i < 0) {
            if (b.bc_xlo == 0) {
                s.code = -1 - j;
                return s;
            }
            if (b.bc_xlo == 2) {
                i = -1 - i;
                s.fu = !s.fu;
            } else {
                i = 0;
            }
        } else if (b.bc_xhi == 2) {
            i = 2 * b.nx - 1 - i;
            s.fu = !s.fu;
        } else {
            i = b.nx - 1;
        }
    }
    s.code = j * b.nx + i;
    return s;
}

// Raw buffer access to one plane of a state array: the plane's base and size sit
// in a scalar resource descriptor and the cell offset in one vector register, so a
// load or store needs no 64-bit vector address arithmetic (one shared offset serves
// all planes).  The hardware range check reads 0 past the plane's end and drops
// such stores; every access here is inside the plane.
constexpr int kBufferWord3 = 0x00020000;   // resource word 3 of a raw buffer on gfx9-family GPUs
template <class R> __device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const R *base, long plane)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<R *>(base), 0, (int)(plane * (long)sizeof(R)),
                                             kBufferWord3);
}
__device__ __forceinline__ float buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, float)
{
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}
__device__ __forceinline__ double buf_ld(__amdgpu_buffer_rsrc_t r, unsigned off, double)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, (int)off, 0, 0);
}
__device__ __forceinline__ void buf_st(__amdgpu_buffer_rsrc_t r, unsigned off, double x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(__attribute__((ext_vector_type(2))) unsigned, x), r,
                                          (int)off, 0, 0);
}
// element k of plane v of the state array U
template <class R> __device__ __forceinline__ R ld_plane(const R *U, long plane, int v, unsigned k)
{
    return buf_ld(plane_rsrc(U + v * plane, plane), k * (unsigned)sizeof(R), R(0));
}
template <class R> __device__ __forceinline__ void st_plane(R *U, long plane, int v, unsigned k, R x)
{
    buf_st(plane_rsrc(U + v * plane, plane), k * (unsigned)sizeof(R), x);
}

template <class R>
__device__ __forceinline__ R fetch(const R *U, long plane, const BcInfo &b, int code, int v)
{
    if (code >= 0) return U[v * plane + code];
    if (v >= NVAR) return R(0);   // the inflow and the far field carry no homogeneous droplets
    if (code == kAmbient) return (R)b.ambient[v];
    return (R)b.inflow[(-1 - code) * NVAR + v];
}

// ------------------------------------------------------------------ stage
template <class R> __device__ __forceinline__ R vl_slope(R a, R b)
{
    // van Leer limiter in harmonic form: 2ab/(a+b) where a, b have the same sign
    const R q = tdiv(R(2) * a * b, a + b);   // selected away where a b <= 0
    return (a * b > R(0)) ? q : R(0);
}

// LDS tile: primitives of TX x TY cells plus a 2-cell halo (ext, EX x EY), vapour
// diffusivity, molecular and eddy viscosity and limited slopes of one direction on the
// tile plus a 1-cell ring (RX x RY), and one face buffer reused for the x-faces and the
// r-faces (the mass flux is its first component, which is also the Roe mass flux the
// scalars are upwinded with).  Whatever is cheap to recompute (the faces' eddy
// diffusivity, a halo cell's source address) is not stored: the FP32 tile then fits six
// workgroups per CU.
template <class R, int TX, int TY> struct Tile {
    static constexpr int EX = TX + 4, EY = TY + 4, N = EX * EY;
    static constexpr int RX = TX + 2, RY = TY + 2, NR = RX * RY;
    static constexpr int NFX = (TX + 1) * TY, NFR = TX * (TY + 1);
    static constexpr int NF = NFX > NFR ? NFX : NFR;
    // slopes: x slopes on the ring's rows 1..TY (RX x TY), then r slopes on its columns
    // 1..TX (TX x (TY + 2)), each with its own compact index
    static constexpr int NSX = RX * TY, NSR = TX * (TY + 2), NS = NSX > NSR ? NSX : NSR;
    static constexpr int NFB = 5 * NF;
    R rho[N], u[N], v[N], p[N], T[N], Y[N];   // u..Y are reused for 5 scalars at a time
    R D[NR], mu[NR], mut[NR];
    R sl[5][NS];                 // gas slopes of one direction (x, then r)
    R fbuf[NFB];                 // faces: F (5 components, [5][NF]); F[0] is the Roe mass flux
    int nonzero[3];              // per scalar group: bit k set when scalar k is non-zero somewhere in the tile
    unsigned omask;              // non-zero passive scalars of the tile's output (bit v: variable v)
    __device__ R (*face())[NF] { return reinterpret_cast<R(*)[NF]>(fbuf); }
};

// Eddy diffusivity / dn of the passive scalars at a face, from the cells' eddy
// viscosities (recomputed where the scalar fluxes need it rather than kept in LDS).
template <class R> __device__ __forceinline__ R face_kd(R mut_a, R mut_b, R inv_dn)
{
    const R mut = R(0.5) * (mut_a + mut_b);
    return mut * R(1.0 / kSct) * inv_dn;
}

// ext index of ring cell r, and ring index of ext cell e (inside the ring)
template <int TX, int TY> __device__ __forceinline__ int ext_of_ring(int r)
{
    return (r / (TX + 2) + 1) * (TX + 4) + r % (TX + 2) + 1;
}
template <int TX, int TY> __device__ __forceinline__ int ring_of_ext(int e)
{
    return (e / (TX + 4) - 1) * (TX + 2) + e % (TX + 4) - 1;
}

// Gas flux through the face between ext cells a and b = a + s (normal stride s,
// tangential stride ts; ra, rb their ring indices, sa, sb their slope indices): MUSCL states from the cell
// slopes, Roe convective flux, central viscous + eddy flux.  Writes F^c - F^v on
// (rho, rho u, rho v, rho E, rho Y) in global components; F[0] is the Roe mass flux.
template <class R, class TileT>
__device__ __forceinline__ void gas_face(const TileT &t, int a, int ra, int rb, int sa, int sb, int s, int ts, bool xdir, R inv_dn,
                                         R inv_d2t, R inv_r, R pref, R *F)
{
    const int b = a + s;
    const R(*sl)[TileT::NS] = t.sl;   // slopes of the face-normal direction
    const R *un_ = xdir ? t.u : t.v;
    const R *ut_ = xdir ? t.v : t.u;
    R qL[5], qR[5];
    qL[0] = t.rho[a] + R(0.5) * sl[0][sa];
    qR[0] = t.rho[b] - R(0.5) * sl[0][sb];
    qL[1] = un_[a] + R(0.5) * sl[xdir ? 1 : 2][sa];
    qR[1] = un_[b] - R(0.5) * sl[xdir ? 1 : 2][sb];
    qL[2] = ut_[a] + R(0.5) * sl[xdir ? 2 : 1][sa];
    qR[2] = ut_[b] - R(0.5) * sl[xdir ? 2 : 1][sb];
    qL[3] = t.p[a] + R(0.5) * sl[3][sa];
    qR[3] = t.p[b] - R(0.5) * sl[3][sb];
    qL[4] = t.Y[a] + R(0.5) * sl[4][sa];
    qR[4] = t.Y[b] - R(0.5) * sl[4][sb];
    R Fc[4];
    roe_flux(qL, qR, pref, Fc);
    const R Fm = Fc[0];
    const R FY = Fm * (Fm >= R(0) ? qL[4] : qR[4]);

    const R mu = R(0.5) * (t.mu[ra] + t.mu[rb]);
    const R mut = R(0.5) * (t.mut[ra] + t.mut[rb]);
    const R rho = R(0.5) * (t.rho[a] + t.rho[b]);
    const R cpf = R(0.5) * (gas_cp(t.Y[a]) + gas_cp(t.Y[b]));
    const R Df = R(0.5) * (t.D[ra] + t.D[rb]);
    const R dhf = R(kLv0) + R(kCpv - kCpa) * (R(0.5) * (t.T[a] + t.T[b]) - R(kTref));
    const R uf = R(0.5) * (t.u[a] + t.u[b]), vf = R(0.5) * (t.v[a] + t.v[b]);
    const R un_n = (un_[b] - un_[a]) * inv_dn;
    const R ut_n = (ut_[b] - ut_[a]) * inv_dn;
    const R dT_n = (t.T[b] - t.T[a]) * inv_dn;
    const R dY_n = (t.Y[b] - t.Y[a]) * inv_dn;
    const R dut_t = R(0.5) * ((ut_[a + ts] - ut_[a - ts]) + (ut_[b + ts] - ut_[b - ts])) * inv_d2t;
    const R dun_t = R(0.5) * ((un_[a + ts] - un_[a - ts]) + (un_[b + ts] - un_[b - ts])) * inv_d2t;
    const R div = un_n + dut_t + vf * inv_r;
    const R mue = mu + mut;
    const R tnn = mue * (R(2) * un_n - R(2.0 / 3.0) * div);
    const R tnt = mue * (ut_n + dun_t);
    const R diffY = rho * Df + mut * R(1.0 / kSct);
    const R Jv = -diffY * dY_n;
    const R qn = -(cpf * mu * R(1.0 / kPr) + cpf * mut * R(1.0 / kPrT)) * dT_n + dhf * Jv;
    F[0] = Fm;
    if (xdir) {
        F[1] = Fc[1] - tnn;
        F[2] = Fc[2] - tnt;
        F[3] = Fc[3] - (uf * tnn + vf * tnt - qn);
    } else {
        F[1] = Fc[2] - tnt;
        F[2] = Fc[1] - tnn;
        F[3] = Fc[3] - (uf * tnt + vf * tnn - qn);
    }
    F[4] = FY + Jv;
}

// Flux divergence per unit volume from face fluxes, evaluated without contraction
// so that equal opposite faces cancel exactly (free-stream / closed-box symmetry).
template <class R> __device__ __forceinline__ R assemble_x(R fe, R fw, R idx)
{
#pragma clang fp contract(off)
    return -(fe - fw) * idx;
}

template <class R> __device__ __forceinline__ R assemble_r(R rx, R fn, R an, R fs, R as, R ivr)
{
#pragma clang fp contract(off)
    return rx - (fn * an - fs * as) * ivr;
}

// Quasi-1D duct: x faces of areas aw, ae and cell volume 1/iv.
template <class R> __device__ __forceinline__ R assemble_duct(R fe, R ae, R fw, R aw, R iv)
{
#pragma clang fp contract(off)
    return -(fe * ae - fw * aw) * iv;
}

// Passive scalar flux through a face from the two cells' values and limited slopes:
// upwind MUSCL value times the Roe mass flux, minus eddy diffusion.  Both one-sided
// states are formed and the upwind one selected, so the flux is branch-free.
template <class R> __device__ __forceinline__ R scalar_flux(R pa, R pb, R sa, R sb, R Fm, R kd)
{
    const R upL = pa + R(0.5) * sa;
    const R upR = pb - R(0.5) * sb;
    return Fm * (Fm >= R(0) ? upL : upR) - kd * (pb - pa);
}

// Slot k of a group of five passive scalars: the primitive arrays are free once the
// gas fluxes are assembled.
template <class TileT> __device__ __forceinline__ auto *scalar_slot(TileT &t, int k)
{
    return k == 0 ? t.u : (k == 1 ? t.v : (k == 2 ? t.p : (k == 3 ? t.T : t.Y)));
}

// phi = U / rho with one transport reciprocal per cell and group.
template <class R> __device__ __forceinline__ R inv_rho(R rho) { return trcp(rho); }
// The product is rounded on its own (never fused into a later operation), whether
// it goes through the tile's slots or straight into a flux: both paths then see the
// same per-mass values.
template <class R> __device__ __forceinline__ R per_mass(R U, R, R ir)
{
#pragma clang fp contract(off)
    return U * ir;
}

// Fold the surrogate's per-stage counters into its running totals and clear them.
__device__ __forceinline__ void sur_fold_counts(int *cnt, unsigned long long *tot)
{
    tot[0] += (unsigned long long)(cnt[0] - cnt[2]);   // network cells kept
    tot[1] += (unsigned long long)(cnt[1] + cnt[2]);   // exact: gate fallback + rejected decodes
    cnt[0] = 0;
    cnt[1] = 0;
    cnt[2] = 0;
}

// XCD-aware order: workgroups are dealt round-robin to the 8 XCDs, so workgroup b
// takes item xcd*q + min(xcd, rem) + b/8 -- a contiguous band of tiles per XCD, whose
// neighbouring tiles then share their halos in that XCD's L2.
__device__ __forceinline__ int xcd_band(int b, int nb)
{
    const int xcd = b & 7, q = nb >> 3, rem = nb & 7;
    return xcd * q + min(xcd, rem) + (b >> 3);
}

// Bits of a cell's passive scalars (variables 5..NV-1) that are non-zero.
template <class R, int NV> __device__ __forceinline__ unsigned scalar_bits(const R *x)
{
    unsigned b = 0;
    #pragma unroll
    for (int v = 5; v < NV; ++v) b |= (x[v] != R(0)) ? (1u << v) : 0u;
    return b;
}

// Widen the output tile mask by the non-zero scalars of cell c's new state.
__device__ __forceinline__ void mask_mark(const TileMask &m, long c, unsigned bits)
{
    if (!m.out || !bits) return;
    const int i = (int)(c % m.nx), j = (int)(c / m.nx);
    atomicOr(&m.out[(j / m.ty) * m.gx + i / m.tx], bits);
}

// OR of a value over the wavefront.
__device__ __forceinline__ unsigned wave_or(unsigned x)
{
    #pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o, 64);
    return x;
}

// One fused SSP-RK3 stage on the TX x TY tile whose first cell is (i0, j0).
// DUCT: the quasi-1D duct (one row, x faces of the duct areas, no r faces, wall
// force on axial momentum), a separate instantiation so that the axisymmetric and
// planar kernels carry none of its code.  NV: variables per cell, NVAR or NVAR_BI
// (two liquid populations: the passive scalars go in three groups, 5 + 5 + 4).
template <class R, int TX, int TY, bool DUCT = false, int NV = NVAR>
__device__ __forceinline__ void stage_tile(const StageArgs<R> &a, int i0, int j0, Tile<R, TX, TY> &t)
{
    using TileT = Tile<R, TX, TY>;
    constexpr int EX = TileT::EX, NE = TileT::N, NT = TX * TY;
    constexpr int RX = TileT::RX, NRG = TileT::NR;
    const BcInfo &bc = a.bc;
    const Metrics<R> &m = a.m;
    const int nx = bc.nx, nr = bc.nr;
    const int tid = threadIdx.x;
    const R pref = (R)a.pref;
    const bool axi = !DUCT && bc.geom == kGeomAxi;
    constexpr bool q1d = DUCT;

    // A tile whose 2-cell halo lies inside the mesh (most tiles) addresses its cells
    // directly; only boundary tiles go through the ghost-cell mapping.
    const bool inner = i0 >= 2 && j0 >= 2 && i0 + TX + 2 <= nx && j0 + TY + 2 <= nr;
    R(*face)[TileT::NF] = t.face();

    if (tid == 0) {
        t.nonzero[0] = t.nonzero[1] = t.nonzero[2] = 0;
        t.omask = 0;
    }
    // phase 1: gas primitives of tile + halo
    auto put_prims = [&](int e, R U0, R U1, R U2, R U3, R U4) {
        const R ir = trcp(U0);
        const R u = U1 * ir, v = U2 * ir, Y = U4 * ir;
        const R eint = U3 * ir - R(0.5) * (u * u + v * v);
        const R T = tdiv(eint + (R(1) - Y) * R(kCpa * kTref) - Y * R(kLv0 - kCpv * kTref), gas_cv(Y));
        t.rho[e] = U0;
        t.u[e] = u;
        t.v[e] = v;
        t.Y[e] = Y;
        t.T[e] = T;
        t.p[e] = U0 * gas_R(Y) * T;
    };
    if (inner) {
        // every load of the thread's cells is issued before the first is used: one
        // round trip to memory per tile rather than one per pass of the loop
        constexpr int NP = (NE + NT - 1) / NT;
        R Ub[NP][5];
        #pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int e = min(tid + q * NT, NE - 1);   // a spare lane reloads the last cell
            const unsigned code = (unsigned)((j0 + e / EX - 2) * nx + i0 + e % EX - 2);
            #pragma unroll
            for (int v = 0; v < 5; ++v) Ub[q][v] = ld_plane(a.Uin, a.plane, v, code);
        }
        #pragma unroll
        for (int q = 0; q < NP; ++q)
            if (tid + q * NT < NE) put_prims(tid + q * NT, Ub[q][0], Ub[q][1], Ub[q][2], Ub[q][3], Ub[q][4]);
    } else {
        // boundary tile: the sources of all the thread's cells (ghost cells mapped to
        // their mirror, copy or boundary state), then all their loads, then the primitives
        constexpr int NP = (NE + NT - 1) / NT;
        CellSrc cs[NP];
        R Ub[NP][5];
        #pragma unroll
        for (int q = 0; q < NP; ++q) {
            const int e = tid + q * NT;
            cs[q] = CellSrc{0, false, false};
            if (e < NE) cs[q] = map_cell(min(i0 + e % EX - 2, nx + 1), min(j0 + e / EX - 2, nr + 1), bc);
        }
        #pragma unroll
        for (int q = 0; q < NP; ++q)
            if (tid + q * NT < NE) {
                #pragma unroll
                for (int v = 0; v < 5; ++v) Ub[q][v] = fetch(a.Uin, a.plane, bc, cs[q].code, v);
            }
        #pragma unroll
        for (int q = 0; q < NP; ++q)
            if (tid + q * NT < NE)
                put_prims(tid + q * NT, Ub[q][0], cs[q].fu ? -Ub[q][1] : Ub[q][1], cs[q].fv ? -Ub[q][2] : Ub[q][2],
                          Ub[q][3], Ub[q][4]);
    }
    __syncthreads();
    // phase 2 (tile + ring): molecular viscosity, vapour diffusivity, eddy viscosity
    // mu_t = rho l^2 |du/dr + dv/dx|, and van Leer x slopes of the gas primitives (the
    // x-faces need them on the tile's rows only, not on the ring's first and last)
    for (int r = tid; r < NRG; r += NT) {
        const int l = ext_of_ring<TX, TY>(r);
        const int i = min(i0 + r % RX - 1, nx), j = min(j0 + r / RX - 1, nr);
        const R T = t.T[l];
        t.mu[r] = sutherland_t(T);
        t.D[r] = R(kD0) * fpow_pos(T * R(1.0 / kTref), R(kDexp)) * tdiv(R(kP0), t.p[l]);
        const R dudr = (t.u[l + EX] - t.u[l - EX]) * m.inv_d2r[j + 1];
        const R dvdx = (t.v[l + 1] - t.v[l - 1]) * m.inv_d2x[i + 1];
        t.mut[r] = t.rho[l] * m.lm2[i + 1] * fabs(dudr + dvdx);
        if (r >= RX && r < RX * (TY + 1)) {
            const R *w[5] = {t.rho, t.u, t.v, t.p, t.Y};
            #pragma unroll
            for (int k = 0; k < 5; ++k) t.sl[k][r - RX] = vl_slope(w[k][l] - w[k][l - 1], w[k][l + 1] - w[k][l]);
        }
    }
    __syncthreads();

    const int tx = tid % TX, ty = tid / TX;
    const int i = i0 + tx, j = j0 + ty;
    const bool valid = i < nx && j < nr;
    const int l = (ty + 2) * EX + tx + 2;
    const int rl = (ty + 1) * RX + tx + 1;

    // phase 3: x-faces, each once
    for (int f = tid; f < TileT::NFX; f += NT) {
        const int fi = f % (TX + 1), fj = f / (TX + 1);
        const int ig = min(i0 + fi, nx), jg = min(j0 + fj, nr);
        const int la = (fj + 2) * EX + fi + 1;
        const int ra = (fj + 1) * RX + fi;
        R F[5];
        gas_face<R>(t, la, ra, ra + 1, ra - RX, ra - RX + 1, 1, EX, true, m.inv_dxf[ig], m.inv_d2r[jg + 1],
                    m.inv_rc[jg + 1], pref, F);
        #pragma unroll
        for (int k = 0; k < 5; ++k) face[k][f] = F[k];
    }
    __syncthreads();
    R res[NV];
    R Fm0 = R(0), Fm1 = R(0), Fm2 = R(0), Fm3 = R(0), kd0 = R(0), kd1 = R(0), kd2 = R(0), kd3 = R(0);
    const R idx = valid ? m.inv_dx[i] : R(0);
    // everything a cell needs from the primitive arrays after the faces is read here,
    // before they are reused for the passive scalars: the cell's T (source-activity
    // test) and the axisymmetric pressure / hoop-stress source
    R Tcell = R(0), hoop = R(0);
    if (valid) {
        Tcell = t.T[l];
        if (axi) {   // (p - p_ref - tau_thetatheta) / r_c on radial momentum
            const R ir = m.inv_rc[j + 1];
            const R dudx = (t.u[l + 1] - t.u[l - 1]) * m.inv_d2x[i + 1];
            const R dvdr = (t.v[l + EX] - t.v[l - EX]) * m.inv_d2r[j + 1];
            const R vr = t.v[l] * ir;
            const R mue = t.mu[rl] + t.mut[rl];
            const R ttt = mue * (R(2) * vr - R(2.0 / 3.0) * (dudx + dvdr + vr));
            hoop = ((t.p[l] - pref) - ttt) * ir;
        }
    }
    if (valid) {
        const int fw = ty * (TX + 1) + tx;
        if (q1d) {
            // duct: the walls push with (p - p_ref)(A_e - A_w) on axial momentum, the
            // reference pressure having been taken out of the momentum fluxes as well
            const R aw = m.axf[i], ae = m.axf[i + 1], iv = m.invVx[i];
            #pragma unroll
            for (int k = 0; k < 5; ++k) res[k] = assemble_duct(face[k][fw + 1], ae, face[k][fw], aw, iv);
            res[1] += ((t.p[l] - pref) * (ae - aw)) * iv;
        } else {
            #pragma unroll
            for (int k = 0; k < 5; ++k) res[k] = assemble_x(face[k][fw + 1], face[k][fw], idx);
        }
        Fm0 = face[0][fw];
        Fm1 = face[0][fw + 1];
        kd0 = face_kd(t.mut[rl - 1], t.mut[rl], m.inv_dxf[i]);
        kd1 = face_kd(t.mut[rl], t.mut[rl + 1], m.inv_dxf[i + 1]);
    }
    // r-direction gas slopes, over the x slopes the x-faces no longer need: the r-faces
    // need them on the tile's columns only, not on the ring's first and last
    for (int q = tid; q < TX * (TY + 2); q += NT) {
        const int r = (q / TX) * RX + q % TX + 1;
        const int le = ext_of_ring<TX, TY>(r);
        const R *w[5] = {t.rho, t.u, t.v, t.p, t.Y};
        #pragma unroll
        for (int k = 0; k < 5; ++k) t.sl[k][q] = vl_slope(w[k][le] - w[k][le - EX], w[k][le + EX] - w[k][le]);
    }
    __syncthreads();
    // phase 4: r-faces, each once (the axis face has zero area)
    for (int f = tid; f < TileT::NFR; f += NT) {
        const int fi = f % TX, fj = f / TX;
        const int ig = min(i0 + fi, nx), jg = min(j0 + fj, nr);
        R F[5] = {R(0), R(0), R(0), R(0), R(0)};
        if (!(axi && jg == 0) && !q1d) {
            const int la = (fj + 1) * EX + fi + 2;
            const int ra = fj * RX + fi + 1;
            gas_face<R>(t, la, ra, ra + RX, f, f + TX, EX, 1, false, m.inv_drf[jg], m.inv_d2x[ig + 1],
                        m.inv_rf[jg], pref, F);
        }
        #pragma unroll
        for (int k = 0; k < 5; ++k) face[k][f] = F[k];
    }
    __syncthreads();
    if (valid) {
        const int fs = ty * TX + tx, fn = fs + TX;
        const R ivr = m.invV_r[j], as = m.rfa[j], an = m.rfa[j + 1];
        #pragma unroll
        for (int k = 0; k < 5; ++k) res[k] = assemble_r(res[k], face[k][fn], an, face[k][fs], as, ivr);
        Fm2 = face[0][fs];
        Fm3 = face[0][fn];
        if (!q1d) {   // the axis face's scalar flux is zeroed where it is used
            kd2 = face_kd(t.mut[rl - RX], t.mut[rl], m.inv_drf[j]);
            kd3 = face_kd(t.mut[rl], t.mut[rl + RX], m.inv_drf[j + 1]);
        }
        if (axi) res[2] += hoop;
    }
    // phase 5: passive scalars, five at a time in the freed primitive arrays.  T of
    // the cell is kept for the source-activity test.  A scalar
    // that is zero on the whole tile and halo (no particles there) has zero slopes
    // and zero fluxes, so its slope and flux work is skipped: the result is the same
    // zero (the stage output is bit-identical).
    constexpr int NG = (NV - 5 + 4) / 5;
    // Scalars that can be non-zero in the tile and its halo: the halo lies in the eight
    // neighbouring tiles, so the OR of their input masks; a ghost cell is a mirror or
    // copy of a cell of those tiles, or a boundary state (the inflow profile, the
    // ambient far field), whose scalars are in mask.ghost.  A scalar outside that set
    // is zero on the whole stencil, and is neither loaded nor transported.
    unsigned cand = ~0u, own_in = ~0u, own_un = ~0u;   // own_*: the tile's own words
    // scalars the output buffer may hold non-zero on the tile now (its mask before this
    // stage rewrites it at the end): a zero output of another scalar need not be stored
    unsigned old_out = ~0u;
    if (a.mask.in) {
        const int ti = i0 / TX, tj = j0 / TY, gx = a.mask.gx, gy = a.mask.gy;
        own_in = __builtin_amdgcn_readfirstlane(a.mask.in[tj * gx + ti]);
        if (a.mask.out) old_out = __builtin_amdgcn_readfirstlane(a.mask.out[tj * gx + ti]);
        if (a.mask.un) own_un = __builtin_amdgcn_readfirstlane(a.mask.un[tj * gx + ti]);
        cand = inner ? 0u : a.mask.ghost;
        #pragma unroll
        for (int dj = -1; dj <= 1; ++dj)
            #pragma unroll
            for (int di = -1; di <= 1; ++di)
                if (ti + di >= 0 && ti + di < gx && tj + dj >= 0 && tj + dj < gy)
                    cand |= a.mask.in[(tj + dj) * gx + ti + di];
        cand = __builtin_amdgcn_readfirstlane(cand);
    }
    // the first group may overwrite the primitive arrays at once: their last reader,
    // the r-face pass, is behind the barrier above
    int prev_live = 0;
    #pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int s0 = 5 + 5 * g;
        const int ng = NV - s0 < 5 ? NV - s0 : 5;   // scalars in this group
        const unsigned cg = (cand >> s0) & ((1u << ng) - 1u);   // block-uniform
        if (!cg) {   // nothing in this group can be non-zero here: zero residual, no work
            if (valid) {
                #pragma unroll
                for (int k = 0; k < 5; ++k)
                    if (k < ng) res[s0 + k] = R(0);
            }
            continue;
        }
        if (!q1d && inner && __builtin_popcount(cg) == 1) {
            // one candidate scalar on an interior tile: each cell reads its stencil of
            // that scalar straight from memory (the same per-mass values, slopes and
            // fluxes as through the tile's slots, without the load pass and its
            // barrier; a scalar zero on the cell's whole stencil gives the same zero)
            const int k = __builtin_ctz(cg);
            #pragma unroll
            for (int q = 0; q < 5; ++q)
                if (q < ng && q != k) res[s0 + q] = R(0);
            const unsigned c0 = (unsigned)(j * nx + i);
            auto phi = [&](int off, int le) {
                const R u = ld_plane(a.Uin, a.plane, s0 + k, c0 + (unsigned)off);
                const R rho = t.rho[le];
                return per_mass(u, rho, inv_rho(rho));
            };
            const R pc = phi(0, l), pw = phi(-1, l - 1), pe = phi(1, l + 1);
            const R pww = phi(-2, l - 2), pee = phi(2, l + 2);
            const R ps = phi(-nx, l - EX), pn = phi(nx, l + EX);
            const R pss = phi(-2 * nx, l - 2 * EX), pnn = phi(2 * nx, l + 2 * EX);
            const R sxw = vl_slope(pw - pww, pc - pw), sxc = vl_slope(pc - pw, pe - pc);
            const R sxe = vl_slope(pe - pc, pee - pe);
            const R fw = scalar_flux(pw, pc, sxw, sxc, Fm0, kd0);
            const R fe = scalar_flux(pc, pe, sxc, sxe, Fm1, kd1);
            const R srs_ = vl_slope(ps - pss, pc - ps), src = vl_slope(pc - ps, pn - pc);
            const R srn = vl_slope(pn - pc, pnn - pn);
            const R fs_raw = scalar_flux(ps, pc, srs_, src, Fm2, kd2);
            const R fsv = (axi && j == 0) ? R(0) : fs_raw;   // zero-area axis face
            const R fnv = scalar_flux(pc, pn, src, srn, Fm3, kd3);
            res[s0 + k] = assemble_r(assemble_x(fe, fw, idx), fnv, m.rfa[j + 1], fsv, m.rfa[j], m.invV_r[j]);
            continue;   // the slots were not written: prev_live stands
        }
        // the slots are free once every thread is done with the previous group's
        // fluxes; a group with nothing live read none of them
        if (prev_live) __syncthreads();
        int nz = 0;
        if (inner) {
            // as in phase 1: every load of the thread's cells is issued before the first
            // is used
            constexpr int NP = (NE + NT - 1) / NT;
            R ub[NP][5];
            #pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int e = min(tid + q * NT, NE - 1);   // a spare lane reloads the last cell
                const unsigned code = (unsigned)((j0 + e / EX - 2) * nx + i0 + e % EX - 2);
                #pragma unroll
                for (int k = 0; k < 5; ++k)
                    if (k < ng && (cg & (1u << k))) ub[q][k] = ld_plane(a.Uin, a.plane, s0 + k, code);
            }
            #pragma unroll
            for (int q = 0; q < NP; ++q) {
                const int e = tid + q * NT;
                if (e >= NE) continue;
                const R rho = t.rho[e], ir = inv_rho(rho);
                #pragma unroll
                for (int k = 0; k < 5; ++k) {
                    if (k >= ng || !(cg & (1u << k))) continue;
                    nz |= (ub[q][k] != R(0)) << k;
                    scalar_slot(t, k)[e] = per_mass(ub[q][k], rho, ir);
                }
            }
        } else {
            for (int e = tid; e < NE; e += NT) {
                const int code = map_cell(min(i0 + e % EX - 2, nx + 1), min(j0 + e / EX - 2, nr + 1), bc).code;
                const R rho = t.rho[e], ir = inv_rho(rho);
                #pragma unroll
                for (int k = 0; k < 5; ++k) {
                    if (k >= ng || !(cg & (1u << k))) continue;
                    const R u = fetch(a.Uin, a.plane, bc, code, s0 + k);
                    nz |= (u != R(0)) << k;
                    scalar_slot(t, k)[e] = per_mass(u, rho, ir);
                }
            }
        }
        if (nz) atomicOr(&t.nonzero[g], nz);
        __syncthreads();
        const int live = __builtin_amdgcn_readfirstlane(t.nonzero[g]);   // block-uniform
        prev_live = live;
        // the limited slopes of a live scalar are formed where the faces need them, from
        // the five cells on each axis through the cell (no slope pass, no barrier): the
        // same van Leer slopes, so the same fluxes
        if (valid) {
            R aw = R(0), ae = R(0), iv = R(0);
            if (q1d) {
                aw = m.axf[i];
                ae = m.axf[i + 1];
                iv = m.invVx[i];
            }
            #pragma unroll
            for (int k = 0; k < 5; ++k) {
                if (k >= ng) continue;
                if (!(live & (1 << k))) {
                    res[s0 + k] = R(0);
                    continue;
                }
                const R *ph = scalar_slot(t, k);
                const R pc = ph[l], pw = ph[l - 1], pe = ph[l + 1];
                const R sxw = vl_slope(pw - ph[l - 2], pc - pw), sxc = vl_slope(pc - pw, pe - pc);
                const R sxe = vl_slope(pe - pc, ph[l + 2] - pe);
                const R fw = scalar_flux(pw, pc, sxw, sxc, Fm0, kd0);
                const R fe = scalar_flux(pc, pe, sxc, sxe, Fm1, kd1);
                if (q1d) {
                    res[s0 + k] = assemble_duct(fe, ae, fw, aw, iv);
                } else {
                    const R ps = ph[l - EX], pn = ph[l + EX];
                    const R srs_ = vl_slope(ps - ph[l - 2 * EX], pc - ps), src = vl_slope(pc - ps, pn - pc);
                    const R srn = vl_slope(pn - pc, ph[l + 2 * EX] - pn);
                    const R fs_raw = scalar_flux(ps, pc, srs_, src, Fm2, kd2);
                    const R fsv = (axi && j == 0) ? R(0) : fs_raw;   // zero-area axis face
                    const R fnv = scalar_flux(pc, pn, src, srn, Fm3, kd3);
                    res[s0 + k] = assemble_r(assemble_x(fe, fw, idx), fnv, m.rfa[j + 1], fsv, m.rfa[j], m.invV_r[j]);
                }
            }
        }
    }
    // phase 6: SSP-RK3 combination with the transport residual.  Cells whose
    // phase-change source can be non-zero are appended to the active list; the
    // source kernel adds b dt Q(U^(s-1), dt) to them (the stage is linear in L).
    bool bad = false;
    unsigned obits = 0;   // non-zero scalars of the cell's output
    if (valid) {
        const long c = (long)j * nx + i;
        const double dt = a.dt_dev ? *a.dt_dev : a.dt;
        if (a.stage < 0) {
            #pragma unroll
            for (int v = 0; v < NV; ++v) {
                a.Uout[v * a.plane + c] = res[v];
                bad |= !isfinite(res[v]);
            }
        } else {
            const R rdt = (R)dt;
            // every load of the cell's old states is issued before the first store (the
            // compiler cannot rule out that Uout aliases them, and would otherwise wait
            // for each load in turn)
            // a scalar that is zero on the whole tile (its bit clear in the tile's mask)
            // is not loaded: zero either way, up to the sign of a zero, which no later
            // operation distinguishes
            R ui[NV], un[NV];
            #pragma unroll
            for (int v = 0; v < NV; ++v)
                ui[v] = (v < 5 || (own_in >> v) & 1u) ? ld_plane(a.Uin, a.plane, v, (unsigned)c) : R(0);
            if (a.stage > 0) {
                #pragma unroll
                for (int v = 0; v < NV; ++v)
                    un[v] = (v < 5 || (own_un >> v) & 1u) ? ld_plane(a.Un, a.plane, v, (unsigned)c) : R(0);
            }
            bool act = false;
            // liquid number of the cell for the pre-filter: either population
            R Mliq = ui[5];
            if constexpr (NV == NVAR_BI) Mliq = ui[15] > Mliq ? ui[15] : Mliq;
            if (a.sp.enabled && !(sizeof(R) == 4 && clearly_inactive<R>(ui[4], Mliq, ui[9], Tcell))) {
                double Ug[NV];
                #pragma unroll
                for (int v = 0; v < NV; ++v) Ug[v] = (v <= 5 || v == 9 || v == 15) ? (double)ui[v] : 0.0;
                CellThermo th;
                cell_thermo(Ug, th);
                act = !source_inactive<NV>(Ug, th.T);
            }
            // append the wavefront's active cells with one atomic
            const unsigned long long mask = __ballot(act);
            if (mask) {
                const int lane = __lane_id(), leader = __ffsll((long long)mask) - 1;
                int base = 0;
                if (lane == leader) base = atomicAdd(a.active_count, __popcll(mask));
                base = __shfl(base, leader, 64);
                if (act) {
                    const int slot = base + __popcll(mask & ((1ull << lane) - 1ull));
                    if (slot < a.plane) a.active_list[slot] = (int)c;
                }
            }
            // a scalar that no input can hold on the tile's stencil (no candidate, clear in
            // U^n's mask) has a zero output: +0, the value the arithmetic below gives, is
            // stored without it -- and not stored at all where the output buffer already
            // holds zero on the whole tile
            const unsigned zero_out = ~cand & (a.stage > 0 ? ~own_un : ~0u);
            #pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (v >= 5 && ((zero_out >> v) & 1u)) {   // block-uniform
                    if ((old_out >> v) & 1u) st_plane(a.Uout, a.plane, v, (unsigned)c, R(0));
                    continue;
                }
                const R L = res[v];
                R out;
                if (a.stage == 0) {
                    out = ui[v] + rdt * L;
                } else {
                    out = a.stage == 1 ? R(0.75) * un[v] + R(0.25) * (ui[v] + rdt * L)
                                       : R(1.0 / 3.0) * un[v] + R(2.0 / 3.0) * (ui[v] + rdt * L);
                }
                st_plane(a.Uout, a.plane, v, (unsigned)c, out);
                bad |= !isfinite(out);
                if (v >= 5) obits |= (out != R(0)) ? (1u << v) : 0u;
            }
        }
    }
    if (bad) atomicOr(a.flag, 1);
    // the output mask of the tile: OR over its cells, one word written by the tile
    if (a.mask.out) {
        obits = wave_or(obits);
        if ((tid & 63) == 0 && obits) atomicOr(&t.omask, obits);
        __syncthreads();
        if (tid == 0) a.mask.out[(j0 / TY) * a.mask.gx + i0 / TX] = t.omask;
    }
}

// FP32: registers held to 80 per lane (6 wavefronts per SIMD), which is what the
// LDS tile allows for 256-thread tiles; FP64 is held to three by both.  The
// 19-variable kernel (two liquid populations) is left free, so that it does not spill.
#define CP_STAGE_WAVES __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 6 : 1)))

template <class R, int TX, int TY, bool DUCT = false, int NV = NVAR>
__global__ void __launch_bounds__(TX *TY) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && NV == NVAR ? 6 : 1)))
k_stage(StageArgs<R> a)
{
    __shared__ Tile<R, TX, TY> t;
    // surrogate counters of the previous stage, consumed by now (saves a launch)
    if (a.sur_cnt && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) sur_fold_counts(a.sur_cnt, a.sur_tot);
    // tiles enumerated column by column, so that each XCD's contiguous band holds
    // whole columns: every XCD then sees the full radial structure of the jet (core,
    // shear layer, far field) and its share of the boundary tiles
    const int gx = gridDim.x, gy = gridDim.y;
    const int tb = xcd_band(blockIdx.y * gx + blockIdx.x, gx * gy);
    stage_tile<R, TX, TY, DUCT, NV>(a, (tb / gy) * TX, (tb % gy) * TY, t);
}

// Batched operating points: workgroup b takes work item b (XCD-banded) of a list of
// (plume, tile) pairs and runs the stage of that plume's tile.
template <class R, int TX, int TY>
__global__ void __launch_bounds__(TX *TY) CP_STAGE_WAVES k_stage_batch(const StageArgs<R> *args, const int *work_plume,
                                                        const int *work_tile, int nwork)
{
    __shared__ Tile<R, TX, TY> t;
    const int w = xcd_band(blockIdx.x, nwork);
    const int p = work_plume[w], tb = work_tile[w];
    // the plume's arguments are read from the table once, at the start, into scalar
    // registers as kernel arguments are (reading each field from the table where it is
    // used made the batch's step 16 % slower)
    const StageArgs<R> a = args[p];
    const int gx = (a.bc.nx + TX - 1) / TX;
    stage_tile<R, TX, TY>(a, (tb % gx) * TX, (tb / gx) * TY, t);
}

// Phase-change source of the listed cells: U^(s) += b dt Q(U^(s-1), dt), b the
// weight of L in the stage (1, 1/4, 2/3).  Q is evaluated in FP64.  Clears the
// list counter of the next stage.
template <class R, int NV = NVAR>
__device__ __forceinline__ void source_fix_body(const SourceFixArgs<R> &a, int bx, int nbx)
{
    const int n = (int)min((long)*a.count, a.plane);
    const double dt = a.dt_dev ? *a.dt_dev : a.dt;
    const double b = a.stage == 0 ? 1.0 : (a.stage == 1 ? 0.25 : 2.0 / 3.0);
    int ns = 0;
    bool bad = false;
    for (int k = bx * blockDim.x + threadIdx.x; k < n; k += nbx * blockDim.x) {
        const long c = a.list[k];
        double Ud[NV], Q[NV];
        #pragma unroll
        for (int v = 0; v < NV; ++v) Ud[v] = (double)a.Uin[v * a.plane + c];
        ns += source_integrate_nv<NV>(Ud, dt, a.sp, Q);
        R uo[NV];   // all loads before the stores (possible aliasing serialises them)
        #pragma unroll
        for (int v = 0; v < NV; ++v) uo[v] = a.Uout[v * a.plane + c];
        unsigned bits = 0;
        #pragma unroll
        for (int v = 0; v < NV; ++v) {
            const R out = uo[v] + (R)(b * dt * Q[v]);
            a.Uout[v * a.plane + c] = out;
            bad |= !isfinite(out);
            if (v >= 5) bits |= (out != R(0)) ? (1u << v) : 0u;
        }
        mask_mark(a.mask, c, bits);
    }
    if (bx == 0 && threadIdx.x == 0 && a.next_count) *a.next_count = 0;
    if (bad) atomicOr(a.flag, 1);
    for (int o = 32; o > 0; o >>= 1) ns += __shfl_xor(ns, o, 64);
    if ((threadIdx.x & 63) == 0 && ns && a.nsub) atomicAdd(a.nsub, (unsigned long long)ns);
}

// One wavefront per workgroup: the active cells are a small, compact fraction of
// the mesh, so they are spread over as many compute units as possible.
// A workgroup with no listed cell leaves at once, before any of the source code
// is fetched (most stages of a jet have no source-active cell at all).
template <class R, int NV = NVAR> __global__ void __launch_bounds__(64) k_source_fix(SourceFixArgs<R> a)
{
    if ((long)blockIdx.x * blockDim.x >= min((long)*a.count, a.plane)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && a.next_count) *a.next_count = 0;
        return;
    }
    source_fix_body<R, NV>(a, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ drift
// Droplets and crystals lag the gas's pressure-driven acceleration with their
// Stokes terminal slip w(r) = 2 rho_p r^2 Cc(r) (1 - rho/rho_p) (dp/dn) / (9 mu rho),
// Cc = 1 + 2 A_C Kn, Kn = lbar / (2 r) (Eq. 24 in the Stokes regime).  A population
// drifts as a whole with the slip of its mean radius r20: every moment crosses a
// face with w(r20) M_k, upwind in its sign (the moment set stays realisable); face
// means of rho, mu, p, T and R; lbar = 1.5 mu sqrt(R T) / p.
struct DriftCell {
    double rho, p, T, Rm, mu, M[8];   // M: liquid then ice moments per unit volume
};

template <class R> __device__ __forceinline__ DriftCell drift_cell(const R *U, long plane, const BcInfo &bc, int i, int j)
{
    const CellSrc cs = map_cell(i, j, bc);
    double u[NVAR];
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) u[v] = (double)fetch(U, plane, bc, cs.code, v);
    CellThermo th;
    cell_thermo(u, th);   // the momentum flips of mirror cells do not change these
    DriftCell d;
    d.rho = th.rho;
    d.p = th.p;
    d.T = th.T;
    d.Rm = th.Rm;
    d.mu = sutherland<double>(th.T);
    #pragma unroll
    for (int k = 0; k < 8; ++k) d.M[k] = u[5 + k];
    return d;
}

// Terminal slip with the Schiller-Naumann factor of Eq. 24: w (1 + 0.15 Re^0.687) =
// w_St, Re = rho |w| 2 r / mu (on the diameter, the number with which C_D Re -> 24 is
// Stokes's law), six fixed-point steps from the Stokes-Cunningham slip w_St.
__device__ __forceinline__ double sn_slip(double w_st, double rho, double r, double mu)
{
    double w = w_st;
    #pragma unroll 1
    for (int it = 0; it < 6; ++it) w = w_st / (1.0 + 0.15 * pow(rho * fabs(w) * 2.0 * r / mu, 0.687));
    return w;
}

// Drift fluxes of the 8 moments through the face from cell a to cell b.
__device__ __forceinline__ void drift_face(const DriftCell &a, const DriftCell &b, double dn, double *F)
{
    const double rho = 0.5 * (a.rho + b.rho), mu = 0.5 * (a.mu + b.mu);
    const double p = 0.5 * (a.p + b.p), T = 0.5 * (a.T + b.T), Rm = 0.5 * (a.Rm + b.Rm);
    const double lbar = 1.5 * mu * sqrt(Rm * T) / p;
    const double dpdn = (b.p - a.p) / dn;
    #pragma unroll
    for (int pop = 0; pop < 2; ++pop) {
        const double rho_p = pop ? kRhoS : kRhoL;
        const double c = 2.0 * rho_p * (1.0 - rho / rho_p) * dpdn / (9.0 * mu * rho);
        const double *M = (c > 0.0 ? a.M : b.M) + 4 * pop;
        #pragma unroll
        for (int k = 0; k < 4; ++k) F[4 * pop + k] = 0.0;
        if (!pop_valid(M[0], M[2], M[3])) continue;
        const double r20 = sqrt(M[2] / M[0]);
        const double Kn = lbar / (2.0 * r20);
        const double W = sn_slip(c * r20 * r20 * (1.0 + 2.0 * (1.257 + 0.4 * exp(-1.1 / (2.0 * Kn))) * Kn), rho,
                                 r20, mu);
        #pragma unroll
        for (int k = 0; k < 4; ++k) F[4 * pop + k] = W * M[k];
    }
}

__device__ __forceinline__ bool has_particles(const DriftCell &d)
{
    return d.M[0] > kNmin || d.M[4] > kNmin;
}

template <class R> __global__ void __launch_bounds__(256) k_drift(DriftArgs<R> a)
{
    const BcInfo &bc = a.bc;
    const int i = blockIdx.x * 64 + threadIdx.x % 64, j = blockIdx.y * 4 + threadIdx.x / 64;
    if (i >= bc.nx || j >= bc.nr) return;
    const DriftCell C = drift_cell(a.Uin, a.plane, bc, i, j);
    const DriftCell W = drift_cell(a.Uin, a.plane, bc, i - 1, j), E = drift_cell(a.Uin, a.plane, bc, i + 1, j);
    const DriftCell S = drift_cell(a.Uin, a.plane, bc, i, j - 1), N = drift_cell(a.Uin, a.plane, bc, i, j + 1);
    if (!(has_particles(C) || has_particles(W) || has_particles(E) || has_particles(S) || has_particles(N))) return;
    double Fw[8], Fe[8], Fs[8], Fn[8];
    drift_face(W, C, a.xc[i + 2] - a.xc[i + 1], Fw);
    drift_face(C, E, a.xc[i + 3] - a.xc[i + 2], Fe);
    drift_face(S, C, a.rc[j + 2] - a.rc[j + 1], Fs);
    drift_face(C, N, a.rc[j + 3] - a.rc[j + 2], Fn);
    const double idx = a.inv_dx[i], as = a.rfa[j], an = a.rfa[j + 1], ivr = a.invV_r[j];
    const bool axis = bc.geom == kGeomAxi && j == 0;   // zero-area axis face
    double w = 1.0;
    if (a.stage >= 0) {
        const double dt = a.dt_dev ? *a.dt_dev : a.dt;
        w = (a.stage == 0 ? 1.0 : (a.stage == 1 ? 0.25 : 2.0 / 3.0)) * dt;
    }
    const long c = (long)j * bc.nx + i;
    bool bad = false;
    #pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double rd = -(Fe[k] - Fw[k]) * idx - (Fn[k] * an - (axis ? 0.0 : Fs[k] * as)) * ivr;
        const R out = a.Uout[(5 + k) * a.plane + c] + (R)(w * rd);
        a.Uout[(5 + k) * a.plane + c] = out;
        bad |= !isfinite(out);
    }
    if (bad) atomicOr(a.flag, 1);
}

// batched: blockIdx.y selects the plume; one wavefront per workgroup, and a
// workgroup past the plume's listed cells leaves at once (as in k_source_fix)
template <class R> __global__ void __launch_bounds__(64) k_source_fix_batch(const SourceFixArgs<R> *args)
{
    const SourceFixArgs<R> &a = args[blockIdx.y];
    if ((long)blockIdx.x * blockDim.x >= min((long)*a.count, a.plane)) {
        if (blockIdx.x == 0 && threadIdx.x == 0 && a.next_count) *a.next_count = 0;
        return;
    }
    source_fix_body(a, blockIdx.x, gridDim.x);
}

// ------------------------------------------------------------------ surrogate
__device__ __forceinline__ uint16_t to_bf16(float f)
{
    uint32_t b = __float_as_uint(f);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Raw network features of one cell (asinh-scaled state, ln dt, log10 of the soot
// number) and its liquid saturation ln S_l; shared by the gate and the feature
// export used to build training sets, so both see identical inputs.
template <class R>
__device__ __forceinline__ double sur_raw_features(const R *U, long plane, long c, double dt, const float *s_in,
                                                   float *f, double *T = nullptr, double *M0 = nullptr)
{
    double Ud[NVAR];
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) Ud[v] = (double)U[v * plane + c];
    CellThermo th;
    cell_thermo(Ud, th);
    if (T) *T = th.T;
    if (M0) *M0 = Ud[5];
    const double pv = fmax(Ud[4] * kRv * th.T, kPvFloor);
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) f[v] = asinhf((float)(Ud[v] / (double)s_in[v]));
    f[15] = (float)log(dt);
    f[16] = (float)log10(fmax(Ud[13], 1.0));
    return log(pv) - ln_psat(kSonW, th.T);
}

template <class R>
__global__ void __launch_bounds__(256) k_sur_features(const R *U, long plane, double dt, SurNorm nm, float *F)
{
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < plane; c += (long)gridDim.x * blockDim.x) {
        float f[17];
        double T;
        const double lnSl = sur_raw_features(U, plane, c, dt, nm.s_in, f, &T);
        #pragma unroll
        for (int q = 0; q < 17; ++q) F[c * 19 + q] = f[q];
        F[c * 19 + 17] = (float)lnSl;
        F[c * 19 + 18] = (float)T;
    }
}

// The gate: the network takes a cell whose standardised features lie inside the
// training envelope, whose vapour is not near saturation (|ln S_l| >= lnS_gate) and
// whose droplets cannot freeze (no droplets, or the gas at or above the melting
// point); every other cell keeps the exact source.  Freezing (Eq. 12-15) changes the
// crystal number by orders of magnitude per kelvin: that regime stays with the exact
// source.  f receives the standardised features.
template <class R> __device__ __forceinline__ bool sur_gate_cell(const SurArgs<R> &a, long c, double dt, float *f)
{
    double T, M0;
    const double lnSl = sur_raw_features(a.Uin, a.plane, c, dt, a.nm.s_in, f, &T, &M0);
    const bool freezing = T < kTmelt && M0 > kNmin;
    bool inside = !freezing && fabs(lnSl) >= (double)a.nm.lnS_gate && lnSl >= (double)a.nm.lnS_lo &&
                  lnSl <= (double)a.nm.lnS_hi;
    #pragma unroll
    for (int q = 0; q < 17; ++q) {
        f[q] = (f[q] - a.nm.mu_in[q]) / a.nm.sd_in[q];
        inside = inside && f[q] >= a.nm.lo[q] && f[q] <= a.nm.hi[q];
    }
    return inside;
}

// Gate and network in one launch.  Each workgroup takes the active cells 64 at a time:
// its first wavefront gates one cell per lane, appends the rejected cells to the
// fallback list and packs the accepted ones into the rows of the network's input tile
// (one counter update per wavefront for each list), and the whole workgroup then
// evaluates the network on those rows (fused_net_tile), whose outputs land in Y at the
// rows the cells were given in mlp_cells.  The workgroups stride over the list.
template <class R>
__global__ void __launch_bounds__(256, 2) k_sur_gate_net(SurArgs<R> a, FusedNet w, float *Y)
{
    __shared__ FusedXTile Xs;
    __shared__ FusedHTile Hs;
    __shared__ int tile_rows, tile_base;
    const int n = (int)min((long)*a.count, a.plane);
    if ((long)blockIdx.x * 64 >= n) return;   // no listed cell for this workgroup
    const double dt = a.dt_dev ? *a.dt_dev : a.dt;
    const int lane = threadIdx.x & 63;
    for (int m0 = blockIdx.x * 64; m0 < n; m0 += gridDim.x * 64) {
        if (threadIdx.x < 64) {
            const int k = m0 + lane;
            const bool listed = k < n;
            bool inside = false;
            long c = 0;
            float f[17];
            if (listed) {
                c = a.list[k];
                inside = sur_gate_cell(a, c, dt, f);
            }
            const unsigned long long in_mask = __ballot(inside), fb_mask = __ballot(listed && !inside);
            const unsigned long long below = (1ull << lane) - 1ull;
            int base = 0, fbase = 0;
            if (lane == 0) {
                if (in_mask) base = atomicAdd(a.cnt, __popcll(in_mask));
                if (fb_mask) fbase = atomicAdd(a.cnt + 1, __popcll(fb_mask));
            }
            base = __shfl(base, 0, 64);
            fbase = __shfl(fbase, 0, 64);
            const int rows = __popcll(in_mask);
            if (listed && !inside) a.fb_list[fbase + __popcll(fb_mask & below)] = (int)c;
            if (inside) {
                const int r = __popcll(in_mask & below);
                a.mlp_cells[base + r] = (int)c;
                #pragma unroll
                for (int q = 0; q < kFusedKin; ++q) Xs[r][q] = q < 17 ? to_bf16(f[q]) : (uint16_t)0;
            }
            if (lane >= rows) {   // the tile's unused rows are zero
                #pragma unroll
                for (int q = 0; q < kFusedKin; ++q) Xs[lane][q] = 0;
            }
            if (lane == 0) {
                tile_rows = rows;
                tile_base = base;
            }
        }
        __syncthreads();
        const int rows = tile_rows, base = tile_base;   // block-uniform
        if (rows > 0)
            fused_net_tile(w, Xs, Hs, rows, 15, Y + (long)base * 15);   // ends with a barrier
        else
            __syncthreads();   // every wave has read tile_rows before it is rewritten
    }
}

// A particle population after a network update is acceptable when it is empty (at
// most kNmin particles carrying at most the mass of kNmin 1 mm particles) or when
// its moments are those of a distribution: positive, log-convex (Cauchy-Schwarz,
// m1^2 <= m0 m2 and m2^2 <= m1 m3) and with a mean radius between 0.1 nm and 1 mm.
__device__ __forceinline__ bool sur_population_ok(double m0, double m1, double m2, double m3)
{
    if (m0 <= kNmin) return m3 <= kNmin * 1e-9;
    const double slack = 1.0 + 1e-6;
    return m1 > 0.0 && m2 > 0.0 && m3 > 0.0 && m1 * m1 <= m0 * m2 * slack && m2 * m2 <= m1 * m3 * slack &&
           m1 >= m0 * 1e-10 && m1 <= m0 * 1e-3;
}

// Decode the network output of row k into the particle sources and close the rest
// exactly.  The network predicts, for each particle moment and the activated-soot
// number, the increment of its feature over dt; the new value s sinh(f + df)
// (floored at zero) gives Q_v = (U'_v - U_v) / dt.  The vapour sink then follows
// from the condensate sources (water exactly conserved), the gas mass and momentum
// follow the vapour, the gas energy loses the enthalpy of the condensed water (the
// freezing enthalpy cancels between the two condensates) and the soot number is
// unchanged.  Returns false (the cell takes the exact source) when a predicted
// increment leaves the trust bound df_max (df_max_ice for the crystal moments, whose
// freezing source the network reproduces least well), a population is not realizable after
// the update, the vapour would turn negative or a value is not finite.
template <class R>
__device__ __forceinline__ bool sur_decode(const SurArgs<R> &a, int k, const double *Ud, double dt, double *Q)
{
    double Un[NVAR];
    bool trust = true;
    #pragma unroll
    for (int v = 5; v < NVAR; ++v) {
        if (v == 13) continue;
        const double s = (double)a.nm.s_in[v];
        const double df = (double)(a.Y[(long)k * 15 + v] * a.nm.sd_out[v] + a.nm.mu_out[v]);
        trust = trust && fabs(df) <= (double)((v >= 9 && v <= 12) ? a.nm.df_max_ice : a.nm.df_max);
        const double f1 = fmax(asinh(Ud[v] / s) + df, 0.0);
        Un[v] = s * sinh(f1);
        Q[v] = (Un[v] - Ud[v]) / dt;
    }
    Q[13] = 0.0;
    trust = trust && sur_population_ok(Un[5], Un[6], Un[7], Un[8]) && sur_population_ok(Un[9], Un[10], Un[11], Un[12]);
    // at most the soot present can be activated (the soot number is unchanged)
    trust = trust && Un[14] <= Ud[13] * (1.0 + 1e-12);
    CellThermo th;
    cell_thermo(Ud, th);
    const double ml = kFourThirdsPi * kRhoL * Q[8], ms = kFourThirdsPi * kRhoS * Q[12];
    Q[4] = -(ml + ms);
    Q[0] = Q[4];
    Q[1] = Q[4] * th.u;
    Q[2] = Q[4] * th.v;
    const double T = th.T;
    const double hfg = kLv0 + (kCpv - kCl) * (T - kTref);
    const double hsg = kLs0 + (kCpv - kCi) * (T - kTref);
    const double hv = kLv0 + kCpv * (T - kTref);
    const double ke = 0.5 * (th.u * th.u + th.v * th.v);
    Q[3] = -ml * (hv - hfg + ke) - ms * (hv - hsg + ke);
    bool ok = trust && Ud[4] + dt * Q[4] >= 0.0;
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) ok = ok && isfinite(Q[v]);
    return ok;
}

// Second half of a surrogate stage: the network rows (decoded, or given the exact
// source where the decode is rejected) followed by the gate's fallback cells (exact
// source), each adding b dt Q to the stage output -- or, for cp_source (q_only),
// writing the network's Q over the exact Q already in place.  Clears the list
// counter of the next stage like the exact source kernel.
template <class R> __global__ void __launch_bounds__(64) k_sur_finish(SurArgs<R> a, SourceParams sp,
                                                                      int *next_count, unsigned long long *nsub)
{
    const int n_net = min(a.cnt[0], (int)a.plane), n_fb = min(a.cnt[1], (int)a.plane);
    if ((long)blockIdx.x * blockDim.x >= (long)n_net + n_fb) {   // no row for this workgroup
        if (blockIdx.x == 0 && threadIdx.x == 0 && next_count) *next_count = 0;
        return;
    }
    const double dt = a.dt_dev ? *a.dt_dev : a.dt;
    const double b = a.stage == 0 ? 1.0 : (a.stage == 1 ? 0.25 : 2.0 / 3.0);
    bool bad = false;
    int ns = 0, rejected = 0;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_net + n_fb; k += gridDim.x * blockDim.x) {
        const bool net = k < n_net;
        const long c = net ? a.mlp_cells[k] : a.fb_list[k - n_net];
        double Ud[NVAR], Q[NVAR];
        #pragma unroll
        for (int v = 0; v < NVAR; ++v) Ud[v] = (double)a.Uin[v * a.plane + c];
        bool exact = !net;
        if (net && !sur_decode(a, k, Ud, dt, Q)) {
            exact = true;
            ++rejected;
        }
        if (a.q_only) {   // the exact source is already in the output
            if (!exact) {
                #pragma unroll
                for (int v = 0; v < NVAR; ++v) a.Uout[v * a.plane + c] = (R)Q[v];
            }
            continue;
        }
        if (exact) ns += source_integrate(Ud, dt, sp, Q);
        R uo[NVAR];   // all loads before the stores (possible aliasing serialises them)
        #pragma unroll
        for (int v = 0; v < NVAR; ++v) uo[v] = a.Uout[v * a.plane + c];
        unsigned bits = 0;
        #pragma unroll
        for (int v = 0; v < NVAR; ++v) {
            const R out = uo[v] + (R)(b * dt * Q[v]);
            a.Uout[v * a.plane + c] = out;
            bad |= !isfinite(out);
            if (v >= 5) bits |= (out != R(0)) ? (1u << v) : 0u;
        }
        mask_mark(a.mask, c, bits);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && next_count) *next_count = 0;
    if (bad) atomicOr(a.flag, 1);
    for (int o = 32; o > 0; o >>= 1) {
        ns += __shfl_xor(ns, o, 64);
        rejected += __shfl_xor(rejected, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (ns && nsub) atomicAdd(nsub, (unsigned long long)ns);
        if (rejected) atomicAdd(a.cnt + 2, rejected);
    }
}

// Cells whose phase-change source does not vanish identically (the FP64 test the
// stage kernel applies after its storage-precision pre-filter).
template <class R> __global__ void __launch_bounds__(256) k_active_list(const R *U, long plane, int *count, int *list)
{
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < plane; c += (long)gridDim.x * blockDim.x) {
        double Ud[NVAR];
        #pragma unroll
        for (int v = 0; v < NVAR; ++v) Ud[v] = (double)U[v * plane + c];
        CellThermo th;
        cell_thermo(Ud, th);
        if (!source_inactive(Ud, th.T)) list[atomicAdd(count, 1)] = (int)c;
    }
}

__global__ void k_sur_reset(int *cnt, unsigned long long *tot) { sur_fold_counts(cnt, tot); }

// Drag-law diagnostics (Eq. 24): response time of the droplets and of the crystals
// at their mean radius r20, tau_p = rho_p (2 r20)^2 Cc / (18 mu) (zero slip), and the
// Stokes number tau_p |u| / dx_i; planes [2][nr][nx], zero without a population.
template <class R>
__global__ void __launch_bounds__(256) k_particle_times(const R *U, long plane, int nx, const double *inv_dx,
                                                        double *tau, double *St)
{
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < plane; c += (long)gridDim.x * blockDim.x) {
        double u[NVAR];
        #pragma unroll
        for (int v = 0; v < NVAR; ++v) u[v] = (double)U[v * plane + c];
        CellThermo th;
        cell_thermo(u, th);
        const double mu = sutherland<double>(th.T);
        const double lbar = 1.5 * mu * sqrt(th.Rm * th.T) / th.p;
        const double speed = sqrt(th.u * th.u + th.v * th.v);
        #pragma unroll
        for (int pop = 0; pop < 2; ++pop) {
            const double *M = u + (pop ? 9 : 5);
            const double rho_p = pop ? kRhoS : kRhoL;
            double t = 0.0;
            if (pop_valid(M[0], M[2], M[3])) {
                const double r20 = sqrt(M[2] / M[0]);
                const double Kn = lbar / (2.0 * r20);
                const double Cc = 1.0 + 2.0 * (1.257 + 0.4 * exp(-1.1 / (2.0 * Kn))) * Kn;
                t = rho_p * (2.0 * r20) * (2.0 * r20) * Cc / (18.0 * mu);
            }
            tau[pop * plane + c] = t;
            St[pop * plane + c] = t * speed * inv_dx[c % nx];
        }
    }
}

// Tile masks of a state (one workgroup per tile of the given shape).
template <class R>
__global__ void __launch_bounds__(256) k_tile_mask(const R *U, long plane, int nx, int nr, int nv, int tx, int ty,
                                                   unsigned *mask, unsigned *unknown_a, unsigned *unknown_b)
{
    __shared__ unsigned acc;
    const int gx = (nx + tx - 1) / tx;
    const int ti = blockIdx.x % gx, tj = blockIdx.x / gx;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    unsigned bits = 0;
    for (int e = threadIdx.x; e < tx * ty; e += blockDim.x) {
        const int i = ti * tx + e % tx, j = tj * ty + e / tx;
        if (i >= nx || j >= nr) continue;
        const long c = (long)j * nx + i;
        for (int v = 5; v < nv; ++v) bits |= (U[v * plane + c] != R(0)) ? (1u << v) : 0u;
    }
    bits = wave_or(bits);
    if ((threadIdx.x & 63) == 0 && bits) atomicOr(&acc, bits);
    __syncthreads();
    if (threadIdx.x == 0) {
        mask[blockIdx.x] = acc;
        // the stage buffers: whatever they hold now is not known to be zero anywhere
        if (unknown_a) unknown_a[blockIdx.x] = ~0u;
        if (unknown_b) unknown_b[blockIdx.x] = ~0u;
    }
}

// ------------------------------------------------------------------ CFL
// Per-cell limit 1/((|u|+c)/dx + (|v|+c)/dr + 2 nu_eff (1/dx^2 + 1/dr^2)), written
// without contraction so that the FP64 result is reproducible operation by
// operation; the block minimum is merged with an unsigned 64-bit atomic min (the
// bit patterns of positive doubles order like the values).
struct PrimD {
    double rho, u, v, T, Y;
};

__device__ __forceinline__ PrimD cfl_prim_of(double U0, double U1, double U2, double U3, double U4)
{
#pragma clang fp contract(off)
    PrimD w;
    w.rho = U0;
    w.u = U1 / U0;
    w.v = U2 / U0;
    w.Y = U4 / U0;
    const double e = U3 / U0 - 0.5 * (w.u * w.u + w.v * w.v);
    const double cv = (1.0 - w.Y) * kCva + w.Y * kCvv;
    w.T = (e + (1.0 - w.Y) * kCpa * kTref - w.Y * (kLv0 - kCpv * kTref)) / cv;
    return w;
}

// Time-step limit of cell (i, j) from its primitives and the neighbour velocities
// that enter the eddy viscosity.
template <class R>
__device__ __forceinline__ double cfl_limit(const CflArgs<R> &a, int i, int j, const PrimD &w, double uN, double uS,
                                            double vE, double vW)
{
#pragma clang fp contract(off)
    const double dudr = (uN - uS) / (a.rc[j + 3] - a.rc[j + 1]);
    const double dvdx = (vE - vW) / (a.xc[i + 3] - a.xc[i + 1]);
    const double lm = a.kappa_m * (a.delta0 + a.s_delta * a.xc[i + 2]);
    const double mut = w.rho * lm * lm * fabs(dudr + dvdx);
    const double Rm = (1.0 - w.Y) * kRa + w.Y * kRv;
    const double cpm = (1.0 - w.Y) * kCpa + w.Y * kCpv;
    const double cvm = (1.0 - w.Y) * kCva + w.Y * kCvv;
    const double gam = cpm / cvm;
    const double snd = sqrt(gam * Rm * w.T);
    const double t = w.T / kTref;
    const double mu = kMu0 * t * sqrt(t) * (kTref + kSuth) / (w.T + kSuth);
    double fac = gam / kPr;
    if (fac < 4.0 / 3.0) fac = 4.0 / 3.0;
    const double nu = (mu + mut) / w.rho * fac;
    const double idx = a.inv_dx[i], idr = a.inv_dr[j];
    const double rate = (fabs(w.u) + snd) * idx + (fabs(w.v) + snd) * idr + 2.0 * nu * (idx * idx + idr * idr);
    return 1.0 / rate;
}

// Block minimum (wavefront shuffles, then LDS).  With a per-workgroup array the
// block writes its minimum there and the finalize kernel reduces the array (no
// atomics on one word, which serialise across thousands of workgroups); otherwise
// it is merged into the running minimum with a 64-bit atomic min, issued only when
// it is below the value the block reads (the minimum only decreases).  A
// non-positive limit is recorded as 0, so dt collapses to 0 (reported as CP_EDT).
__device__ __forceinline__ void cfl_block_min(double best, unsigned long long *acc, double *block_min)
{
    for (int o = 32; o > 0; o >>= 1) best = fmin(best, __shfl_xor(best, o, 64));
    __shared__ double part[16];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = part[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k) b = fmin(b, part[k]);
        if (block_min) {
            block_min[blockIdx.y * gridDim.x + blockIdx.x] = b > 0.0 ? b : 0.0;
        } else {
            const unsigned long long key = b > 0.0 ? (unsigned long long)__double_as_longlong(b) : 0ull;
            if (key < __hip_atomic_load(acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(acc, key);
        }
    }
}

// The same limit in the storage precision of the mixed path: FP32 arithmetic with the
// hardware reciprocal and square root (the time step needs no more than the state it
// advances); the minimum is merged as a double.
struct PrimF {
    float rho, u, v, T, Y;
};

__device__ __forceinline__ PrimF cfl_prim_f32_of(float U0, float U1, float U2, float U3, float U4)
{
#pragma clang fp contract(off)   // the same operations wherever it is inlined
    const float ir = __builtin_amdgcn_rcpf(U0);
    PrimF w;
    w.rho = U0;
    w.u = U1 * ir;
    w.v = U2 * ir;
    w.Y = U4 * ir;
    const float e = U3 * ir - 0.5f * (w.u * w.u + w.v * w.v);
    const float cv = (1.0f - w.Y) * float(kCva) + w.Y * float(kCvv);
    w.T = (e + (1.0f - w.Y) * float(kCpa * kTref) - w.Y * float(kLv0 - kCpv * kTref)) * __builtin_amdgcn_rcpf(cv);
    return w;
}

__device__ __forceinline__ float cfl_limit_f32(const CflArgs<float> &a, int i, int j, const PrimF &w, float uN,
                                               float uS, float vE, float vW)
{
#pragma clang fp contract(off)
    const float dudr = (uN - uS) * a.f_d2r[j + 1];
    const float dvdx = (vE - vW) * a.f_d2x[i + 1];
    const float mut = w.rho * a.f_lm2[i + 1] * fabsf(dudr + dvdx);
    const float Rm = (1.0f - w.Y) * float(kRa) + w.Y * float(kRv);
    const float cpm = (1.0f - w.Y) * float(kCpa) + w.Y * float(kCpv);
    const float cvm = (1.0f - w.Y) * float(kCva) + w.Y * float(kCvv);
    const float gam = cpm * __builtin_amdgcn_rcpf(cvm);
    const float snd = __builtin_amdgcn_sqrtf(gam * Rm * w.T);
    const float t = w.T * float(1.0 / kTref);
    const float mu = float(kMu0) * t * __builtin_amdgcn_sqrtf(t) * float(kTref + kSuth) * __builtin_amdgcn_rcpf(w.T + float(kSuth));
    const float fac = fmaxf(gam * float(1.0 / kPr), 4.0f / 3.0f);
    const float nu = (mu + mut) * __builtin_amdgcn_rcpf(w.rho) * fac;
    const float idx = a.f_idx[i], idr = (float)a.inv_dr[j];
    const float rate = (fabsf(w.u) + snd) * idx + (fabsf(w.v) + snd) * idr + 2.0f * nu * (idx * idx + idr * idr);
    return __builtin_amdgcn_rcpf(rate);
}

// BX x BY threads over a BX x (BY * RPT) tile (RPT rows per thread).  A tile whose
// 1-cell ring lies inside the mesh loads its cells directly, all five variables at
// once; boundary tiles go through the ghost-cell mapping.
template <int BX, int BY, int RPT> __device__ __forceinline__ void cfl_tile_f32_body(const CflArgs<float> &a, int bxi,
                                                                                     int byi)
{
    constexpr int TY = BY * RPT, EXC = BX + 2, NEC = EXC * (TY + 2);
    __shared__ float pr[5][NEC];
    const BcInfo &bc = a.bc;
    const int i0 = bxi * BX, j0 = byi * TY;
    const bool inner = i0 >= 1 && j0 >= 1 && i0 + BX + 1 <= bc.nx && j0 + TY + 1 <= bc.nr;
    if (inner) {
        // every load of the thread's ring cells in flight before the first use
        constexpr int NT = BX * BY, IT = (NEC + NT - 1) / NT;
        float q[IT][5];
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                const float *u = a.U + (long)(j0 + e / EXC - 1) * bc.nx + i0 + e % EXC - 1;
                #pragma unroll
                for (int k = 0; k < 5; ++k) q[it][k] = u[k * a.plane];
            }
        }
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                const PrimF w = cfl_prim_f32_of(q[it][0], q[it][1], q[it][2], q[it][3], q[it][4]);
                pr[0][e] = w.rho;
                pr[1][e] = w.u;
                pr[2][e] = w.v;
                pr[3][e] = w.T;
                pr[4][e] = w.Y;
            }
        }
    } else {
        // boundary tile: the sources of all the thread's cells (tile and ring, ghost cells
        // mapped) first, then all their loads, so that one round trip serves them all
        constexpr int NT = BX * BY, IT = (NEC + NT - 1) / NT;
        CellSrc cs[IT];
        float q[IT][5];
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            cs[it] = CellSrc{0, false, false};
            if (e < NEC) cs[it] = map_cell(min(i0 + e % EXC - 1, bc.nx), min(j0 + e / EXC - 1, bc.nr), bc);
        }
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                #pragma unroll
                for (int k = 0; k < 5; ++k) q[it][k] = fetch(a.U, a.plane, bc, cs[it].code, k);
            }
        }
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                const PrimF w = cfl_prim_f32_of(q[it][0], cs[it].fu ? -q[it][1] : q[it][1],
                                                cs[it].fv ? -q[it][2] : q[it][2], q[it][3], q[it][4]);
                pr[0][e] = w.rho;
                pr[1][e] = w.u;
                pr[2][e] = w.v;
                pr[3][e] = w.T;
                pr[4][e] = w.Y;
            }
        }
    }
    __syncthreads();
    double best = __builtin_huge_val();
    const int tx = threadIdx.x % BX;
    #pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ty = threadIdx.x / BX + r * BY;
        const int i = i0 + tx, j = j0 + ty;
        if (i < bc.nx && j < bc.nr) {
            const int l = (ty + 1) * EXC + tx + 1;
            const PrimF w{pr[0][l], pr[1][l], pr[2][l], pr[3][l], pr[4][l]};
            const double d =
                (double)cfl_limit_f32(a, i, j, w, pr[1][l + EXC], pr[1][l - EXC], pr[2][l + 1], pr[2][l - 1]);
            if (d < best) best = d;
        }
    }
    cfl_block_min(best, a.acc, a.block_min);
}

template <int BX, int BY, int RPT> __global__ void __launch_bounds__(BX *BY) k_cfl_tile_f32(CflArgs<float> a)
{
    cfl_tile_f32_body<BX, BY, RPT>(a, blockIdx.x, blockIdx.y);
}

// Tiled form: the primitives of a BX x (BY * RPT) tile and its 1-cell ring are
// computed once into LDS and shared by the neighbouring cells' limits (the same
// arithmetic for interior and boundary tiles, so the minimum does not depend on how
// the mesh is cut into tiles); interior tiles load their cells directly.
template <class R, int BX, int BY, int RPT>
__device__ __forceinline__ void cfl_tile_body(const CflArgs<R> &a, int bxi, int byi)
{
    constexpr int TY = BY * RPT, EXC = BX + 2, NEC = EXC * (TY + 2);
    __shared__ double pr[5][NEC];
    const BcInfo &bc = a.bc;
    const int i0 = bxi * BX, j0 = byi * TY;
    const bool inner = i0 >= 1 && j0 >= 1 && i0 + BX + 1 <= bc.nx && j0 + TY + 1 <= bc.nr;
    if (inner) {
        // every load of the thread's ring cells in flight before the first use
        constexpr int NT = BX * BY, IT = (NEC + NT - 1) / NT;
        R q[IT][5];
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                const R *u = a.U + (long)(j0 + e / EXC - 1) * bc.nx + i0 + e % EXC - 1;
                #pragma unroll
                for (int k = 0; k < 5; ++k) q[it][k] = u[k * a.plane];
            }
        }
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                const PrimD w = cfl_prim_of((double)q[it][0], (double)q[it][1], (double)q[it][2], (double)q[it][3],
                                            (double)q[it][4]);
                pr[0][e] = w.rho;
                pr[1][e] = w.u;
                pr[2][e] = w.v;
                pr[3][e] = w.T;
                pr[4][e] = w.Y;
            }
        }
    } else {
        // boundary tile: the sources of all the thread's cells (tile and ring, ghost cells
        // mapped) first, then all their loads, so that one round trip serves them all
        constexpr int NT = BX * BY, IT = (NEC + NT - 1) / NT;
        CellSrc cs[IT];
        R q[IT][5];
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            cs[it] = CellSrc{0, false, false};
            if (e < NEC) cs[it] = map_cell(min(i0 + e % EXC - 1, bc.nx), min(j0 + e / EXC - 1, bc.nr), bc);
        }
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                #pragma unroll
                for (int k = 0; k < 5; ++k) q[it][k] = fetch(a.U, a.plane, bc, cs[it].code, k);
            }
        }
        #pragma unroll
        for (int it = 0; it < IT; ++it) {
            const int e = threadIdx.x + it * NT;
            if (e < NEC) {
                double U1 = (double)q[it][1], U2 = (double)q[it][2];
                if (cs[it].fu) U1 = -U1;
                if (cs[it].fv) U2 = -U2;
                const PrimD w = cfl_prim_of((double)q[it][0], U1, U2, (double)q[it][3], (double)q[it][4]);
                pr[0][e] = w.rho;
                pr[1][e] = w.u;
                pr[2][e] = w.v;
                pr[3][e] = w.T;
                pr[4][e] = w.Y;
            }
        }
    }
    __syncthreads();
    double best = __builtin_huge_val();
    const int tx = threadIdx.x % BX;
    #pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int ty = threadIdx.x / BX + r * BY;
        const int i = i0 + tx, j = j0 + ty;
        if (i < bc.nx && j < bc.nr) {
            const int l = (ty + 1) * EXC + tx + 1;
            const PrimD w{pr[0][l], pr[1][l], pr[2][l], pr[3][l], pr[4][l]};
            const double d = cfl_limit(a, i, j, w, pr[1][l + EXC], pr[1][l - EXC], pr[2][l + 1], pr[2][l - 1]);
            if (d < best) best = d;
        }
    }
    cfl_block_min(best, a.acc, a.block_min);
}

template <class R, int BX, int BY, int RPT> __global__ void __launch_bounds__(BX *BY) k_cfl_tile(CflArgs<R> a)
{
    cfl_tile_body<R, BX, BY, RPT>(a, blockIdx.x, blockIdx.y);
}

// batched: blockIdx.y selects the plume, blockIdx.x one of its tiles (row by row);
// each plume reduces into its own slot
template <class R, int BX, int BY, int RPT> __global__ void __launch_bounds__(BX *BY) k_cfl_batch(const CflArgs<R> *args)
{
    const CflArgs<R> &a = args[blockIdx.y];
    constexpr int TY = BY * RPT;
    const int gx = (a.bc.nx + BX - 1) / BX, gy = (a.bc.nr + TY - 1) / TY;
    const int t = blockIdx.x;
    if (t >= gx * gy) return;   // past this plume's tiles (the whole workgroup)
    if constexpr (sizeof(R) == 4)
        cfl_tile_f32_body<BX, BY, RPT>(a, t % gx, t / gx);
    else
        cfl_tile_body<R, BX, BY, RPT>(a, t % gx, t / gx);
}

__global__ void k_cfl_finalize_batch(unsigned long long *acc, const double *cfl, double *dt, double *t, int n)
{
#pragma clang fp contract(off)
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double d = cfl[p] * __longlong_as_double((long long)acc[p]);
    dt[p] = d;
    t[p] = t[p] + d;
    acc[p] = 0x7FF0000000000000ull;
}

// dt = cfl * (minimum of the per-workgroup minima), one workgroup.
__global__ void __launch_bounds__(256) k_cfl_finalize_blocks(const double *bm, int n, double cfl, double *dt, double *t)
{
#pragma clang fp contract(off)
    // eight loads per thread in flight at once (the minimum does not depend on the order)
    double m = __builtin_huge_val();
    for (int k0 = threadIdx.x; k0 < n; k0 += 8 * blockDim.x) {
        double v[8];
        #pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + u * (int)blockDim.x;
            v[u] = k < n ? bm[k] : __builtin_huge_val();
        }
        #pragma unroll
        for (int u = 0; u < 8; ++u) m = fmin(m, v[u]);
    }
    for (int o = 32; o > 0; o >>= 1) m = fmin(m, __shfl_xor(m, o, 64));
    __shared__ double part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = fmin(fmin(part[0], part[1]), fmin(part[2], part[3]));
        const double d = cfl * m;
        *dt = d;
        if (t) *t = *t + d;
    }
}

__global__ void k_acc_reset(unsigned long long *acc) { *acc = 0x7FF0000000000000ull; }

// ------------------------------------------------------------------ source
template <class R, int NV = NVAR>
__global__ void __launch_bounds__(256) k_source(const R *U, R *Q, long n, long plane, double dt, SourceParams sp,
                                                unsigned long long *nsub)
{
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    int ns = 0;
    if (c < n) {
        double Ud[NV], Qd[NV];
        #pragma unroll
        for (int v = 0; v < NV; ++v) Ud[v] = (double)U[v * plane + c];
        ns = source_integrate_nv<NV>(Ud, dt, sp, Qd);
        #pragma unroll
        for (int v = 0; v < NV; ++v) Q[v * plane + c] = (R)Qd[v];
    }
    for (int o = 32; o > 0; o >>= 1) ns += __shfl_xor(ns, o, 64);
    if ((threadIdx.x & 63) == 0 && ns) atomicAdd(nsub, (unsigned long long)ns);
}

// ------------------------------------------------------------------ init
template <class R>
__global__ void __launch_bounds__(256) k_init(R *U, const double *inflow, int nx, int nr, int nv)
{
    const long n = (long)nx * nr;
    const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int j = (int)(c / nx);
    #pragma unroll
    for (int v = 0; v < NVAR; ++v) U[v * n + c] = (R)inflow[j * NVAR + v];
    for (int v = NVAR; v < nv; ++v) U[v * n + c] = R(0);   // no homogeneous droplets yet
}

// ------------------------------------------------------------------ diagnostics
template <class R>
__global__ void __launch_bounds__(256) k_diag(const R *U, long plane, int nx, int nr, const double *vol, double *out,
                                              int nv)
{
    const long n = (long)nx * nr;
    double w = 0.0, ice = 0.0, gas = 0.0, act = 0.0, lnS = -__builtin_huge_val();
    for (long c = (long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long)gridDim.x * blockDim.x) {
        double Ud[NVAR_BI];
        #pragma unroll
        for (int v = 0; v < NVAR_BI; ++v) Ud[v] = v < nv ? (double)U[v * plane + c] : 0.0;
        const double V = vol[c];
        w += V * (Ud[4] + kFourThirdsPi * (kRhoL * (Ud[8] + Ud[18]) + kRhoS * Ud[12]));
        ice += V * Ud[9];
        gas += V * Ud[0];
        CellThermo th;
        cell_thermo(Ud, th);
        double pv = fmax(Ud[4] * kRv * th.T, kPvFloor);
        lnS = fmax(lnS, log(pv) - ln_psat(kSonW, th.T));
        act += source_inactive<NVAR_BI>(Ud, th.T) ? 0.0 : 1.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        w += __shfl_xor(w, o, 64);
        ice += __shfl_xor(ice, o, 64);
        gas += __shfl_xor(gas, o, 64);
        act += __shfl_xor(act, o, 64);
        lnS = fmax(lnS, __shfl_xor(lnS, o, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(out + 0, w);
        atomicAdd(out + 2, ice);
        atomicAdd(out + 3, gas);
        atomicAdd(out + 4, act);
        // max of ln S through an order-preserving integer map of the double
        long long b = __double_as_longlong(lnS);
        unsigned long long key = b >= 0 ? ((unsigned long long)b | 0x8000000000000000ull) : ~(unsigned long long)b;
        atomicMax((unsigned long long *)(out + 1), key);
    }
}

// ------------------------------------------------------------------ launchers
static const std::vector<std::pair<int, int>> kTiles = {{32, 8}, {16, 16}, {64, 4}, {32, 4}, {16, 8}, {32, 16}, {64, 8}};

const std::vector<std::pair<int, int>> &tile_list() { return kTiles; }

bool tile_supported(int tx, int ty)
{
    for (auto &p : kTiles)
        if (p.first == tx && p.second == ty) return true;
    return false;
}

template <class R, int TX, int TY, bool DUCT = false, int NV = NVAR>
static hipError_t stage_launch(const StageArgs<R> &a, hipStream_t s)
{
    dim3 grid((a.bc.nx + TX - 1) / TX, (a.bc.nr + TY - 1) / TY);
    hipLaunchKernelGGL((k_stage<R, TX, TY, DUCT, NV>), grid, dim3(TX * TY), 0, s, a);
    return hipGetLastError();
}

// The duct (one row) always takes its own 64 x 4 instantiation; two liquid
// populations (nv = NVAR_BI) the 32 x 8 one.
template <class R> hipError_t launch_stage(const StageArgs<R> &a, int tx, int ty, int nv, hipStream_t s)
{
    if (nv == NVAR_BI) {
        if (a.bc.geom == kGeomQuasi1D || tx != 32 || ty != 8) return hipErrorInvalidValue;
        return stage_launch<R, 32, 8, false, NVAR_BI>(a, s);
    }
    if (nv != NVAR) return hipErrorInvalidValue;
    if (a.bc.geom == kGeomQuasi1D) return stage_launch<R, 64, 4, true>(a, s);
    if (tx == 32 && ty == 8) return stage_launch<R, 32, 8>(a, s);
    if (tx == 16 && ty == 16) return stage_launch<R, 16, 16>(a, s);
    if (tx == 64 && ty == 4) return stage_launch<R, 64, 4>(a, s);
    if (tx == 32 && ty == 4) return stage_launch<R, 32, 4>(a, s);
    if (tx == 16 && ty == 8) return stage_launch<R, 16, 8>(a, s);
    if (tx == 32 && ty == 16) return stage_launch<R, 32, 16>(a, s);
    if (tx == 64 && ty == 8) return stage_launch<R, 64, 8>(a, s);
    return hipErrorInvalidValue;
}

template <class R, int TX, int TY>
static hipError_t stage_batch_launch(const StageArgs<R> *args, const int *wp, const int *wt, int nwork, hipStream_t s)
{
    hipLaunchKernelGGL((k_stage_batch<R, TX, TY>), dim3(nwork), dim3(TX * TY), 0, s, args, wp, wt, nwork);
    return hipGetLastError();
}

template <class R>
hipError_t launch_stage_batch(const StageArgs<R> *args, const int *wp, const int *wt, int nwork, int tx, int ty,
                              hipStream_t s)
{
    if (tx == 32 && ty == 8) return stage_batch_launch<R, 32, 8>(args, wp, wt, nwork, s);
    if (tx == 16 && ty == 16) return stage_batch_launch<R, 16, 16>(args, wp, wt, nwork, s);
    if (tx == 64 && ty == 4) return stage_batch_launch<R, 64, 4>(args, wp, wt, nwork, s);
    if (tx == 32 && ty == 4) return stage_batch_launch<R, 32, 4>(args, wp, wt, nwork, s);
    if (tx == 16 && ty == 8) return stage_batch_launch<R, 16, 8>(args, wp, wt, nwork, s);
    if (tx == 32 && ty == 16) return stage_batch_launch<R, 32, 16>(args, wp, wt, nwork, s);
    if (tx == 64 && ty == 8) return stage_batch_launch<R, 64, 8>(args, wp, wt, nwork, s);
    return hipErrorInvalidValue;
}

template <class R>
hipError_t launch_source_fix_batch(const SourceFixArgs<R> *args, int nplumes, long max_cells, hipStream_t s)
{
    // up to 64 one-wavefront workgroups per plume, striding over its list
    int bx = (int)std::max<long>(1, std::min<long>((max_cells + 63) / 64, 64));
    hipLaunchKernelGGL((k_source_fix_batch<R>), dim3(bx, nplumes), dim3(64), 0, s, args);
    return hipGetLastError();
}

int cfl_batch_tiles(int nx, int nr)
{
    return ((nx + kCflBX - 1) / kCflBX) * ((nr + kCflBY * kCflRows - 1) / (kCflBY * kCflRows));
}

template <class R> hipError_t launch_cfl_batch(const CflArgs<R> *args, int nplumes, int max_tiles, hipStream_t s)
{
    constexpr int BX = kCflBX, BY = kCflBY, RPT = kCflRows;
    hipLaunchKernelGGL((k_cfl_batch<R, BX, BY, RPT>), dim3(std::max(1, max_tiles), nplumes), dim3(BX * BY), 0, s, args);
    return hipGetLastError();
}

hipError_t launch_cfl_finalize_batch(unsigned long long *acc, const double *cfl, double *dt, double *t, int n,
                                     hipStream_t s)
{
    hipLaunchKernelGGL(k_cfl_finalize_batch, dim3((n + 63) / 64), dim3(64), 0, s, acc, cfl, dt, t, n);
    return hipGetLastError();
}

template <class R> hipError_t launch_drift(const DriftArgs<R> &a, hipStream_t s)
{
    dim3 grid((a.bc.nx + 63) / 64, (a.bc.nr + 3) / 4);
    hipLaunchKernelGGL((k_drift<R>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <class R> hipError_t launch_source_fix(const SourceFixArgs<R> &a, long max_cells, int nv, hipStream_t s)
{
    // enough one-wavefront workgroups for every CU; the list length is only known
    // on the device, so the workgroups stride over it
    int blocks = (int)std::max<long>(1, std::min<long>((max_cells + 63) / 64, 512));
    if (nv == NVAR_BI)
        hipLaunchKernelGGL((k_source_fix<R, NVAR_BI>), dim3(blocks), dim3(64), 0, s, a);
    else if (nv == NVAR)
        hipLaunchKernelGGL((k_source_fix<R>), dim3(blocks), dim3(64), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class R>
hipError_t launch_sur_gate_net(const SurArgs<R> &a, const FusedNet &w, float *Y, long max_cells, hipStream_t s)
{
    // the workgroups the device holds at once, striding over the list
    static const int resident = [] {
        int dev = 0, cus = 256, per_cu = 2;
        if (hipGetDevice(&dev) == hipSuccess) {
            if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 256;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sur_gate_net<R>, 256, 0) != hipSuccess)
                per_cu = 2;
        }
        return std::max(1, cus) * std::max(1, per_cu);
    }();
    const int blocks = (int)std::max<long>(1, std::min<long>((max_cells + 63) / 64, resident));
    hipLaunchKernelGGL((k_sur_gate_net<R>), dim3(blocks), dim3(256), 0, s, a, w, Y);
    return hipGetLastError();
}

template <class R>
hipError_t launch_sur_finish(const SurArgs<R> &a, const SourceParams &sp, int *next_count, unsigned long long *nsub,
                             long max_cells, hipStream_t s)
{
    int blocks = (int)std::max<long>(1, std::min<long>((max_cells + 63) / 64, 512));
    hipLaunchKernelGGL((k_sur_finish<R>), dim3(blocks), dim3(64), 0, s, a, sp, next_count, nsub);
    return hipGetLastError();
}

template <class R> hipError_t launch_sur_features(const R *U, long plane, double dt, const SurNorm &nm, float *F,
                                                  hipStream_t s)
{
    int blocks = (int)std::max<long>(1, std::min<long>((plane + 255) / 256, 4096));
    hipLaunchKernelGGL((k_sur_features<R>), dim3(blocks), dim3(256), 0, s, U, plane, dt, nm, F);
    return hipGetLastError();
}

template <class R> hipError_t launch_active_list(const R *U, long plane, int *count, int *list, hipStream_t s)
{
    int blocks = (int)std::max<long>(1, std::min<long>((plane + 255) / 256, 4096));
    hipLaunchKernelGGL((k_active_list<R>), dim3(blocks), dim3(256), 0, s, U, plane, count, list);
    return hipGetLastError();
}

template <class R>
hipError_t launch_particle_times(const R *U, long plane, int nx, const double *inv_dx, double *tau, double *St,
                                 hipStream_t s)
{
    const int blocks = (int)std::max<long>(1, std::min<long>((plane + 255) / 256, 4096));
    hipLaunchKernelGGL((k_particle_times<R>), dim3(blocks), dim3(256), 0, s, U, plane, nx, inv_dx, tau, St);
    return hipGetLastError();
}

template <class R>
hipError_t launch_tile_mask(const R *U, long plane, int nx, int nr, int nv, int tx, int ty, unsigned *mask,
                            unsigned *unknown_a, unsigned *unknown_b, hipStream_t s)
{
    const int tiles = ((nx + tx - 1) / tx) * ((nr + ty - 1) / ty);
    hipLaunchKernelGGL((k_tile_mask<R>), dim3(tiles), dim3(256), 0, s, U, plane, nx, nr, nv, tx, ty, mask, unknown_a,
                       unknown_b);
    return hipGetLastError();
}

hipError_t launch_sur_reset(int *cnt, unsigned long long *tot, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_reset, dim3(1), dim3(1), 0, s, cnt, tot);
    return hipGetLastError();
}

template <class R> hipError_t launch_cfl(const CflArgs<R> &a, hipStream_t s)
{
    constexpr int BX = kCflBX, BY = kCflBY, RPT = kCflRows;
    dim3 grid((a.bc.nx + BX - 1) / BX, (a.bc.nr + BY * RPT - 1) / (BY * RPT));
    if constexpr (sizeof(R) == 4)
        hipLaunchKernelGGL((k_cfl_tile_f32<BX, BY, RPT>), grid, dim3(BX * BY), 0, s, a);
    else
        hipLaunchKernelGGL((k_cfl_tile<R, BX, BY, RPT>), grid, dim3(BX * BY), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_cfl_finalize_blocks(const double *block_min, int n, double cfl, double *dt, double *t, hipStream_t s)
{
    hipLaunchKernelGGL(k_cfl_finalize_blocks, dim3(1), dim3(256), 0, s, block_min, n, cfl, dt, t);
    return hipGetLastError();
}

hipError_t launch_acc_reset(unsigned long long *acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_acc_reset, dim3(1), dim3(1), 0, s, acc);
    return hipGetLastError();
}

template <class R>
hipError_t launch_source(const R *U, R *Q, long n, long plane, double dt, const SourceParams &sp,
                         unsigned long long *nsub, int nv, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 255) / 256));
    if (nv == NVAR_BI)
        hipLaunchKernelGGL((k_source<R, NVAR_BI>), grid, dim3(256), 0, s, U, Q, n, plane, dt, sp, nsub);
    else if (nv == NVAR)
        hipLaunchKernelGGL((k_source<R>), grid, dim3(256), 0, s, U, Q, n, plane, dt, sp, nsub);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <class R> hipError_t launch_init(R *U, const double *inflow, int nx, int nr, int nv, hipStream_t s)
{
    const long n = (long)nx * nr;
    if (nv != NVAR && nv != NVAR_BI) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_init<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, U, inflow, nx, nr, nv);
    return hipGetLastError();
}

template <class R>
hipError_t launch_diag(const R *U, long plane, int nx, int nr, const double *vol, double *out, int nv, hipStream_t s)
{
    const long n = (long)nx * nr;
    if (nv != NVAR && nv != NVAR_BI) return hipErrorInvalidValue;
    int blocks = (int)std::min<long>((n + 255) / 256, 2048);
    hipLaunchKernelGGL((k_diag<R>), dim3(blocks), dim3(256), 0, s, U, plane, nx, nr, vol, out, nv);
    return hipGetLastError();
}

#define CP_INSTANTIATE(R)                                                                                   \
    template hipError_t launch_stage<R>(const StageArgs<R> &, int, int, int, hipStream_t);                   \
    template hipError_t launch_cfl<R>(const CflArgs<R> &, hipStream_t);                                      \
    template hipError_t launch_sur_gate_net<R>(const SurArgs<R> &, const FusedNet &, float *, long, hipStream_t); \
    template hipError_t launch_sur_finish<R>(const SurArgs<R> &, const SourceParams &, int *,                 \
                                             unsigned long long *, long, hipStream_t);                        \
    template hipError_t launch_active_list<R>(const R *, long, int *, int *, hipStream_t);                    \
    template hipError_t launch_tile_mask<R>(const R *, long, int, int, int, int, int, unsigned *, unsigned *,      \
                                            unsigned *, hipStream_t);                                          \
    template hipError_t launch_particle_times<R>(const R *, long, int, const double *, double *, double *,      \
                                                 hipStream_t);                                                 \
    template hipError_t launch_sur_features<R>(const R *, long, double, const SurNorm &, float *, hipStream_t); \
    template hipError_t launch_source_fix<R>(const SourceFixArgs<R> &, long, int, hipStream_t);              \
    template hipError_t launch_drift<R>(const DriftArgs<R> &, hipStream_t);                                  \
    template hipError_t launch_stage_batch<R>(const StageArgs<R> *, const int *, const int *, int, int, int,   \
                                              hipStream_t);                                                   \
    template hipError_t launch_source_fix_batch<R>(const SourceFixArgs<R> *, int, long, hipStream_t);        \
    template hipError_t launch_cfl_batch<R>(const CflArgs<R> *, int, int, hipStream_t);                      \
    template hipError_t launch_source<R>(const R *, R *, long, long, double, const SourceParams &,           \
                                         unsigned long long *, int, hipStream_t);                             \
    template hipError_t launch_init<R>(R *, const double *, int, int, int, hipStream_t);                      \
    template hipError_t launch_diag<R>(const R *, long, int, int, const double *, double *, int, hipStream_t);

CP_INSTANTIATE(double)
CP_INSTANTIATE(float)

}  // namespace cp
