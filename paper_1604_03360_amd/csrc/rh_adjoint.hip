// rh_adjoint.hip -- gfx950 kernels of the adjoint of L and of the SSP-RK3 step.
//
// One adjoint sweep per axis, all reading a per-cell pack of the primitive
// recovery and its derivatives (FP64 arithmetic).  The x sweep stages
// contiguous rows in LDS, differentiates each face once and gathers the face
// partials per cell; it writes the output from the caller's linear combination
// plus its part.  On periodic rows of 32..256 cells it takes whole rows
// (adj_xrow) and also computes and stores the pack; otherwise it takes tiles
// (adj_x) after a separate pack launch (adj_pack).  The y and z sweeps (adj_roll)
// give each lane a segment [k0, k1) of one grid line; the lane rolls along it
// over every face whose stencil reaches an owned position (the segment plus R
// faces on each side), keeping a register window of 2R cells of split fluxes
// and of split-flux adjoints; for each face it adds the face weight
// g = (w_{i+1} - w_i)/h times the WENO gradients to the window, and a position
// leaving the window is complete and, if the lane owns it, is mapped through
// the flux Jacobian and added to the adjoint field.  Every cell (and every
// ghost position that copies it under outflow boundaries) is owned by exactly
// one lane per sweep, so the read-modify-write needs no atomics.
#include "rh_internal.hpp"
#include "rh_adjoint.hpp"
#include "../../include/rh.h"

namespace rh {

namespace {

// A field's base pointer made opaque once per lane-line: loads through it then
// keep the scalar-base + 32-bit-offset form instead of being re-associated by
// the compiler into per-lane 64-bit address arithmetic (one 64-bit add per
// access).
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> opaque_base(T* p) {
    gptr<T> g = (gptr<T>)p;
    asm("" : "+s"(g));
    return g;
}
template <class T>
__device__ __forceinline__ T ld_off(gptr<const T> base, uint32_t off) {
    return *(gptr<const T>)((gptr<const char>)base + off);
}
template <class T>
__device__ __forceinline__ void st_off(gptr<T> base, uint32_t off, T v) {
    *(gptr<T>)((gptr<char>)base + off) = v;
}

template <class T, int DIR>
struct Column {
    gptr<const T> u[5];    // field base pointers (uniform)
    gptr<const T> w[5];
    gptr<const T> pk[6];
    gptr<T> ub[5];
    // lane -> line: plane axes are (y, z) for DIR 0, (x, z) for DIR 1, (x, y) for DIR 2;
    // byte offsets of the line's first cell and between consecutive cells
    uint32_t cb;
    uint32_t sb;
    int ia, ib;   // the two transverse indices
};

template <class T, int DIR>
__device__ __forceinline__ bool column_of(const AdjArgs<T>& A, unsigned p, Column<T, DIR>& C) {
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        C.u[f] = opaque_base(A.u + f * A.fstride);
        C.w[f] = opaque_base(A.w + f * A.fstride);
        C.ub[f] = opaque_base(A.ub + f * A.fstride);
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) C.pk[f] = opaque_base(A.pk + f * A.fstride);
    if (DIR == 0) {
        const int y = (int)(p % (unsigned)ny), z = (int)(p / (unsigned)ny);
        if (z >= nz) return false;
        C.ia = y;
        C.ib = z;
        C.cb = (uint32_t)sizeof(T) * ((uint32_t)nx * ((uint32_t)y + (uint32_t)ny * (uint32_t)z));
        C.sb = (uint32_t)sizeof(T);
    } else if (DIR == 1) {
        const int x = (int)(p % (unsigned)nx), z = (int)(p / (unsigned)nx);
        if (z >= nz) return false;
        C.ia = x;
        C.ib = z;
        C.cb = (uint32_t)sizeof(T) * ((uint32_t)x + (uint32_t)nx * (uint32_t)ny * (uint32_t)z);
        C.sb = (uint32_t)sizeof(T) * (uint32_t)nx;
    } else {
        const int x = (int)(p % (unsigned)nx), y = (int)(p / (unsigned)nx);
        if (y >= ny) return false;
        C.ia = x;
        C.ib = y;
        C.cb = (uint32_t)sizeof(T) * ((uint32_t)x + (uint32_t)nx * (uint32_t)y);
        C.sb = (uint32_t)sizeof(T) * ((uint32_t)nx * (uint32_t)ny);
    }
    return true;
}

template <class T, int DIR>
__device__ __forceinline__ void cell_xyz(const Column<T, DIR>& C, int m, int c[3]) {
    if (DIR == 0) { c[0] = m; c[1] = C.ia; c[2] = C.ib; }
    else if (DIR == 1) { c[0] = C.ia; c[1] = m; c[2] = C.ib; }
    else { c[0] = C.ia; c[1] = C.ib; c[2] = m; }
}

// state at line position m (ghosts by the boundary condition of the axis)
template <class T, int DIR>
__device__ __forceinline__ void adj_load(const AdjArgs<T>& A, const Column<T, DIR>& C, int m, T u[5]) {
    const int nd = A.n[DIR];
    int mm = m;
    if (m < 0 || m >= nd) {
        if (A.bc == RH_BC_PERIODIC) {
            mm = m % nd;
            if (mm < 0) mm += nd;
        } else if (A.bc == RH_BC_OUTFLOW) {
            mm = m < 0 ? 0 : nd - 1;
        } else {
            int c[3];
            cell_xyz(C, m, c);
            double uh[5];
            hubble_conserved(A.hb, A.hb.c0[0] + c[0] * A.hb.h[0], A.hb.c0[1] + c[1] * A.hb.h[1],
                             A.hb.c0[2] + c[2] * A.hb.h[2], uh);
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = (T)uh[f];
            return;
        }
    }
    const uint32_t off = C.cb + (uint32_t)mm * C.sb;
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = ld_off(C.u[f], off);
}

// State at line position m with its velocity along the sweep axis and pressure,
// taken from the recovery pack (interior, periodic and outflow positions) or,
// for analytic ghosts, evaluated and recovered here in FP64.  HUB = false
// compiles the analytic branch out (its FP64 registers would otherwise count
// against the whole rolling window).
template <class T, int DIR, bool HUB>
__device__ __forceinline__ void adj_state(const AdjArgs<T>& A, const Column<T, DIR>& C, int m, T u[5], T& v,
                                          T& P) {
    const int nd = A.n[DIR];
    int mm = m;
    if (m < 0 || m >= nd) {
        if (A.bc == RH_BC_PERIODIC) {
            mm = m % nd;
            if (mm < 0) mm += nd;
        } else if (!HUB || A.bc == RH_BC_OUTFLOW) {
            mm = m < 0 ? 0 : nd - 1;
        } else {
            adj_load<T, DIR>(A, C, m, u);
            double vd, pd;
            unsigned dummy = 0;
            recover_vp<DIR>((double)u[0], (double)u[1], (double)u[2], (double)u[3], vd, pd, dummy);
            v = (T)vd;
            P = (T)pd;
            return;
        }
    }
    const uint32_t off = C.cb + (uint32_t)mm * C.sb;
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = ld_off(C.u[f], off);
    v = ld_off(C.pk[0], off) * u[1 + DIR];
    P = ld_off(C.pk[1], off);
}

// weights at line position m: zero outside the grid unless periodic
template <class T, int DIR>
__device__ __forceinline__ void adj_weight(const AdjArgs<T>& A, const Column<T, DIR>& C, int m, T w[5]) {
    const int nd = A.n[DIR];
    int mm = m;
    if (m < 0 || m >= nd) {
        if (A.bc != RH_BC_PERIODIC) {
#pragma unroll
            for (int f = 0; f < 5; ++f) w[f] = (T)0;
            return;
        }
        mm = m % nd;
        if (mm < 0) mm += nd;
    }
    const uint32_t off = C.cb + (uint32_t)mm * C.sb;
#pragma unroll
    for (int f = 0; f < 5; ++f) w[f] = ld_off(C.w[f], off);
}

}  // namespace

// The WENO reconstruction is component-wise, so the face gradients of each
// conserved component need only that component's window; the components are
// therefore processed in groups, one pass per group over the lane's segment,
// each pass carrying only its group's window (which keeps the register file
// small enough for several waves per SIMD).  A pass adds its group's part of
// (d f+/du)^T a+ + (d f-/du)^T a- to every field of the owned cells.
//
// Components per pass: FP32 WENO5 3 (passes {0,1,2}, {3,4}); otherwise 2.
template <class T, int ORDER>
struct AdjGroup {
    static constexpr int value = (sizeof(T) == 4 && ORDER == 5) ? 3 : 2;
};

template <class T, int ORDER, int DIR, int CLO, int CHI, bool HUB>
__device__ __forceinline__ void adj_pass(const AdjArgs<T>& A, const Column<T, DIR>& C, int k0, int k1) {
    constexpr int R = (ORDER + 1) / 2, W = 2 * R, NC = CHI - CLO;
    // WENO5 gradient in the first differences (fewer instructions, more live
    // values) except where the analytic-ghost branch leaves too few registers
    // for it at three FP32 waves per SIMD
    constexpr bool EFORM = !(sizeof(T) == 4 && HUB);
    const int nd = A.n[DIR];
    const bool periodic = A.bc == RH_BC_PERIODIC;
    int i_lo = k0 - R, i_hi = k1 + R - 2;
    if (!periodic) {
        i_lo = max(i_lo, -1);
        i_hi = min(i_hi, nd - 1);
    }
    // owned positions [own_lo, own_hi): outflow edges also own the ghost positions
    const int own_lo = (!periodic && k0 == 0 && A.bc == RH_BC_OUTFLOW) ? -(1 << 30) : k0;
    const int own_hi = (!periodic && k1 == nd && A.bc == RH_BC_OUTFLOW) ? (1 << 30) : k1;
    const T eps = A.eps;
    const T half = (T)0.5;
    // adjoint fields this group changes: its own components, and with any
    // momentum or charge component the energy and the momenta (through the
    // velocity and pressure); the others are neither loaded nor stored
    auto touched = [](int f) {
        return (f >= CLO && f < CHI) || (CHI > 1 && f < 4) || (CLO == 0 && f == 1 + DIR);
    };

    // doubled split fluxes F +- u of the group's components from a cell state:
    // the reconstruction is homogeneous of degree one in (f, sqrt(eps)), so its
    // gradient at (2 f, 4 eps) equals the gradient at (f, eps), bit for bit
    // (all scalings are powers of two); the 1/2 of the split stays in finish
    auto group_flux = [&](const T u[5], T v, T P, T fp[NC], T fm[NC]) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int c = CLO + q;
            T f;
            if (c == 0) f = u[1 + DIR];
            else if (c == 4) f = u[4] * v;
            else f = u[c] * v + (c == 1 + DIR ? P : (T)0);
            fp[q] = f + u[c];
            fm[q] = f - u[c];
        }
    };
    // Owned position pos -> the cell whose adjoint it updates (outflow ghost
    // positions fold onto the edge cell; analytic ghosts are constants).
    auto target = [&](int pos, int& tgt) -> bool {
        if (pos < own_lo || pos >= own_hi) return false;
        tgt = pos;
        if (pos < 0 || pos >= nd) {
            if (A.bc != RH_BC_OUTFLOW) return false;
            tgt = pos < 0 ? 0 : nd - 1;
        }
        return true;
    };
    // state and running adjoint of the cell updated next; consecutive updates
    // of one cell (outflow edges) continue from registers
    int last_tgt = -1;
    T ubo[5], uf[5], pkf[5];
    auto fetch_cell = [&](int tgt) {
        const uint32_t off = C.cb + (uint32_t)tgt * C.sb;
#pragma unroll
        for (int f = 0; f < 5; ++f) uf[f] = ld_off(C.u[f], off);
        if constexpr (CHI > 1) {
            pkf[0] = ld_off(C.pk[0], off);
#pragma unroll
            for (int q = 1; q < 5; ++q) pkf[q] = ld_off(C.pk[q + 1], off);
        }
        if (tgt == last_tgt) return;
#pragma unroll
        for (int f = 0; f < 5; ++f)
            if (touched(f)) ubo[f] = ld_off(C.ub[f], off);
    };
    // ub += scale * sum over the group of (d f+_c/du)^T a+_c + (d f-_c/du)^T a-_c
    auto finish = [&](int tgt, const T apj[NC], const T amj[NC]) {
        // pkf = (kappa, dkappa/dE, dkappa/dM2, dP/dE, dP/dM2); v_d = kappa M_d
        T lam[5] = {(T)0, (T)0, (T)0, (T)0, (T)0}, g[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            lam[CLO + q] = half * (apj[q] + amj[q]);
            g[CLO + q] = half * (apj[q] - amj[q]);
        }
        g[1 + DIR] += lam[0];
        if constexpr (CHI > 1) {
            const T Md = uf[1 + DIR], vd = pkf[0] * Md;
            T S = (T)0;
#pragma unroll
            for (int c = (CLO > 1 ? CLO : 1); c < CHI; ++c) {
                S += lam[c] * uf[c];
                g[c] += lam[c] * vd;
            }
            const T lp = lam[1 + DIR];
            // dv_d/dE = M_d kappa_E, dv_d/dM_m = kappa delta_dm + 2 M_d M_m kappa_M2,
            // dP/dE = P_E, dP/dM_m = 2 M_m P_M2
            g[0] += S * (Md * pkf[1]) + lp * pkf[3];
            const T sk = (T)2 * S * Md * pkf[2], sp = (T)2 * lp * pkf[4];
#pragma unroll
            for (int m = 0; m < 3; ++m) g[1 + m] += (sk + sp) * uf[1 + m];
            g[1 + DIR] += S * pkf[0];
        }
        const uint32_t off = C.cb + (uint32_t)tgt * C.sb;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            if (!touched(f)) continue;
            ubo[f] = ubo[f] + A.scale * g[f];
            st_off(C.ub[f], off, ubo[f]);
        }
        last_tgt = tgt;
    };
    T wp[NC][W], wm[NC][W], ap[NC][W], am[NC][W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T u[5], v, P, fp[NC], fm[NC];
        adj_state<T, DIR, HUB>(A, C, i_lo - R + 1 + j, u, v, P);
        group_flux(u, v, P, fp, fm);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            wp[q][j] = fp[q];
            wm[q][j] = fm[q];
            ap[q][j] = (T)0;
            am[q][j] = (T)0;
        }
    }
    // loads run one face ahead: the weights of the next face's right cell and
    // the state of the next cell to enter the window are in flight while this
    // face is differentiated (positions past the segment stay in bounds)
    T wl[NC], wn[NC], un[5], vn, Pn;
    {
        T w5[5];
        adj_weight<T, DIR>(A, C, i_lo, w5);
#pragma unroll
        for (int q = 0; q < NC; ++q) wl[q] = w5[CLO + q];
        adj_weight<T, DIR>(A, C, i_lo + 1, w5);
#pragma unroll
        for (int q = 0; q < NC; ++q) wn[q] = w5[CLO + q];
    }
    adj_state<T, DIR, HUB>(A, C, i_lo + R + 1, un, vn, Pn);
    // two faces per trip: the second face's window is the first one's renamed,
    // so the register moves of the shift are paid once per two faces
#pragma unroll 2
    for (int i = i_lo; i <= i_hi; ++i) {
        T wr[NC], unew[5];
#pragma unroll
        for (int q = 0; q < NC; ++q) wr[q] = wn[q];
#pragma unroll
        for (int f = 0; f < 5; ++f) unew[f] = un[f];
        const T vnew = vn, Pnew = Pn;
        {
            T w5[5];
            adj_weight<T, DIR>(A, C, i + 2, w5);
#pragma unroll
            for (int q = 0; q < NC; ++q) wn[q] = w5[CLO + q];
        }
        adj_state<T, DIR, HUB>(A, C, i + R + 2, un, vn, Pn);
        int tgt = 0;
        const bool own = target(i - R + 1, tgt);
        if (own) fetch_cell(tgt);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const T g = (wr[q] - wl[q]) * A.inv_h;
            wl[q] = wr[q];
            if constexpr (ORDER == 5) {
                if constexpr (EFORM) {
                    weno5_grad_acc_e<T>(wp[q][0], wp[q][1], wp[q][2], wp[q][3], wp[q][4], (T)16 * eps, g,
                                        ap[q][0], ap[q][1], ap[q][2], ap[q][3], ap[q][4]);
                    weno5_grad_acc_e<T>(wm[q][5], wm[q][4], wm[q][3], wm[q][2], wm[q][1], (T)16 * eps, g,
                                        am[q][5], am[q][4], am[q][3], am[q][2], am[q][1]);
                } else {
                    weno5_grad_acc<T>(wp[q][0], wp[q][1], wp[q][2], wp[q][3], wp[q][4], (T)16 * eps, g,
                                      ap[q][0], ap[q][1], ap[q][2], ap[q][3], ap[q][4]);
                    weno5_grad_acc<T>(wm[q][5], wm[q][4], wm[q][3], wm[q][2], wm[q][1], (T)16 * eps, g,
                                      am[q][5], am[q][4], am[q][3], am[q][2], am[q][1]);
                }
            } else {
                T sv[7], o[7];
#pragma unroll
                for (int j = 0; j < 7; ++j) { sv[j] = wp[q][j]; o[j] = (T)0; }
                weno7_grad_acc<T>(sv, (T)4 * eps, g, o);
#pragma unroll
                for (int j = 0; j < 7; ++j) ap[q][j] += o[j];
#pragma unroll
                for (int j = 0; j < 7; ++j) { sv[j] = wm[q][7 - j]; o[j] = (T)0; }
                weno7_grad_acc<T>(sv, (T)4 * eps, g, o);
#pragma unroll
                for (int j = 0; j < 7; ++j) am[q][7 - j] += o[j];
            }
        }
        if (own) {
            T a0p[NC], a0m[NC];
#pragma unroll
            for (int q = 0; q < NC; ++q) {
                a0p[q] = ap[q][0];
                a0m[q] = am[q][0];
            }
            finish(tgt, a0p, a0m);
        }
        if (i < i_hi) {
            T fp[NC], fm[NC];
            group_flux(unew, vnew, Pnew, fp, fm);
#pragma unroll
            for (int q = 0; q < NC; ++q) {
#pragma unroll
                for (int j = 0; j < W - 1; ++j) {
                    wp[q][j] = wp[q][j + 1];
                    wm[q][j] = wm[q][j + 1];
                    ap[q][j] = ap[q][j + 1];
                    am[q][j] = am[q][j + 1];
                }
                wp[q][W - 1] = fp[q];
                wm[q][W - 1] = fm[q];
                ap[q][W - 1] = (T)0;
                am[q][W - 1] = (T)0;
            }
        }
    }
    // positions still in the window after the last face
#pragma unroll
    for (int j = 1; j < W; ++j) {
        int tgt = 0;
        if (!target(i_hi - R + 1 + j, tgt)) continue;
        fetch_cell(tgt);
        T ajp[NC], ajm[NC];
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            ajp[q] = ap[q][j];
            ajm[q] = am[q][j];
        }
        finish(tgt, ajp, ajm);
    }
}

template <class T, int ORDER, int DIR, int CLO, bool HUB>
__device__ __forceinline__ void adj_passes(const AdjArgs<T>& A, const Column<T, DIR>& C, int k0, int k1) {
    if constexpr (CLO < 5) {
        constexpr int GS = AdjGroup<T, ORDER>::value;
        constexpr int CHI = CLO + GS < 5 ? CLO + GS : 5;
        adj_pass<T, ORDER, DIR, CLO, CHI, HUB>(A, C, k0, k1);
        adj_passes<T, ORDER, DIR, CHI, HUB>(A, C, k0, k1);
    }
}

// Three waves per SIMD for FP32 (the register window fits in 168 VGPRs); FP64
// takes what the window needs.
template <class T>
struct AdjMinBlocks {
    static constexpr int value = sizeof(T) == 4 ? 3 : 1;
};

template <class T, int ORDER, int DIR, bool HUB>
__global__ void __launch_bounds__(256, (AdjMinBlocks<T>::value)) adj_roll(AdjArgs<T> A) {
    Column<T, DIR> C;
    if (!column_of<T, DIR>(A, blockIdx.x * 256u + threadIdx.x, C)) return;
    const int k0 = blockIdx.y * A.seg;
    const int k1 = min(k0 + A.seg, A.n[DIR]);
    adj_passes<T, ORDER, DIR, 0, HUB>(A, C, k0, k1);
}

template <class T>
__global__ void adj_pack(const T* __restrict__ u, T* __restrict__ pk, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const RecoveryPack o = recovery_pack((double)u[i], (double)u[n + i], (double)u[2 * n + i],
                                             (double)u[3 * n + i]);
        pk[i] = (T)o.kap;
        pk[n + i] = (T)o.p;
        pk[2 * n + i] = (T)o.kap_E;
        pk[3 * n + i] = (T)o.kap_M2;
        pk[4 * n + i] = (T)o.p_E;
        pk[5 * n + i] = (T)o.p_M2;
    }
}

// ---------------------------------------------------------------------------
// x axis: x is contiguous, so a block takes a tile of TX cells x TY rows plus
// ghosts in LDS, as the forward x sweep does.  Per component, each lane
// differentiates one face (the tile's faces are spread over the lanes) and
// writes the face's stencil partials to LDS; after a barrier each lane sums
// the partials of the faces that reach its cell in a fixed order.  With all
// five split-flux adjoints of its cell in registers the lane applies the flux
// Jacobian once and writes out = (linear combination of init terms) + scale g.
// Outflow ghost positions fold onto the edge cells (same state, so their
// split-flux adjoints add before the Jacobian); analytic ghosts are constants.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ void x_state(const AdjArgs<T>& A, int gx, int row, T u[5], T& v, T& P) {
    const int nx = A.n[0];
    int mx = gx;
    if (gx < 0 || gx >= nx) {
        if (A.bc == RH_BC_PERIODIC) {
            mx = gx % nx;
            if (mx < 0) mx += nx;
        } else if (A.bc == RH_BC_OUTFLOW) {
            mx = gx < 0 ? 0 : nx - 1;
        } else {
            const int y = row % A.n[1], z = row / A.n[1];
            double uh[5];
            hubble_conserved(A.hb, A.hb.c0[0] + gx * A.hb.h[0], A.hb.c0[1] + y * A.hb.h[1],
                             A.hb.c0[2] + z * A.hb.h[2], uh);
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = (T)uh[f];
            double vd, pd;
            unsigned dummy = 0;
            recover_vp<0>(uh[0], uh[1], uh[2], uh[3], vd, pd, dummy);
            v = (T)vd;
            P = (T)pd;
            return;
        }
    }
    const long long id = mx + (long long)nx * row;
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = A.u[f * A.fstride + id];
    v = A.pk[id] * u[1];
    P = A.pk[A.fstride + id];
}

template <class T, int ORDER, int TX, int TY>
__global__ void __launch_bounds__(256) adj_x(AdjArgs<T> A, Lin3<T> init) {
    constexpr int R = (ORDER + 1) / 2, K = 2 * R - 1;
    constexpr int CPL = TX * TY / 256;   // cells per lane
    constexpr int NF = TX + 2 * R - 1;   // faces x0-R .. x0+TX+R-2 (face i: between cells i and i+1)
    constexpr int NC = TX + 4 * R - 2;   // cells x0-2R+1 .. x0+TX+2R-2
    constexpr int NW = TX + 2 * R;       // weights x0-R .. x0+TX+R-1
    static_assert(TX * TY % 256 == 0, "whole cells per lane");
    __shared__ T sfp[5][TY][NC];
    __shared__ T sfm[5][TY][NC];
    __shared__ T sw[5][TY][NW];
    __shared__ T sp[TY][NF][K];          // plus partials of face fl for cells fl .. fl+K-1 (local)
    __shared__ T sm[TY][NF][K];          // minus partials of face fl for cells fl+1 .. fl+K
    const int nx = A.n[0];
    const int nrows = A.n[1] * A.n[2];
    const int ntx = (nx + TX - 1) / TX;
    const int bx = blockIdx.x % ntx, by = blockIdx.x / ntx;
    const int x0 = bx * TX, r0 = by * TY;
    const int tid = threadIdx.x;
    const bool periodic = A.bc == RH_BC_PERIODIC;
    const T half = (T)0.5;

    for (int idx = tid; idx < TY * NC; idx += 256) {
        const int ly = idx / NC, lx = idx - ly * NC;
        const int row = r0 + ly;
        T fp[5] = {(T)0, (T)0, (T)0, (T)0, (T)0}, fm[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
        if (row < nrows) {
            T u[5], v, P;
            x_state<T>(A, x0 - 2 * R + 1 + lx, row, u, v, P);
            T f[5];
            f[0] = u[1];
            f[1] = u[1] * v + P;
            f[2] = u[2] * v;
            f[3] = u[3] * v;
            f[4] = u[4] * v;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                fp[c] = f[c] + u[c];   // doubled split fluxes (eps scaled by 4 below)
                fm[c] = f[c] - u[c];
            }
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            sfp[c][ly][lx] = fp[c];
            sfm[c][ly][lx] = fm[c];
        }
    }
    for (int idx = tid; idx < TY * NW; idx += 256) {
        const int ly = idx / NW, lx = idx - ly * NW;
        const int row = r0 + ly;
        int gx = x0 - R + lx;
        bool inside = row < nrows;
        if (inside && (gx < 0 || gx >= nx)) {
            if (periodic) {
                gx %= nx;
                if (gx < 0) gx += nx;
            } else {
                inside = false;   // weights vanish outside a non-periodic grid
            }
        }
        const long long id = gx + (long long)nx * row;
#pragma unroll
        for (int c = 0; c < 5; ++c) sw[c][ly][lx] = inside ? A.w[c * A.fstride + id] : (T)0;
    }
    __syncthreads();

    T ap[CPL][5], am[CPL][5];
#pragma unroll 1
    for (int c = 0; c < 5; ++c) {
        for (int f = tid; f < TY * NF; f += 256) {
            const int fy = f / NF, fl = f - fy * NF;
            const int i = x0 - R + fl;
            T op[K], om[K];
#pragma unroll
            for (int k = 0; k < K; ++k) op[k] = om[k] = (T)0;
            if ((periodic || (i >= -1 && i <= nx - 1)) && r0 + fy < nrows) {
                const T g = (sw[c][fy][fl + 1] - sw[c][fy][fl]) * A.inv_h;
                if constexpr (ORDER == 5) {
                    weno5_grad_acc_e<T>(sfp[c][fy][fl], sfp[c][fy][fl + 1], sfp[c][fy][fl + 2], sfp[c][fy][fl + 3],
                                      sfp[c][fy][fl + 4], (T)16 * A.eps, g, op[0], op[1], op[2], op[3], op[4]);
                    weno5_grad_acc_e<T>(sfm[c][fy][fl + 5], sfm[c][fy][fl + 4], sfm[c][fy][fl + 3],
                                      sfm[c][fy][fl + 2], sfm[c][fy][fl + 1], (T)16 * A.eps, g, om[4], om[3],
                                      om[2], om[1], om[0]);
                } else {
                    T sv[7], o[7];
#pragma unroll
                    for (int j = 0; j < 7; ++j) {
                        sv[j] = sfp[c][fy][fl + j];
                        o[j] = (T)0;
                    }
                    weno7_grad_acc<T>(sv, (T)4 * A.eps, g, o);
#pragma unroll
                    for (int j = 0; j < 7; ++j) op[j] = o[j];
#pragma unroll
                    for (int j = 0; j < 7; ++j) {
                        sv[j] = sfm[c][fy][fl + 7 - j];
                        o[j] = (T)0;
                    }
                    weno7_grad_acc<T>(sv, (T)4 * A.eps, g, o);
#pragma unroll
                    for (int j = 0; j < 7; ++j) om[6 - j] = o[j];
                }
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                sp[fy][fl][k] = op[k];
                sm[fy][fl][k] = om[k];
            }
        }
        __syncthreads();
        // partials reaching staged cell q: plus from faces q-k, minus from faces q-1-k
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const int cell = tid + 256 * j, lx = cell % TX, ly = cell / TX;
            const int q = lx + 2 * R - 1;   // every face reaching an owned cell is in the tile
            T a_p = (T)0, a_m = (T)0;
#pragma unroll
            for (int k = 0; k < K; ++k) {
                a_p += sp[ly][q - k][k];
                a_m += sm[ly][q - 1 - k][k];
            }
            const int gx = x0 + lx;
            if (A.bc == RH_BC_OUTFLOW && (gx == 0 || gx == nx - 1) && r0 + ly < nrows) {
                // ghost positions beyond the edge fold onto the edge cell
                for (int e = 1; e < 2 * R; ++e) {
                    const int qe = gx == 0 ? q - e : q + e;
                    for (int k = 0; k < K; ++k) {
                        const int fp_ = qe - k, fm_ = qe - 1 - k;
                        if (fp_ >= 0 && fp_ < NF) a_p += sp[ly][fp_][k];
                        if (fm_ >= 0 && fm_ < NF) a_m += sm[ly][fm_][k];
                    }
                }
            }
            ap[j][c] = a_p;
            am[j][c] = a_m;
        }
        __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int cell = tid + 256 * j, lx = cell % TX, ly = cell / TX;
        const int gx = x0 + lx, row = r0 + ly;
        if (gx >= nx || row >= nrows) continue;
        const long long id = gx + (long long)nx * row;
        T uf[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) uf[f] = A.u[f * A.fstride + id];
        const T kap = A.pk[id], kE = A.pk[2 * A.fstride + id], kM2 = A.pk[3 * A.fstride + id];
        const T pE = A.pk[4 * A.fstride + id], pM2 = A.pk[5 * A.fstride + id];
        T lam[5], g[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            lam[c] = half * (ap[j][c] + am[j][c]);
            g[c] = half * (ap[j][c] - am[j][c]);
        }
        // F = (Mx, Mx v + p, My v, Mz v, N v) with v = kappa Mx
        const T Mx = uf[1], vd = kap * Mx;
        g[1] += lam[0];
        T S = (T)0;
#pragma unroll
        for (int c = 1; c < 5; ++c) {
            S += lam[c] * uf[c];
            g[c] += lam[c] * vd;
        }
        const T lp = lam[1];
        g[0] += S * (Mx * kE) + lp * pE;
        const T sk = (T)2 * S * Mx * kM2, spp = (T)2 * lp * pM2;
#pragma unroll
        for (int m = 0; m < 3; ++m) g[1 + m] += (sk + spp) * uf[1 + m];
        g[1] += S * kap;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const long long o = f * A.fstride + id;
            T acc = (T)0;
            if (init.X1) acc += init.a1 * init.X1[o];
            if (init.X2) acc += init.a2 * init.X2[o];
            if (init.X3) acc += init.a3 * init.X3[o];
            A.ub[o] = acc + A.scale * g[f];
        }
    }
}

// ---------------------------------------------------------------------------
// x axis of a periodic grid whose rows hold NX = 32 .. 256 cells: a block of
// (256 / NX) x NX lanes takes whole rows, one cell per lane.  The lane stages
// its own cell's split fluxes and weight (the periodic ghosts are extra LDS
// copies written by the cells they copy), differentiates the face to its right
// and gathers the partials of the faces that reach its cell.  No lane stages a
// ghost from HBM or differentiates a halo face, which the tiled kernel does for
// 2R - 1 faces per row (a fifth of its face rounds at 64 x 4).  The arithmetic
// and the order of every sum are those of adj_x, so both give the same bits.
// ---------------------------------------------------------------------------
// FP32 WENO5 rows: six waves per SIMD, the most that the LDS of 256-cell row
// blocks allows (62 registers instead of 82; 0.5% faster at 256^3).
template <class T, int ORDER>
struct AdjRowWaves {
    static constexpr int value = (sizeof(T) == 4 && ORDER == 5) ? 6 : 1;
};

template <class T, int ORDER, int NX>
__global__ void __launch_bounds__(256, (AdjRowWaves<T, ORDER>::value)) adj_xrow(AdjArgs<T> A, Lin3<T> init) {
    constexpr int R = (ORDER + 1) / 2, K = 2 * R - 1;
    constexpr int RPB = 256 / NX;        // rows per block
    constexpr int NP = NX + 2 * R - 1;   // padded row: cells -(R-1) .. NX+R-1 at p = cell + R - 1
    static_assert(NX >= 2 * R && RPB >= 1, "row longer than the stencil");
    __shared__ T sfp[5][RPB][NP];
    __shared__ T sfm[5][RPB][NP];
    __shared__ T sw[5][RPB][NX];
    __shared__ T sp[RPB][NX][K];         // plus partials of face x for cells x-R+1 .. x+R-1
    __shared__ T sm[RPB][NX][K];         // minus partials of face x for cells x-R+2 .. x+R
    const int tid = threadIdx.x;
    const int ly = tid / NX, x = tid - ly * NX;
    const long long row = (long long)blockIdx.x * RPB + ly;
    const bool live = row < (long long)A.n[1] * A.n[2];
    const long long id = x + (long long)NX * row;
    const T half = (T)0.5;

    T uf[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
    T kap = (T)0, kE = (T)0, kM2 = (T)0, pE = (T)0, pM2 = (T)0;
    {
        T fp[5] = {(T)0, (T)0, (T)0, (T)0, (T)0}, fm[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
        T w5[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
        if (live) {
#pragma unroll
            for (int f = 0; f < 5; ++f) {
                uf[f] = A.u[f * A.fstride + id];
                w5[f] = A.w[f * A.fstride + id];
            }
            // the recovery pack of the lane's cell (as adj_pack computes it),
            // also stored for the y and z sweeps
            const RecoveryPack o = recovery_pack((double)uf[0], (double)uf[1], (double)uf[2], (double)uf[3]);
            kap = (T)o.kap;
            const T P = (T)o.p;
            kE = (T)o.kap_E;
            kM2 = (T)o.kap_M2;
            pE = (T)o.p_E;
            pM2 = (T)o.p_M2;
            A.pk[id] = kap;
            A.pk[A.fstride + id] = P;
            A.pk[2 * A.fstride + id] = kE;
            A.pk[3 * A.fstride + id] = kM2;
            A.pk[4 * A.fstride + id] = pE;
            A.pk[5 * A.fstride + id] = pM2;
            const T v = kap * uf[1];
            T f[5];
            f[0] = uf[1];
            f[1] = uf[1] * v + P;
            f[2] = uf[2] * v;
            f[3] = uf[3] * v;
            f[4] = uf[4] * v;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                fp[c] = f[c] + uf[c];   // doubled split fluxes (eps scaled by 4 below)
                fm[c] = f[c] - uf[c];
            }
        }
        const int p = x + R - 1;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            sfp[c][ly][p] = fp[c];
            sfm[c][ly][p] = fm[c];
            sw[c][ly][x] = w5[c];
        }
        if (x >= NX - (R - 1)) {   // left ghosts -(R-1) .. -1
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                sfp[c][ly][p - NX] = fp[c];
                sfm[c][ly][p - NX] = fm[c];
            }
        }
        if (x < R) {               // right ghosts NX .. NX+R-1
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                sfp[c][ly][p + NX] = fp[c];
                sfm[c][ly][p + NX] = fm[c];
            }
        }
    }
    __syncthreads();

    const int xr = x + 1 < NX ? x + 1 : 0;
    T ap[5], am[5];
#pragma unroll 1
    for (int c = 0; c < 5; ++c) {
        {
            // face x (between cells x and x+1); its plus stencil starts at p = x
            T op[K], om[K];
#pragma unroll
            for (int k = 0; k < K; ++k) op[k] = om[k] = (T)0;
            const T g = (sw[c][ly][xr] - sw[c][ly][x]) * A.inv_h;
            if constexpr (ORDER == 5) {
                weno5_grad_acc_e<T>(sfp[c][ly][x], sfp[c][ly][x + 1], sfp[c][ly][x + 2], sfp[c][ly][x + 3],
                                    sfp[c][ly][x + 4], (T)16 * A.eps, g, op[0], op[1], op[2], op[3], op[4]);
                weno5_grad_acc_e<T>(sfm[c][ly][x + 5], sfm[c][ly][x + 4], sfm[c][ly][x + 3], sfm[c][ly][x + 2],
                                    sfm[c][ly][x + 1], (T)16 * A.eps, g, om[4], om[3], om[2], om[1], om[0]);
            } else {
                T sv[7], o[7];
#pragma unroll
                for (int j = 0; j < 7; ++j) {
                    sv[j] = sfp[c][ly][x + j];
                    o[j] = (T)0;
                }
                weno7_grad_acc<T>(sv, (T)4 * A.eps, g, o);
#pragma unroll
                for (int j = 0; j < 7; ++j) op[j] = o[j];
#pragma unroll
                for (int j = 0; j < 7; ++j) {
                    sv[j] = sfm[c][ly][x + 7 - j];
                    o[j] = (T)0;
                }
                weno7_grad_acc<T>(sv, (T)4 * A.eps, g, o);
#pragma unroll
                for (int j = 0; j < 7; ++j) om[6 - j] = o[j];
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                sp[ly][x][k] = op[k];
                sm[ly][x][k] = om[k];
            }
        }
        __syncthreads();
        // partials reaching cell x: plus from faces x+R-1-k, minus from faces x+R-2-k
        T a_p = (T)0, a_m = (T)0;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            int fp_ = x + R - 1 - k, fm_ = x + R - 2 - k;
            fp_ = fp_ < 0 ? fp_ + NX : (fp_ >= NX ? fp_ - NX : fp_);
            fm_ = fm_ < 0 ? fm_ + NX : (fm_ >= NX ? fm_ - NX : fm_);
            a_p += sp[ly][fp_][k];
            a_m += sm[ly][fm_][k];
        }
        ap[c] = a_p;
        am[c] = a_m;
        __syncthreads();
    }
    if (!live) return;
    T lam[5], g[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        lam[c] = half * (ap[c] + am[c]);
        g[c] = half * (ap[c] - am[c]);
    }
    // F = (Mx, Mx v + p, My v, Mz v, N v) with v = kappa Mx
    const T Mx = uf[1], vd = kap * Mx;
    g[1] += lam[0];
    T S = (T)0;
#pragma unroll
    for (int c = 1; c < 5; ++c) {
        S += lam[c] * uf[c];
        g[c] += lam[c] * vd;
    }
    const T lp = lam[1];
    g[0] += S * (Mx * kE) + lp * pE;
    const T sk = (T)2 * S * Mx * kM2, spp = (T)2 * lp * pM2;
#pragma unroll
    for (int m = 0; m < 3; ++m) g[1 + m] += (sk + spp) * uf[1 + m];
    g[1] += S * kap;
#pragma unroll
    for (int f = 0; f < 5; ++f) {
        const long long o = f * A.fstride + id;
        T acc = (T)0;
        if (init.X1) acc += init.a1 * init.X1[o];
        if (init.X2) acc += init.a2 * init.X2[o];
        if (init.X3) acc += init.a3 * init.X3[o];
        A.ub[o] = acc + A.scale * g[f];
    }
}

// Tile of the x adjoint: the narrowest of 64, 32, 16 cells that wastes the
// least on a ragged row end (2R - 1 halo faces per row).  A 128 x 4 tile with
// two cells per lane halves the idle lanes of the last face round but needs
// twice the LDS; it measured 24% slower at 256^3 FP32.
int adjoint_tile_x(int nx) {
    int best = 64;
    double best_cost = 1e300;
    for (int tx : {64, 32, 16}) {
        const int ntx = (nx + tx - 1) / tx;
        const double cost = ntx * (tx + 5.0) / nx;
        if (cost < best_cost - 1e-12) {
            best_cost = cost;
            best = tx;
        }
    }
    return best;
}

template <class T>
__global__ void fill_zero(T* p, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = (T)0;
}

// out = a X + b Y + c Z + d V (null operands skipped)
template <class T>
__global__ void lincomb(T* out, long long n, T a, const T* X, T b, const T* Y, T c, const T* Z, T d,
                        const T* V) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        T v = (T)0;
        if (X) v += a * X[i];
        if (Y) v += b * Y[i];
        if (Z) v += c * Z[i];
        if (V) v += d * V[i];
        out[i] = v;
    }
}

static unsigned blocks_for(long long n) {
    long long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <class T>
hipError_t launch_adjoint_sweep(int dir, int order, AdjArgs<T> a, hipStream_t s) {
    const int nd = a.n[dir];
    const long long plane = dir == 0 ? (long long)a.n[1] * a.n[2]
                          : dir == 1 ? (long long)a.n[0] * a.n[2] : (long long)a.n[0] * a.n[1];
    const unsigned gx = (unsigned)((plane + 255) / 256);
    a.seg = choose_segment(nd, (int)(gx * 256));
    const unsigned gy = (nd + a.seg - 1) / a.seg;
    const dim3 grid(gx, gy), block(256);
    if ((dir != 1 && dir != 2) || !a.pk) return hipErrorInvalidValue;
    const bool hub = a.bc == RH_BC_HUBBLE;
    auto go = [&](auto kernel) { kernel<<<grid, block, 0, s>>>(a); };
    if (order == 5) {
        if (dir == 1) hub ? go(adj_roll<T, 5, 1, true>) : go(adj_roll<T, 5, 1, false>);
        else hub ? go(adj_roll<T, 5, 2, true>) : go(adj_roll<T, 5, 2, false>);
    } else {
        if (dir == 1) hub ? go(adj_roll<T, 7, 1, true>) : go(adj_roll<T, 7, 1, false>);
        else hub ? go(adj_roll<T, 7, 2, true>) : go(adj_roll<T, 7, 2, false>);
    }
    return hipGetLastError();
}

// Whole-row x adjoint for periodic rows of these lengths (RH_ADJ_XROW=0 keeps
// the tiled kernel and the separate pack launch, for comparisons).
bool adjoint_x_rows(const int n[3], int bc_x) {
    static const bool enabled = [] {
        const char* e = getenv("RH_ADJ_XROW");
        return !(e && e[0] == '0');
    }();
    const int nx = n[0];
    return enabled && bc_x == RH_BC_PERIODIC &&
           (nx == 32 || nx == 64 || nx == 96 || nx == 128 || nx == 192 || nx == 256);
}

template <class T, int ORDER>
static void launch_adjoint_rows(const AdjArgs<T>& a, const Lin3<T>& init, hipStream_t s) {
    const int nx = a.n[0];
    const long long nrows = (long long)a.n[1] * a.n[2];
    auto go = [&](auto kernel, int nxk) {
        const int rpb = 256 / nxk;
        kernel<<<dim3((unsigned)((nrows + rpb - 1) / rpb)), dim3(rpb * nxk), 0, s>>>(a, init);
    };
    switch (nx) {
        case 32: go(adj_xrow<T, ORDER, 32>, 32); break;
        case 64: go(adj_xrow<T, ORDER, 64>, 64); break;
        case 96: go(adj_xrow<T, ORDER, 96>, 96); break;
        case 128: go(adj_xrow<T, ORDER, 128>, 128); break;
        case 192: go(adj_xrow<T, ORDER, 192>, 192); break;
        default: go(adj_xrow<T, ORDER, 256>, 256); break;
    }
}

template <class T>
hipError_t launch_adjoint_x(int order, AdjArgs<T> a, Lin3<T> init, hipStream_t s) {
    if (!a.pk) return hipErrorInvalidValue;
    if (adjoint_x_rows(a.n, a.bc)) {
        if (order == 5) launch_adjoint_rows<T, 5>(a, init, s);
        else launch_adjoint_rows<T, 7>(a, init, s);
        return hipGetLastError();
    }
    const int tx = adjoint_tile_x(a.n[0]);
    const int ty = tx == 64 ? 4 : 256 / tx;
    const long long ntx = (a.n[0] + tx - 1) / tx;
    const long long nrt = ((long long)a.n[1] * a.n[2] + ty - 1) / ty;
    const dim3 grid((unsigned)(ntx * nrt));
    if (order == 5) {
        if (tx == 64) adj_x<T, 5, 64, 4><<<grid, 256, 0, s>>>(a, init);
        else if (tx == 32) adj_x<T, 5, 32, 8><<<grid, 256, 0, s>>>(a, init);
        else adj_x<T, 5, 16, 16><<<grid, 256, 0, s>>>(a, init);
    } else {
        if (tx == 64) adj_x<T, 7, 64, 4><<<grid, 256, 0, s>>>(a, init);
        else if (tx == 32) adj_x<T, 7, 32, 8><<<grid, 256, 0, s>>>(a, init);
        else adj_x<T, 7, 16, 16><<<grid, 256, 0, s>>>(a, init);
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_adjoint_pack(const T* u, T* pk, long long ncell, hipStream_t s) {
    adj_pack<T><<<blocks_for(ncell), 256, 0, s>>>(u, pk, ncell);
    return hipGetLastError();
}

template <class T>
hipError_t launch_fill_zero(T* p, long long n, hipStream_t s) {
    fill_zero<T><<<blocks_for(n), 256, 0, s>>>(p, n);
    return hipGetLastError();
}

template <class T>
hipError_t launch_lincomb(T* out, long long n, T a, const T* X, T b, const T* Y, T c, const T* Z, T d,
                          const T* V, hipStream_t s) {
    lincomb<T><<<blocks_for(n), 256, 0, s>>>(out, n, a, X, b, Y, c, Z, d, V);
    return hipGetLastError();
}

#define RH_ADJ_INSTANTIATE(T)                                                                      \
    template hipError_t launch_adjoint_sweep<T>(int, int, AdjArgs<T>, hipStream_t);               \
    template hipError_t launch_fill_zero<T>(T*, long long, hipStream_t);                          \
    template hipError_t launch_adjoint_pack<T>(const T*, T*, long long, hipStream_t);             \
    template hipError_t launch_adjoint_x<T>(int, AdjArgs<T>, Lin3<T>, hipStream_t);                \
    template hipError_t launch_lincomb<T>(T*, long long, T, const T*, T, const T*, T, const T*, T, \
                                          const T*, hipStream_t);

RH_ADJ_INSTANTIATE(float)
RH_ADJ_INSTANTIATE(double)

}  // namespace rh
