// rh_adjoint.hip -- gfx950 kernels of the adjoint of L and of the SSP-RK3 step.
//
// One adjoint sweep per axis.  Each lane owns a segment [k0, k1) of one grid
// line along the sweep axis and rolls along it over every face whose stencil
// reaches an owned position (the segment plus R faces on each side), keeping a
// register window of 2R cells of split fluxes and of split-flux adjoints.  For
// each face it adds the face weight g = (w_{i+1} - w_i)/h times the WENO
// gradients to the window; a position leaving the window is complete and, if
// the lane owns it, is mapped through the flux Jacobian and added to the
// adjoint field.  Every cell (and every ghost position that copies it under
// outflow boundaries) is owned by exactly one lane per sweep, so the
// read-modify-write of the adjoint needs no atomics.
#include "rh_internal.hpp"
#include "rh_adjoint.hpp"
#include "../../include/rh.h"

namespace rh {

namespace {

template <class T, int DIR>
struct Column {
    // lane -> line: plane axes are (y, z) for DIR 0, (x, z) for DIR 1, (x, y) for DIR 2
    long long base;
    long long stride;
    int ia, ib;   // the two transverse indices
};

template <class T, int DIR>
__device__ __forceinline__ bool column_of(const AdjArgs<T>& A, unsigned p, Column<T, DIR>& C) {
    const int nx = A.n[0], ny = A.n[1], nz = A.n[2];
    if (DIR == 0) {
        const int y = (int)(p % (unsigned)ny), z = (int)(p / (unsigned)ny);
        if (z >= nz) return false;
        C.ia = y;
        C.ib = z;
        C.base = (long long)nx * (y + (long long)ny * z);
        C.stride = 1;
    } else if (DIR == 1) {
        const int x = (int)(p % (unsigned)nx), z = (int)(p / (unsigned)nx);
        if (z >= nz) return false;
        C.ia = x;
        C.ib = z;
        C.base = x + (long long)nx * ny * z;
        C.stride = nx;
    } else {
        const int x = (int)(p % (unsigned)nx), y = (int)(p / (unsigned)nx);
        if (y >= ny) return false;
        C.ia = x;
        C.ib = y;
        C.base = x + (long long)nx * y;
        C.stride = (long long)nx * ny;
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
    const long long id = C.base + mm * C.stride;
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = A.u[f * A.fstride + id];
}

// State at line position m with its velocity along the sweep axis and pressure:
// from the recovery pack when one is given (interior, periodic and outflow
// positions), else recovered here in FP64 (always for analytic ghosts).
template <class T, int DIR, bool PACK>
__device__ __forceinline__ void adj_state(const AdjArgs<T>& A, const Column<T, DIR>& C, int m, T u[5], T& v,
                                          T& P) {
    const int nd = A.n[DIR];
    int mm = m;
    bool analytic = false;
    if (m < 0 || m >= nd) {
        if (A.bc == RH_BC_PERIODIC) {
            mm = m % nd;
            if (mm < 0) mm += nd;
        } else if (A.bc == RH_BC_OUTFLOW) {
            mm = m < 0 ? 0 : nd - 1;
        } else {
            analytic = true;
        }
    }
    if (analytic) {
        adj_load<T, DIR>(A, C, m, u);
    } else {
        const long long id = C.base + mm * C.stride;
#pragma unroll
        for (int f = 0; f < 5; ++f) u[f] = A.u[f * A.fstride + id];
        if constexpr (PACK) {
            v = A.pk[id] * u[1 + DIR];
            P = A.pk[A.fstride + id];
            return;
        }
    }
    double vd, pd;
    unsigned dummy = 0;
    recover_vp<DIR>((double)u[0], (double)u[1], (double)u[2], (double)u[3], vd, pd, dummy);
    v = (T)vd;
    P = (T)pd;
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
    const long long id = C.base + mm * C.stride;
#pragma unroll
    for (int f = 0; f < 5; ++f) w[f] = A.w[f * A.fstride + id];
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
#ifndef RH_ADJ_GROUP_F32_W5
#define RH_ADJ_GROUP_F32_W5 3
#endif
#ifndef RH_ADJ_GROUP_OTHER
#define RH_ADJ_GROUP_OTHER 2
#endif

template <class T, int ORDER>
struct AdjGroup {
    static constexpr int value = (sizeof(T) == 4 && ORDER == 5) ? RH_ADJ_GROUP_F32_W5 : RH_ADJ_GROUP_OTHER;
};

template <class T, int ORDER, int DIR, bool PACK, int CLO, int CHI>
__device__ __forceinline__ void adj_pass(const AdjArgs<T>& A, const Column<T, DIR>& C, int k0, int k1) {
    constexpr int R = (ORDER + 1) / 2, W = 2 * R, NC = CHI - CLO;
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

    // split fluxes of the group's components from a cell state
    auto group_flux = [&](const T u[5], T v, T P, T fp[NC], T fm[NC]) {
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const int c = CLO + q;
            T f;
            if (c == 0) f = u[1 + DIR];
            else if (c == 4) f = u[4] * v;
            else f = u[c] * v + (c == 1 + DIR ? P : (T)0);
            fp[q] = half * (f + u[c]);
            fm[q] = half * (f - u[c]);
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
        const long long id = C.base + (long long)tgt * C.stride;
#pragma unroll
        for (int f = 0; f < 5; ++f) uf[f] = A.u[f * A.fstride + id];
        if constexpr (PACK && CHI > 1) {
            pkf[0] = A.pk[id];
#pragma unroll
            for (int q = 1; q < 5; ++q) pkf[q] = A.pk[(q + 1) * A.fstride + id];
        }
        if (tgt == last_tgt) return;
        if (CLO == 0 && A.zero_init) {
#pragma unroll
            for (int f = 0; f < 5; ++f) ubo[f] = (T)0;
            return;
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) ubo[f] = A.ub[f * A.fstride + id];
    };
    // ub += scale * sum over the group of (d f+_c/du)^T a+_c + (d f-_c/du)^T a-_c
    auto finish_pack = [&](int tgt, const T apj[NC], const T amj[NC]) {
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
        const long long id = C.base + (long long)tgt * C.stride;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            ubo[f] = ubo[f] + A.scale * g[f];
            A.ub[f * A.fstride + id] = ubo[f];
        }
        last_tgt = tgt;
    };
    auto finish = [&](int tgt, const T apj[NC], const T amj[NC]) {
        if constexpr (PACK) {
            finish_pack(tgt, apj, amj);
            return;
        }
        double lam[5] = {0.0, 0.0, 0.0, 0.0, 0.0}, dl[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            lam[CLO + q] = 0.5 * ((double)apj[q] + (double)amj[q]);
            dl[CLO + q] = 0.5 * ((double)apj[q] - (double)amj[q]);
        }
        double g[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) g[c] = dl[c];
        g[1 + DIR] += lam[0];
        if constexpr (CHI > 1) {
            double vd, pd, gv[4], gp[4];
            recover_vp_grad<DIR>((double)uf[0], (double)uf[1], (double)uf[2], (double)uf[3], vd, pd, gv, gp);
            // F_c = M_c v + p delta(c, 1+DIR) (c = 1..3), F_4 = N v
            double S = 0.0;
#pragma unroll
            for (int c = (CLO > 1 ? CLO : 1); c < CHI; ++c) {
                S += lam[c] * (double)uf[c];
                g[c] += lam[c] * vd;
            }
            const double lp = lam[1 + DIR];
#pragma unroll
            for (int m = 0; m < 4; ++m) g[m] += S * gv[m] + lp * gp[m];
        }
        const long long id = C.base + (long long)tgt * C.stride;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            ubo[f] = ubo[f] + A.scale * (T)g[f];
            A.ub[f * A.fstride + id] = ubo[f];
        }
        last_tgt = tgt;
    };

    T wp[NC][W], wm[NC][W], ap[NC][W], am[NC][W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T u[5], v, P, fp[NC], fm[NC];
        adj_state<T, DIR, PACK>(A, C, i_lo - R + 1 + j, u, v, P);
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
    adj_state<T, DIR, PACK>(A, C, i_lo + R + 1, un, vn, Pn);
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
        adj_state<T, DIR, PACK>(A, C, i + R + 2, un, vn, Pn);
        int tgt = 0;
        const bool own = target(i - R + 1, tgt);
        if (own) fetch_cell(tgt);
#pragma unroll
        for (int q = 0; q < NC; ++q) {
            const T g = (wr[q] - wl[q]) * A.inv_h;
            wl[q] = wr[q];
            if constexpr (ORDER == 5) {
                weno5_grad_acc<T>(wp[q][0], wp[q][1], wp[q][2], wp[q][3], wp[q][4], (T)4 * eps, g,
                                  ap[q][0], ap[q][1], ap[q][2], ap[q][3], ap[q][4]);
                weno5_grad_acc<T>(wm[q][5], wm[q][4], wm[q][3], wm[q][2], wm[q][1], (T)4 * eps, g,
                                  am[q][5], am[q][4], am[q][3], am[q][2], am[q][1]);
            } else {
                T sv[7], o[7];
#pragma unroll
                for (int j = 0; j < 7; ++j) { sv[j] = wp[q][j]; o[j] = (T)0; }
                weno7_grad_acc<T>(sv, eps, g, o);
#pragma unroll
                for (int j = 0; j < 7; ++j) ap[q][j] += o[j];
#pragma unroll
                for (int j = 0; j < 7; ++j) { sv[j] = wm[q][7 - j]; o[j] = (T)0; }
                weno7_grad_acc<T>(sv, eps, g, o);
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

template <class T, int ORDER, int DIR, bool PACK, int CLO>
__device__ __forceinline__ void adj_passes(const AdjArgs<T>& A, const Column<T, DIR>& C, int k0, int k1) {
    if constexpr (CLO < 5) {
        constexpr int GS = AdjGroup<T, ORDER>::value;
        constexpr int CHI = CLO + GS < 5 ? CLO + GS : 5;
        adj_pass<T, ORDER, DIR, PACK, CLO, CHI>(A, C, k0, k1);
        adj_passes<T, ORDER, DIR, PACK, CHI>(A, C, k0, k1);
    }
}

// Three waves per SIMD for the FP32 sweeps that read the recovery pack (their
// register window fits in 168 VGPRs); the others take what the window needs.
template <class T, bool PACK>
struct AdjMinBlocks {
    static constexpr int value = (sizeof(T) == 4 && PACK) ? 3 : 1;
};

template <class T, int ORDER, int DIR, bool PACK>
__global__ void __launch_bounds__(256, (AdjMinBlocks<T, PACK>::value)) adj_roll(AdjArgs<T> A) {
    Column<T, DIR> C;
    if (!column_of<T, DIR>(A, blockIdx.x * 256u + threadIdx.x, C)) return;
    const int k0 = blockIdx.y * A.seg;
    const int k1 = min(k0 + A.seg, A.n[DIR]);
    adj_passes<T, ORDER, DIR, PACK, 0>(A, C, k0, k1);
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

// Square tiles of 256-byte rows through LDS (64 x 64 FP32, 32 x 32 FP64), so
// that every read and write of a wave is a contiguous 256-byte run.  init may
// alias out (each element is read and written by the same lane).
template <class T>
struct TransposeTile {
    static constexpr int value = 256 / sizeof(T);
};

template <class T, bool INIT>
__global__ void __launch_bounds__(256) transpose_xy(const T* __restrict__ in, T* out, int R, int C, int nz,
                                                    long long fs, Lin3<T> init, T s) {
    constexpr int TS = TransposeTile<T>::value, RS = 256 / TS;
    __shared__ T tile[TS][TS + 1];
    const int z = blockIdx.z % nz, f = blockIdx.z / nz;
    const int fo = f == 1 ? 2 : (f == 2 ? 1 : f);
    const long long plane = (long long)R * C;
    const T* src = in + f * fs + z * plane;
    const long long dbase = fo * fs + z * plane;
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int c0 = blockIdx.x * TS, r0 = blockIdx.y * TS;
#pragma unroll
    for (int kk = 0; kk < TS / RS; ++kk) {
        const int k = ty + kk * RS;
        const int r = r0 + k, c = c0 + tx;
        if (r < R && c < C) tile[k][tx] = src[(long long)r * C + c];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TS / RS; ++kk) {
        const int k = ty + kk * RS;
        const int c = c0 + k, r = r0 + tx;   // output row c, column r
        if (r < R && c < C) {
            const long long o = dbase + (long long)c * R + r;
            T v = s * tile[tx][k];
            if (INIT) {
                T acc = (T)0;
                if (init.X1) acc += init.a1 * init.X1[o];
                if (init.X2) acc += init.a2 * init.X2[o];
                if (init.X3) acc += init.a3 * init.X3[o];
                v = acc + v;
            }
            out[o] = v;
        }
    }
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
    if (dir != 1 && dir != 2) return hipErrorInvalidValue;
    if (dir == 2 && !a.pk) return hipErrorInvalidValue;   // z always runs with the pack
    if (order == 5) {
        if (dir == 1 && !a.pk) adj_roll<T, 5, 1, false><<<grid, block, 0, s>>>(a);
        else if (dir == 1) adj_roll<T, 5, 1, true><<<grid, block, 0, s>>>(a);
        else adj_roll<T, 5, 2, true><<<grid, block, 0, s>>>(a);
    } else {
        if (dir == 1 && !a.pk) adj_roll<T, 7, 1, false><<<grid, block, 0, s>>>(a);
        else if (dir == 1) adj_roll<T, 7, 1, true><<<grid, block, 0, s>>>(a);
        else adj_roll<T, 7, 2, true><<<grid, block, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_adjoint_pack(const T* u, T* pk, long long ncell, hipStream_t s) {
    adj_pack<T><<<blocks_for(ncell), 256, 0, s>>>(u, pk, ncell);
    return hipGetLastError();
}

template <class T>
hipError_t launch_transpose_xy(const T* in, T* out, int R, int C, int nz, long long fs, Lin3<T> init, T s,
                               hipStream_t st) {
    constexpr int TS = TransposeTile<T>::value;
    if ((long long)5 * nz > 65535) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((C + TS - 1) / TS), (unsigned)((R + TS - 1) / TS), (unsigned)(5 * nz));
    if (init.X1 || init.X2 || init.X3) transpose_xy<T, true><<<grid, 256, 0, st>>>(in, out, R, C, nz, fs, init, s);
    else transpose_xy<T, false><<<grid, 256, 0, st>>>(in, out, R, C, nz, fs, init, s);
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
    template hipError_t launch_transpose_xy<T>(const T*, T*, int, int, int, long long, Lin3<T>, T,     \
                                               hipStream_t);                                       \
    template hipError_t launch_lincomb<T>(T*, long long, T, const T*, T, const T*, T, const T*, T, \
                                          const T*, hipStream_t);

RH_ADJ_INSTANTIATE(float)
RH_ADJ_INSTANTIATE(double)

}  // namespace rh
