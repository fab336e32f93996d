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

template <class T, int ORDER, int DIR>
__global__ void __launch_bounds__(256) adj_roll(AdjArgs<T> A) {
    constexpr int R = (ORDER + 1) / 2, W = 2 * R;
    Column<T, DIR> C;
    if (!column_of<T, DIR>(A, blockIdx.x * 256u + threadIdx.x, C)) return;
    const int nd = A.n[DIR];
    const bool periodic = A.bc == RH_BC_PERIODIC;
    const int k0 = blockIdx.y * A.seg;
    const int k1 = min(k0 + A.seg, nd);
    int i_lo = k0 - R, i_hi = k1 + R - 2;
    if (!periodic) {
        i_lo = max(i_lo, -1);
        i_hi = min(i_hi, nd - 1);
    }
    // owned positions [own_lo, own_hi): outflow edges also own the ghost positions
    const int own_lo = (!periodic && k0 == 0 && A.bc == RH_BC_OUTFLOW) ? -(1 << 30) : k0;
    const int own_hi = (!periodic && k1 == nd && A.bc == RH_BC_OUTFLOW) ? (1 << 30) : k1;
    const T eps = A.eps;

    auto finalize = [&](int pos, const T ap[5], const T am[5]) {
        if (pos < own_lo || pos >= own_hi) return;
        int tgt = pos;
        if (pos < 0 || pos >= nd) {
            if (A.bc != RH_BC_OUTFLOW) return;   // analytic ghosts are constants
            tgt = pos < 0 ? 0 : nd - 1;
        }
        T u[5], ub[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
        adj_load<T, DIR>(A, C, tgt, u);
        split_flux_vjp<T, DIR>(u, ap, am, ub);
        const long long id = C.base + (long long)tgt * C.stride;
#pragma unroll
        for (int f = 0; f < 5; ++f) A.ub[f * A.fstride + id] += ub[f];
    };

    T wp[5][W], wm[5][W], ap[5][W], am[5][W];
    unsigned dummy = 0;
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T u[5], fp[5], fm[5];
        adj_load<T, DIR>(A, C, i_lo - R + 1 + j, u);
        split_flux<T, DIR>(u, fp, fm, dummy);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            wp[c][j] = fp[c];
            wm[c][j] = fm[c];
            ap[c][j] = (T)0;
            am[c][j] = (T)0;
        }
    }
    T wl[5];
    adj_weight<T, DIR>(A, C, i_lo, wl);
    for (int i = i_lo; i <= i_hi; ++i) {
        T wr[5];
        adj_weight<T, DIR>(A, C, i + 1, wr);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T g = (wr[c] - wl[c]) * A.inv_h;
            wl[c] = wr[c];
            if constexpr (ORDER == 5) {
                weno5_grad_acc<T>(wp[c][0], wp[c][1], wp[c][2], wp[c][3], wp[c][4], (T)4 * eps, g,
                                  ap[c][0], ap[c][1], ap[c][2], ap[c][3], ap[c][4]);
                weno5_grad_acc<T>(wm[c][5], wm[c][4], wm[c][3], wm[c][2], wm[c][1], (T)4 * eps, g,
                                  am[c][5], am[c][4], am[c][3], am[c][2], am[c][1]);
            } else {
                T s[7], o[7];
                for (int j = 0; j < 7; ++j) { s[j] = wp[c][j]; o[j] = (T)0; }
                weno7_grad_acc<T>(s, eps, g, o);
                for (int j = 0; j < 7; ++j) ap[c][j] += o[j];
                for (int j = 0; j < 7; ++j) { s[j] = wm[c][7 - j]; o[j] = (T)0; }
                weno7_grad_acc<T>(s, eps, g, o);
                for (int j = 0; j < 7; ++j) am[c][7 - j] += o[j];
            }
        }
        {
            T a0p[5], a0m[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                a0p[c] = ap[c][0];
                a0m[c] = am[c][0];
            }
            finalize(i - R + 1, a0p, a0m);
        }
        if (i < i_hi) {
            T u[5], fp[5], fm[5];
            adj_load<T, DIR>(A, C, i + R + 1, u);
            split_flux<T, DIR>(u, fp, fm, dummy);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
#pragma unroll
                for (int j = 0; j < W - 1; ++j) {
                    wp[c][j] = wp[c][j + 1];
                    wm[c][j] = wm[c][j + 1];
                    ap[c][j] = ap[c][j + 1];
                    am[c][j] = am[c][j + 1];
                }
                wp[c][W - 1] = fp[c];
                wm[c][W - 1] = fm[c];
                ap[c][W - 1] = (T)0;
                am[c][W - 1] = (T)0;
            }
        }
    }
    // positions still in the window after the last face
#pragma unroll
    for (int j = 1; j < W; ++j) {
        T ajp[5], ajm[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            ajp[c] = ap[c][j];
            ajm[c] = am[c][j];
        }
        finalize(i_hi - R + 1 + j, ajp, ajm);
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
    if (order == 5) {
        if (dir == 0) adj_roll<T, 5, 0><<<grid, block, 0, s>>>(a);
        else if (dir == 1) adj_roll<T, 5, 1><<<grid, block, 0, s>>>(a);
        else adj_roll<T, 5, 2><<<grid, block, 0, s>>>(a);
    } else {
        if (dir == 0) adj_roll<T, 7, 0><<<grid, block, 0, s>>>(a);
        else if (dir == 1) adj_roll<T, 7, 1><<<grid, block, 0, s>>>(a);
        else adj_roll<T, 7, 2><<<grid, block, 0, s>>>(a);
    }
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
    template hipError_t launch_lincomb<T>(T*, long long, T, const T*, T, const T*, T, const T*, T, \
                                          const T*, hipStream_t);

RH_ADJ_INSTANTIATE(float)
RH_ADJ_INSTANTIATE(double)

}  // namespace rh
