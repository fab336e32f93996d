// rh_kernels.hip -- gfx950 kernels of the WENO / SSP-RK3 hot path.
//
// One evaluation of L(u) (Eq. (2) of Sikorski et al., arXiv:1604.03360) is split
// into one sweep per grid axis, in the order x, y, z; each sweep adds its flux
// difference to an L accumulator in HBM and the last one fuses the Runge-Kutta
// stage combine (Sec. 1).  Fields are SoA [5][nz][ny][nx], x fastest.
//
//  * sweep_x: x is the contiguous axis, so a 256-thread block stages a tile of
//    TX x TY cells plus G ghost columns per side in LDS (coalesced loads, one
//    primitive recovery and flux split per staged cell), each lane computes the
//    numerical flux at the right face of its cell, the left faces of the tile's
//    first column are spread over lanes as single reconstructions, and the
//    face fluxes are exchanged through LDS for the difference.
//  * sweep_roll<DIR>: y and z are strided axes; each lane owns one (x, w)
//    column segment and rolls a register window of 2R cells of split fluxes
//    along the axis, so each face flux is computed once and each cell is
//    loaded and recovered once (plus 2R halo cells per segment).  Lanes of a
//    wave hold 64 consecutive x, so every load and store is coalesced.
#include <stdlib.h>

#include "rh_internal.hpp"
#include "../../include/rh.h"

namespace rh {

// ---------------------------------------------------------------------------
// Cell loads with the boundary condition of the sweep axis
// ---------------------------------------------------------------------------
template <class T, int DIR>
__device__ __forceinline__ void load_cell(const SweepArgs<T>& A, int ix, int iy, int iz, T u[5]) {
    int c[3] = {ix, iy, iz};
    const int nd = A.n[DIR];
    int m = c[DIR];
    if (m < 0 || m >= nd) {
        if (A.bc == RH_BC_PERIODIC) {
            m %= nd;
            if (m < 0) m += nd;
            c[DIR] = m;
        } else if (A.bc == RH_BC_OUTFLOW) {
            c[DIR] = m < 0 ? 0 : nd - 1;
        } else {
            double uh[5];
            hubble_conserved(A.hb, A.hb.c0[0] + c[0] * A.hb.h[0], A.hb.c0[1] + c[1] * A.hb.h[1],
                             A.hb.c0[2] + c[2] * A.hb.h[2], uh);
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = (T)uh[f];
            return;
        }
    }
    const long long id = c[0] + (long long)A.n[0] * (c[1] + (long long)A.n[1] * c[2]);
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = A.us[f * A.fstride + id];
}

// State of cell x of grid row `row` (row = y + ny z), ghosts along x by the
// boundary condition; the row is split into (y, z) only for analytic ghosts.
template <class T>
__device__ __forceinline__ void load_cell_x(const SweepArgs<T>& A, int x, int row, T u[5]) {
    const int nx = A.n[0];
    if (x < 0 || x >= nx) {
        if (A.bc == RH_BC_PERIODIC) {
            x %= nx;
            if (x < 0) x += nx;
        } else if (A.bc == RH_BC_OUTFLOW) {
            x = x < 0 ? 0 : nx - 1;
        } else {
            load_cell<T, 0>(A, x, row % A.n[1], row / A.n[1], u);
            return;
        }
    }
    const long long id = x + (long long)nx * row;
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = A.us[f * A.fstride + id];
}

// One reconstruction from a window of 2R split fluxes of cells i-R+1 .. i+R
// (interface i+1/2): plus = left-biased on f+, minus = mirrored on f-.
// WENO5 takes 4 eps (its smoothness indicators are carried as 4 beta).
template <class T, int ORDER>
__device__ __forceinline__ T recon_plus(const T* w, T eps) {
    if constexpr (ORDER == 5) return weno5<T>(w[0], w[1], w[2], w[3], w[4], (T)4 * eps);
    else return weno7<T>(w[0], w[1], w[2], w[3], w[4], w[5], w[6], eps);
}
template <class T, int ORDER>
__device__ __forceinline__ T recon_minus(const T* w, T eps) {
    if constexpr (ORDER == 5) return weno5<T>(w[5], w[4], w[3], w[2], w[1], (T)4 * eps);
    else return weno7<T>(w[7], w[6], w[5], w[4], w[3], w[2], w[1], eps);
}

// Accumulate L of this direction and either store L or apply the stage combine:
// stage 1: u1 = u + dt L; stage 2: 3/4 u^n + 1/4 (u1 + dt L);
// stage 3: 1/3 u^n + 2/3 (u2 + dt L).
template <class T>
__device__ __forceinline__ void epilogue(const SweepArgs<T>& A, long long id, T L[5]) {
    if (!A.first) {
#pragma unroll
        for (int c = 0; c < 5; ++c) L[c] = A.lacc[c * A.fstride + id] + L[c];
    }
    if (A.stage == STAGE_WRITE_L) {
#pragma unroll
        for (int c = 0; c < 5; ++c) A.lacc[c * A.fstride + id] = L[c];
        return;
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const long long q = c * A.fstride + id;
        T v = A.us[q] + A.dt * L[c];
        if (A.stage == STAGE_2) v = (T)0.75 * A.u0[q] + (T)0.25 * v;
        else if (A.stage == STAGE_3) v = rk3_last(A.u0[q], v);
        A.uout[q] = v;
    }
}

// ---------------------------------------------------------------------------
// x sweep: LDS tile
// ---------------------------------------------------------------------------
// blk: linear block index within the grid (x tile fastest, then row tile)
template <class T, int ORDER, int TX>
__device__ __forceinline__ void sweep_x_body(const SweepArgs<T>& A, int blk) {
    constexpr int R = (ORDER + 1) / 2, G = R, TY = 256 / TX, PW = TX + 2 * G;
    __shared__ T sp[5 * TY * PW];
    __shared__ T sm[5 * TY * PW];
    const int nx = A.n[0], ny = A.n[1];
    const int nrows = ny * A.n[2];
    const int ntx = (nx + TX - 1) / TX;
    const int bx = blk % ntx, by = blk / ntx;
    const int x0 = bx * TX, r0 = by * TY;
    const int tid = threadIdx.x;
    unsigned clamped = 0;

    for (int idx = tid; idx < TY * PW; idx += 256) {
        const int ly = idx / PW, lx = idx - ly * PW;
        const int row = r0 + ly, gx = x0 + lx - G;
        if (row < nrows && gx < nx + G) {
            T u[5], fp[5], fm[5];
            load_cell_x<T>(A, gx, row, u);
            unsigned c = 0;
            split_flux<T, 0>(u, fp, fm, c);
            // floors are counted once per cell and evaluation of L: by the
            // first sweep, for the cells it owns
            if (A.first && lx >= G && lx < G + TX && gx < nx) clamped += c;
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                sp[(c * TY + ly) * PW + lx] = fp[c];
                sm[(c * TY + ly) * PW + lx] = fm[c];
            }
        }
    }
    __syncthreads();

    const int lx = tid % TX, ly = tid / TX;
    const int gx = x0 + lx, row = r0 + ly;
    const bool active = gx < nx && row < nrows;
    const T eps2 = (T)4 * A.eps;   // the staged split fluxes are doubled
    T Fr[5];
    if (active) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const int o = (c * TY + ly) * PW + lx + 1;
            Fr[c] = recon_plus<T, ORDER>(sp + o, eps2) + recon_minus<T, ORDER>(sm + o, eps2);
        }
    }
    // left face of the tile's first column, one reconstruction per lane:
    // job = row * 10 + component * 2 + sign
    const bool has_ex = tid < 10 * TY;
    T ex = (T)0;
    if (has_ex) {
        const int ely = tid / 10, ec = (tid % 10) >> 1, esg = tid & 1;
        if (r0 + ely < nrows) {
            const int o = (ec * TY + ely) * PW;   // window starts at staged column 0
            ex = esg == 0 ? recon_plus<T, ORDER>(sp + o, eps2) : recon_minus<T, ORDER>(sm + o, eps2);
        }
    }
    __syncthreads();
    T* fh = sp;   // face fluxes [5][TY][TX+1]
    T* fe = sm;   // left-face reconstructions [TY][10]
    if (active) {
#pragma unroll
        for (int c = 0; c < 5; ++c) fh[(c * TY + ly) * (TX + 1) + lx + 1] = Fr[c];
    }
    if (has_ex) fe[tid] = ex;
    __syncthreads();
    if (active) {
        T L[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T Fl = lx == 0 ? fe[ly * 10 + c * 2] + fe[ly * 10 + c * 2 + 1]
                                 : fh[(c * TY + ly) * (TX + 1) + lx];
            L[c] = (Fl - Fr[c]) * ((T)0.5 * A.inv_h);
        }
        epilogue(A, gx + (long long)nx * row, L);
    }
    if (clamped) atomicAdd(A.clamps, clamped);
}

// ---------------------------------------------------------------------------
// y / z sweeps: per-lane rolling register window
// ---------------------------------------------------------------------------
// bx: 256-lane chunk of the (x, w) plane; by: segment along the sweep axis
template <class T, int ORDER, int DIR>
__device__ __forceinline__ void sweep_roll_body(const SweepArgs<T>& A, unsigned bx, int by) {
    constexpr int R = (ORDER + 1) / 2, W = 2 * R;
    constexpr int WD = DIR == 1 ? 2 : 1;   // the other transverse axis
    const int nx = A.n[0], nw = A.n[WD];
    // lanes enumerate the (x, w) plane x-fastest, so a wave reads at most two
    // contiguous runs of x per field whatever nx is
    const unsigned p = bx * 256u + threadIdx.x;
    const int x = (int)(p % (unsigned)nx), w = (int)(p / (unsigned)nx);
    if (w >= nw) return;
    const int nd = A.n[DIR];
    const int k0 = by * A.seg;
    const int kend = min(k0 + A.seg, nd);
    const uint32_t sb = (uint32_t)sizeof(T) * (DIR == 1 ? (uint32_t)nx : (uint32_t)nx * A.n[1]);
    const uint32_t cb = (uint32_t)sizeof(T) *
                        (DIR == 1 ? (uint32_t)x + (uint32_t)nx * A.n[1] * (uint32_t)w
                                  : (uint32_t)x + (uint32_t)nx * (uint32_t)w);
    const long long F = A.fstride;
    unsigned clamped = 0;

    auto fetch = [&](int m, T u[5]) {
        if (m >= 0 && m < nd) {
            const uint32_t off = cb + (uint32_t)m * sb;
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = ld_off(A.us + f * F, off);
        } else if (DIR == 1) {
            load_cell<T, DIR>(A, x, m, w, u);
        } else {
            load_cell<T, DIR>(A, x, w, m, u);
        }
    };

    // The stage combine of cell k needs the stage input u(k), loaded R + 1 steps
    // earlier as the window's newest cell; by then a strided sweep has streamed
    // several MB through L2 and a second load would go to memory again.  Each
    // lane therefore keeps u of its last R + 1 cells in a private LDS ring
    // (slot = cell mod D, lanes in consecutive words; no barrier, a lane reads
    // only what it wrote).
    constexpr int D = R + 1 <= 4 ? 4 : 8;
    __shared__ T uring[D][5][256];
    const bool combine = A.stage != STAGE_WRITE_L;
    auto ring_put = [&](int m, const T uu[5]) {
#pragma unroll
        for (int f = 0; f < 5; ++f) uring[m & (D - 1)][f][threadIdx.x] = uu[f];
    };

    // window of interface k-1/2: cells k-R .. k+R-1
    T wp[5][W], wm[5][W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T u[5], fp[5], fm[5];
        fetch(k0 - R + j, u);
        if (j >= R && combine) ring_put(k0 - R + j, u);
        unsigned c = 0;
        split_flux<T, DIR>(u, fp, fm, c);
        if (A.first && j >= R && k0 - R + j < kend) clamped += c;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            wp[c][j] = fp[c];
            wm[c][j] = fm[c];
        }
    }
    const T eps2 = (T)4 * A.eps;   // the window holds doubled split fluxes
    const T hinv = (T)0.5 * A.inv_h;
    T Fl[5];
#pragma unroll
    for (int c = 0; c < 5; ++c)
        Fl[c] = recon_plus<T, ORDER>(wp[c], eps2) + recon_minus<T, ORDER>(wm[c], eps2);

    T nxt[5];
    fetch(k0 + R, nxt);
    for (int k = k0; k < kend; ++k) {
        T u[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) u[f] = nxt[f];
        fetch(k + 1 + R, nxt);   // next iteration's new cell, in flight during this one
        if (combine) ring_put(k + R, u);
        // epilogue operands of cell k: FP32 issues them before the arithmetic;
        // FP64 loads them after it to keep the register window within 256 VGPRs
        const uint32_t off = cb + (uint32_t)k * sb;
        T lo[5], us[5], u0[5];
        auto load_epilogue = [&]() {
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                lo[c] = A.first ? (T)0 : ld_off(A.lacc + c * F, off);
                us[c] = combine ? uring[k & (D - 1)][c][threadIdx.x] : (T)0;
                u0[c] = A.stage >= STAGE_2 ? ld_off(A.u0 + c * F, off) : (T)0;
            }
        };
        if constexpr (sizeof(T) == 4) load_epilogue();
        T fp[5], fm[5];
        unsigned c = 0;
        split_flux<T, DIR>(u, fp, fm, c);
        if (A.first && k + R < kend) clamped += c;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
            for (int j = 0; j < W - 1; ++j) {
                wp[c][j] = wp[c][j + 1];
                wm[c][j] = wm[c][j + 1];
            }
            wp[c][W - 1] = fp[c];
            wm[c][W - 1] = fm[c];
        }
        T Lk[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T Fr = recon_plus<T, ORDER>(wp[c], eps2) + recon_minus<T, ORDER>(wm[c], eps2);
            Lk[c] = (Fl[c] - Fr) * hinv;
            Fl[c] = Fr;
        }
        if constexpr (sizeof(T) != 4) load_epilogue();
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            T L = Lk[c];
            if (!A.first) L = lo[c] + L;
            T v;
            if (A.stage == STAGE_WRITE_L) {
                v = L;
            } else {
                v = us[c] + A.dt * L;
                if (A.stage == STAGE_2) v = (T)0.75 * u0[c] + (T)0.25 * v;
                else if (A.stage == STAGE_3) v = rk3_last(u0[c], v);
            }
            st_off(A.stage == STAGE_WRITE_L ? A.lacc + c * F : A.uout + c * F, off, v);
        }
    }
    if (clamped) atomicAdd(A.clamps, clamped);
}

// Minimum resident 256-thread blocks per CU for the rolling sweeps (= waves per
// SIMD); caps the register window so that enough waves hide load latency.
template <class T, int ORDER>
struct RollMinBlocks {
    static constexpr int value = sizeof(T) == 4 ? 3 : (ORDER == 5 ? 2 : 1);
};

template <class T, int ORDER, int TX>
__global__ void __launch_bounds__(256) sweep_x(SweepArgs<T> A) {
    sweep_x_body<T, ORDER, TX>(A, blockIdx.x);
}

template <class T, int ORDER, int DIR>
__global__ void __launch_bounds__(256, (RollMinBlocks<T, ORDER>::value)) sweep_roll(SweepArgs<T> A) {
    sweep_roll_body<T, ORDER, DIR>(A, blockIdx.x, blockIdx.y);
}

// ---------------------------------------------------------------------------
// Batched sweeps: one launch covers the same sweep of every grid of an event
// ensemble.  Each grid owns a contiguous range of the launch's blocks; a block
// finds its grid by binary search over the per-grid first-block table and runs
// the single-grid body on that grid's slice of the concatenated buffers.
// ---------------------------------------------------------------------------
template <class T>
__device__ __forceinline__ int find_grid(const BatchArgs<T>& B, int cls, int blk) {
    int lo = 0, hi = B.ngrid - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (B.grids[mid].blk0[cls] <= blk) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class T>
__device__ __forceinline__ SweepArgs<T> grid_args(const BatchArgs<T>& B, int g, int d) {
    const BatchGrid<T>& G = B.grids[g];
    SweepArgs<T> A = B.base;
    A.us = B.base.us + G.off;
    A.u0 = B.base.u0 + G.off;
    A.lacc = B.base.lacc + G.off;
    A.uout = B.base.uout ? B.base.uout + G.off : nullptr;
    A.fstride = (long long)G.n[0] * G.n[1] * G.n[2];
    A.n[0] = G.n[0];
    A.n[1] = G.n[1];
    A.n[2] = G.n[2];
    A.bc = G.bc[d];
    A.inv_h = G.inv_h[d];
    A.seg = G.seg[d];
    A.eps = G.eps;
    A.hb.t0 = G.t0;
    A.hb.e0 = G.e0;
    A.hb.n0 = G.n0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        A.hb.c0[a] = G.c0[a];
        A.hb.h[a] = G.h[a];
    }
    return A;
}

template <class T, int ORDER, int TX>
__global__ void __launch_bounds__(256) sweep_x_batch(BatchArgs<T> B) {
    const int g = find_grid(B, 0, blockIdx.x);
    const SweepArgs<T> A = grid_args(B, g, 0);
    sweep_x_body<T, ORDER, TX>(A, blockIdx.x - B.grids[g].blk0[0]);
}

template <class T, int ORDER, int DIR>
__global__ void __launch_bounds__(256, (RollMinBlocks<T, ORDER>::value)) sweep_roll_batch(BatchArgs<T> B) {
    const int g = find_grid(B, DIR, blockIdx.x);
    const SweepArgs<T> A = grid_args(B, g, DIR);
    const int lb = blockIdx.x - B.grids[g].blk0[DIR];
    const int gx = B.grids[g].nchunk[DIR];
    sweep_roll_body<T, ORDER, DIR>(A, (unsigned)(lb % gx), lb / gx);
}

// Stage combine with L = 0 (grids with no axis longer than one cell).
template <class T>
__global__ void combine_zero_L(SweepArgs<T> A) {
    const long long n = A.fstride;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        T L[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
        SweepArgs<T> B = A;
        B.first = 1;
        epilogue(B, i, L);
    }
}

// ---------------------------------------------------------------------------
// Field conversion
// ---------------------------------------------------------------------------
__device__ inline void prim_to_cons(const double pr[5], double u[5]) {
    const double e = pr[0], vx = pr[1], vy = pr[2], vz = pr[3], n = pr[4];
    const double p = e / 3.0;
    const double g2 = 1.0 / (1.0 - (vx * vx + vy * vy + vz * vz));
    const double w = e + p;
    u[0] = w * g2 - p;
    u[1] = w * g2 * vx;
    u[2] = w * g2 * vy;
    u[3] = w * g2 * vz;
    u[4] = n * sqrt(g2);
}

// Full FP64 primitive recovery (e, v, n) with the same floors as the sweeps.
__device__ inline void cons_to_prim(const double u[5], double pr[5], unsigned& clamped) {
    const double E = u[0], N = u[4];
    double Mx = u[1], My = u[2], Mz = u[3];
    if (E < kEFloor) {
        pr[0] = (E > 0.0 ? E : 0.0);
        pr[1] = pr[2] = pr[3] = 0.0;
        pr[4] = N;
        ++clamped;
        return;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    const double cap = (1.0 - kVDelta) * E * E;
    if (M2 > cap) {
        const double s = sqrt(cap / M2);
        Mx *= s; My *= s; Mz *= s;
        M2 = cap;
        ++clamped;
    }
    const double D = sqrt(4.0 * E * E - 3.0 * M2);
    const double k = 3.0 / (2.0 * E + D);
    pr[0] = 3.0 * ((E * E - M2) / (E + D));
    pr[1] = k * Mx;
    pr[2] = k * My;
    pr[3] = k * Mz;
    pr[4] = N * sqrt(1.0 - k * k * M2);
}

// Ideal gas: primitive -> conserved with p = (gamma - 1)(e - n), and the
// Newton recovery back.
__device__ inline void prim_to_cons_ideal(const double pr[5], double gm1, double u[5]) {
    const double e = pr[0], vx = pr[1], vy = pr[2], vz = pr[3], nn = pr[4];
    const double p = ideal_p(gm1, e, nn);
    const double g2 = 1.0 / (1.0 - (vx * vx + vy * vy + vz * vz));
    const double w = e + p;
    u[0] = w * g2 - p;
    u[1] = w * g2 * vx;
    u[2] = w * g2 * vy;
    u[3] = w * g2 * vz;
    u[4] = nn * sqrt(g2);
}

__device__ inline void cons_to_prim_ideal(const double u[5], double gm1, double pr[5], unsigned& clamped) {
    double kap, Mxs, Mys, Mzs, p, e;
    recover_ideal(u[0], u[1], u[2], u[3], u[4], gm1, kap, Mxs, Mys, Mzs, p, e, clamped);
    pr[0] = e;
    pr[1] = kap * Mxs;
    pr[2] = kap * Mys;
    pr[3] = kap * Mzs;
    pr[4] = u[4] * sqrt(1.0 - (pr[1] * pr[1] + pr[2] * pr[2] + pr[3] * pr[3]));
}

template <class T>
__global__ void set_fields_kernel(T* state, const double* src, int kind, long long n, int eos, double gm1) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double a[5], u[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) a[f] = src[f * n + i];
        if (kind == RH_FIELDS_PRIMITIVE && eos == EOS_IDEAL) prim_to_cons_ideal(a, gm1, u);
        else if (kind == RH_FIELDS_PRIMITIVE) prim_to_cons(a, u);
        else {
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = a[f];
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) state[f * n + i] = (T)u[f];
    }
}

template <class T>
__global__ void get_fields_kernel(const T* state, double* dst, int kind, long long n,
                                  unsigned* clamps, int eos, double gm1) {
    unsigned clamped = 0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        double u[5], o[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) u[f] = (double)state[f * n + i];
        if (kind == RH_FIELDS_PRIMITIVE && eos == EOS_IDEAL) cons_to_prim_ideal(u, gm1, o, clamped);
        else if (kind == RH_FIELDS_PRIMITIVE) cons_to_prim(u, o, clamped);
        else {
#pragma unroll
            for (int f = 0; f < 5; ++f) o[f] = u[f];
        }
#pragma unroll
        for (int f = 0; f < 5; ++f) dst[f * n + i] = o[f];
    }
    if (clamped) atomicAdd(clamps, clamped);
}

// ---------------------------------------------------------------------------
// FP64 totals: fixed partition of cells over blocks, fixed-order tree in LDS,
// then one block sums the partials in a fixed order -- deterministic.
// partials: [6][nblk] (5 sums and the count of cells with a non-finite value).
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) totals_pass1(const T* u, long long n, double* partials,
                                                    int nblk) {
    __shared__ double red[6][256];
    const long long chunk = (n + nblk - 1) / nblk;
    const long long beg = blockIdx.x * chunk;
    const long long end = min(n, beg + chunk);
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (long long i = beg + threadIdx.x; i < end; i += 256) {
        bool bad = false;
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            const double v = (double)u[f * n + i];
            s[f] += v;
            bad |= !isfinite(v);
        }
        s[5] += bad ? 1.0 : 0.0;
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) red[f][threadIdx.x] = s[f];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int f = 0; f < 6; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) partials[threadIdx.x * nblk + blockIdx.x] = red[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) totals_pass2(const double* partials, int nblk, double* out) {
    __shared__ double red[6][256];
    double s[6] = {0, 0, 0, 0, 0, 0};
    for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
        for (int f = 0; f < 6; ++f) s[f] += partials[f * nblk + b];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) red[f][threadIdx.x] = s[f];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
#pragma unroll
            for (int f = 0; f < 6; ++f) red[f][threadIdx.x] += red[f][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) out[threadIdx.x] = red[threadIdx.x][0];
}

// ---------------------------------------------------------------------------
// Host-side launch configuration
// ---------------------------------------------------------------------------
int choose_tile_x(int nx, int ghosts) {
    // fewest staged cells per useful cell: padded tiles plus their ghost columns
    int best = 64;
    double best_cost = 1e300;
    for (int tx : {64, 32, 16}) {
        const int ntx = (nx + tx - 1) / tx;
        const double cost = ntx * (tx + 2.0 * ghosts * 0.25) / nx;
        if (cost < best_cost - 1e-12) {
            best_cost = cost;
            best = tx;
        }
    }
    return best;
}

int choose_segment(int n, int ncol_lanes) {
    // enough lanes to fill the chip (about 2^19), segments no shorter than 16
    // cells (each segment recomputes 2R + 1 halo cells; at 96^3 segments of 16
    // instead of 32 double the lanes and measured 1.5x faster, at 256^3 the
    // lane target already gives 32)
    const long long target = 1LL << 19;
    long long nseg = (target + ncol_lanes - 1) / ncol_lanes;
    const long long max_seg = (n + 15) / 16;
    if (nseg > max_seg) nseg = max_seg;
    if (nseg < 1) nseg = 1;
    return (int)((n + nseg - 1) / nseg);
}

template <class T, int ORDER>
static hipError_t launch_x(const SweepArgs<T>& a, hipStream_t s) {
    const int tx = choose_tile_x(a.n[0], (ORDER + 1) / 2);
    const int ty = 256 / tx;
    const long long ntx = (a.n[0] + tx - 1) / tx;
    const long long nrt = ((long long)a.n[1] * a.n[2] + ty - 1) / ty;
    const dim3 grid((unsigned)(ntx * nrt));
    if (tx == 64) sweep_x<T, ORDER, 64><<<grid, 256, 0, s>>>(a);
    else if (tx == 32) sweep_x<T, ORDER, 32><<<grid, 256, 0, s>>>(a);
    else sweep_x<T, ORDER, 16><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

template <class T, int ORDER, int DIR>
static hipError_t launch_roll(SweepArgs<T> a, hipStream_t s) {
    const int wd = DIR == 1 ? 2 : 1;
    const long long cols = (long long)a.n[0] * a.n[wd];
    const unsigned gx = (unsigned)((cols + 255) / 256);
    const int seg = choose_segment(a.n[DIR], (int)(gx * 256));
    a.seg = seg;
    const unsigned gy = (a.n[DIR] + seg - 1) / seg;
    sweep_roll<T, ORDER, DIR><<<dim3(gx, gy), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fused x and y sweeps (periodic x, nx a multiple of 64 up to 256; WENO5, and
// WENO7 in FP32)
// ---------------------------------------------------------------------------
// A block holds whole x rows (lane = x) of one z plane and rolls along a y
// segment like sweep_roll_body.  Each row that enters the y window is
// recovered once (FP64) for both axes; when the row is owned its x split fluxes
// go to LDS (with periodic halo copies), every lane reconstructs its right x
// face, the face fluxes are exchanged through LDS and the row's x part of L is
// kept in an LDS ring until the y face of that row is done R steps later.  L is
// the x part plus the y part, summed in that order as in the split sweeps, so
// the result is bitwise that of sweep_x followed by sweep_roll<1>.
template <class T, int ORDER>
__global__ void __launch_bounds__(256, (RollMinBlocks<T, ORDER>::value)) sweep_xy(SweepArgs<T> A, T inv_hx) {
    constexpr int R = (ORDER + 1) / 2, W = 2 * R;
    constexpr int D = R;                  // rows whose x part of L is pending (row k's slot is read before row k + R enters)
    __shared__ T sx[2][5][256 + 2 * R];   // x split fluxes of the current row, halo copies at both ends
    __shared__ T sF[5][256];              // x face fluxes F(x + 1/2) of the current row
    __shared__ T lxr[D][5][256];          // x part of L of the last rows, by row mod D (rows are
                                          // uniform across the block: scalar index arithmetic)
    const int nx = A.n[0], ny = A.n[1];
    const int x = threadIdx.x, w = blockIdx.x;
    const int k0 = blockIdx.y * A.seg;
    const int kend = min(k0 + A.seg, ny);
    const uint32_t sb = (uint32_t)sizeof(T) * (uint32_t)nx;
    const uint32_t cb = (uint32_t)sizeof(T) * ((uint32_t)x + (uint32_t)nx * (uint32_t)ny * (uint32_t)w);
    const long long F = A.fstride;
    const T eps2 = (T)4 * A.eps;   // doubled split fluxes
    const T hinv = (T)0.5 * A.inv_h;
    const T hx = (T)0.5 * inv_hx;
    const int xl = x == 0 ? nx - 1 : x - 1;
    unsigned clamped = 0;

    auto fetch = [&](int m, T u[5]) {
        if (m >= 0 && m < ny) {
            const uint32_t off = cb + (uint32_t)m * sb;
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = ld_off(A.us + f * F, off);
        } else {
            load_cell<T, 1>(A, x, m, w, u);
        }
    };
    // recovery of row m's cell for both axes; y split fluxes out, and the x
    // part of L of row m into the ring when the row is owned (uniform per block)
    auto enter = [&](int m, const T u[5], T fp[5], T fm[5]) {
        double kap, Mxs, Mys, p;
        unsigned c = 0;
        recover_kp((double)u[0], (double)u[1], (double)u[2], (double)u[3], kap, Mxs, Mys, p, c);
        split_flux_vp<T, 1>(u, (T)(kap * Mys), (T)p, fp, fm);
        if (m < k0 || m >= kend) return;
        clamped += c;   // owned rows only: once per cell and evaluation of L
        T fpx[5], fmx[5];
        split_flux_vp<T, 0>(u, (T)(kap * Mxs), (T)p, fpx, fmx);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            sx[0][c][x + R] = fpx[c];
            sx[1][c][x + R] = fmx[c];
            if (x < R) {
                sx[0][c][x + nx + R] = fpx[c];
                sx[1][c][x + nx + R] = fmx[c];
            }
            if (x >= nx - R) {
                sx[0][c][x - nx + R] = fpx[c];
                sx[1][c][x - nx + R] = fmx[c];
            }
        }
        __syncthreads();
        T Fr[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            // window of face x + 1/2: cells x - R + 1 .. x + R at LDS positions x + 1 ..
            Fr[c] = recon_plus<T, ORDER>(&sx[0][c][x + 1], eps2) + recon_minus<T, ORDER>(&sx[1][c][x + 1], eps2);
            sF[c][x] = Fr[c];
        }
        __syncthreads();
        const int slot = m % D;
#pragma unroll
        for (int c = 0; c < 5; ++c) lxr[slot][c][x] = (sF[c][xl] - Fr[c]) * hx;
    };

    // y window of interface k-1/2: cells k-R .. k+R-1
    T wp[5][W], wm[5][W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        T u[5], fp[5], fm[5];
        fetch(k0 - R + j, u);
        enter(k0 - R + j, u, fp, fm);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            wp[c][j] = fp[c];
            wm[c][j] = fm[c];
        }
    }
    T Fl[5];
#pragma unroll
    for (int c = 0; c < 5; ++c)
        Fl[c] = recon_plus<T, ORDER>(wp[c], eps2) + recon_minus<T, ORDER>(wm[c], eps2);

    T nxt[5];
    fetch(k0 + R, nxt);
    for (int k = k0; k < kend; ++k) {
        T u[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) u[f] = nxt[f];
        fetch(k + 1 + R, nxt);
        const uint32_t off = cb + (uint32_t)k * sb;
        T lxk[5];   // x part of L of row k, read before row k + R takes its slot
#pragma unroll
        for (int c = 0; c < 5; ++c) lxk[c] = lxr[k % D][c][x];
        T fp[5], fm[5];
        enter(k + R, u, fp, fm);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
            for (int j = 0; j < W - 1; ++j) {
                wp[c][j] = wp[c][j + 1];
                wm[c][j] = wm[c][j + 1];
            }
            wp[c][W - 1] = fp[c];
            wm[c][W - 1] = fm[c];
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T Fr = recon_plus<T, ORDER>(wp[c], eps2) + recon_minus<T, ORDER>(wm[c], eps2);
            const T Lk = (Fl[c] - Fr) * hinv;
            Fl[c] = Fr;
            const T L = lxk[c] + Lk;
            T v;
            if (A.stage == STAGE_WRITE_L) {
                v = L;
            } else {
                v = ld_off(A.us + c * F, off) + A.dt * L;
                if (A.stage == STAGE_2) v = (T)0.75 * ld_off(A.u0 + c * F, off) + (T)0.25 * v;
                else if (A.stage == STAGE_3) v = rk3_last(ld_off(A.u0 + c * F, off), v);
            }
            st_off(A.stage == STAGE_WRITE_L ? A.lacc + c * F : A.uout + c * F, off, v);
        }
    }
    if (clamped) atomicAdd(A.clamps, clamped);
}

// RH_FUSE_XY=0 in the environment selects the separate sweeps everywhere (the
// results are bitwise the same; used to compare the two paths).
bool sweep_xy_applies(int order, const int n[3], int bc_x) {
    static const bool off = [] {
        const char* e = getenv("RH_FUSE_XY");
        return e && e[0] == '0';
    }();
    return !off && (order == 5 || order == 7) && bc_x == RH_BC_PERIODIC && n[0] % 64 == 0 &&
           n[0] >= 64 && n[0] <= 256 && n[1] > 1;
}

template <class T>
hipError_t launch_sweep_xy(int order, SweepArgs<T> a, T inv_hx, hipStream_t s) {
    if (!(order == 5 || order == 7) || a.n[0] % 64 != 0 || a.n[0] < 64 || a.n[0] > 256)
        return hipErrorInvalidValue;
    const int seg = choose_segment(a.n[1], a.n[0] * a.n[2]);
    a.seg = seg;
    const unsigned gy = (a.n[1] + seg - 1) / seg;
    const dim3 grid((unsigned)a.n[2], gy), block((unsigned)a.n[0]);
    if (order == 5) {
        sweep_xy<T, 5><<<grid, block, 0, s>>>(a, inv_hx);
    } else {
        sweep_xy<T, 7><<<grid, block, 0, s>>>(a, inv_hx);
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_sweep(int dir, int order, const SweepArgs<T>& a, hipStream_t s) {
    if (order == 5) {
        if (dir == 0) return launch_x<T, 5>(a, s);
        if (dir == 1) return launch_roll<T, 5, 1>(a, s);
        return launch_roll<T, 5, 2>(a, s);
    }
    if (dir == 0) return launch_x<T, 7>(a, s);
    if (dir == 1) return launch_roll<T, 7, 1>(a, s);
    return launch_roll<T, 7, 2>(a, s);
}

template <class T>
hipError_t launch_sweep_batch(int dir, int order, int tx, const BatchArgs<T>& b, int nblocks,
                              hipStream_t s) {
    const dim3 grid(nblocks), block(256);
    if (dir == 0) {
        if (order == 5) {
            if (tx == 64) sweep_x_batch<T, 5, 64><<<grid, block, 0, s>>>(b);
            else if (tx == 32) sweep_x_batch<T, 5, 32><<<grid, block, 0, s>>>(b);
            else sweep_x_batch<T, 5, 16><<<grid, block, 0, s>>>(b);
        } else {
            if (tx == 64) sweep_x_batch<T, 7, 64><<<grid, block, 0, s>>>(b);
            else if (tx == 32) sweep_x_batch<T, 7, 32><<<grid, block, 0, s>>>(b);
            else sweep_x_batch<T, 7, 16><<<grid, block, 0, s>>>(b);
        }
    } else if (dir == 1) {
        if (order == 5) sweep_roll_batch<T, 5, 1><<<grid, block, 0, s>>>(b);
        else sweep_roll_batch<T, 7, 1><<<grid, block, 0, s>>>(b);
    } else {
        if (order == 5) sweep_roll_batch<T, 5, 2><<<grid, block, 0, s>>>(b);
        else sweep_roll_batch<T, 7, 2><<<grid, block, 0, s>>>(b);
    }
    return hipGetLastError();
}

// Blocks of one grid in each sweep class for a batched launch (x tile width tx,
// rolling segment seg_y / seg_z); fills blk counts and the rolling chunk counts.
void batch_blocks(const int n[3], int tx, const int seg[3], int blocks[3], int nchunk[3]) {
    const int ty = 256 / tx;
    blocks[0] = ((n[0] + tx - 1) / tx) * (int)(((long long)n[1] * n[2] + ty - 1) / ty);
    nchunk[0] = 0;
    for (int d = 1; d < 3; ++d) {
        const int wd = d == 1 ? 2 : 1;
        const long long cols = (long long)n[0] * n[wd];
        nchunk[d] = (int)((cols + 255) / 256);
        blocks[d] = nchunk[d] * ((n[d] + seg[d] - 1) / seg[d]);
    }
}

static unsigned elementwise_blocks(long long n) {
    long long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <class T>
hipError_t launch_combine(const SweepArgs<T>& a, hipStream_t s) {
    combine_zero_L<T><<<elementwise_blocks(a.fstride), 256, 0, s>>>(a);
    return hipGetLastError();
}

template <class T>
hipError_t launch_set_fields(T* state, const double* src, int kind, long long n, int eos, double gm1,
                             hipStream_t s) {
    set_fields_kernel<T><<<elementwise_blocks(n), 256, 0, s>>>(state, src, kind, n, eos, gm1);
    return hipGetLastError();
}

template <class T>
hipError_t launch_get_fields(const T* state, double* dst, int kind, long long n, unsigned* clamps,
                             int eos, double gm1, hipStream_t s) {
    get_fields_kernel<T><<<elementwise_blocks(n), 256, 0, s>>>(state, dst, kind, n, clamps, eos, gm1);
    return hipGetLastError();
}

template <class T>
hipError_t launch_totals(const T* state, long long n, double* partials, int nblk, double* out,
                         hipStream_t s) {
    totals_pass1<T><<<nblk, 256, 0, s>>>(state, n, partials, nblk);
    totals_pass2<<<1, 256, 0, s>>>(partials, nblk, out);
    return hipGetLastError();
}

#define RH_INSTANTIATE(T)                                                                         \
    template hipError_t launch_sweep<T>(int, int, const SweepArgs<T>&, hipStream_t);               \
    template hipError_t launch_combine<T>(const SweepArgs<T>&, hipStream_t);                       \
    template hipError_t launch_set_fields<T>(T*, const double*, int, long long, int, double,       \
                                             hipStream_t);                                         \
    template hipError_t launch_get_fields<T>(const T*, double*, int, long long, unsigned*, int,    \
                                             double, hipStream_t);                                 \
    template hipError_t launch_totals<T>(const T*, long long, double*, int, double*, hipStream_t); \
    template hipError_t launch_sweep_batch<T>(int, int, int, const BatchArgs<T>&, int, hipStream_t); \
    template hipError_t launch_sweep_xy<T>(int, SweepArgs<T>, T, hipStream_t);

RH_INSTANTIATE(float)
RH_INSTANTIATE(double)

}  // namespace rh
