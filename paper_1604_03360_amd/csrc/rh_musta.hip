// rh_musta.hip -- the MUSTA-FORCE scheme (Sikorski et al., arXiv:1604.03360,
// Sec. 1.1) as one launch per SSP-RK3 stage for gfx950.
//
// The face flux of Eq. (2) is MUSTA on the first-order centred (FORCE) flux:
// MUSCL gives the states on both sides of the face from limited linear slopes
// of the conserved variables (cells i-1 .. i+2 for face i+1/2), then k stages
// each evaluate FORCE = (f_L + 2 f(u_M) + f_R)/4 - (u_R - u_L)/(4 lam) with the
// Richtmyer state u_M = (u_L + u_R)/2 - lam/2 (f_R - f_L), and every stage but
// the last opens the local Riemann fan by one local step on each side:
// u_L -= lam (F - f_L), u_R -= lam (f_R - F).  Every physical flux needs a
// primitive recovery (FP64), three per stage, so the face work is much larger
// than the four cells it reads.
//
// Work items are (grid, x-y tile of 16 x 15 cells, z segment), one block of
// 256 lanes each.  A plane of the tile is staged in LDS with two halo cells
// along x and along y; then the block computes the tile's 17 x 15 x faces (255
// lanes) and 16 x 16 y faces (256 lanes), one face per lane in each round, and
// every lane of a cell column computes the z face above it from a register
// window of four planes.  So every face of the grid is computed once per stage,
// apart from the tile-edge faces, which both tiles compute.  The flux
// difference is summed x, y, z and the stage combine is applied in place of
// storing L.  Axes of one cell contribute nothing.
#include "rh_internal.hpp"
#include "../../include/rh.h"

namespace rh {

namespace {

constexpr int TX = kMustaTX, TY = kMustaTY;
constexpr int G = 2;                 // ghost cells per side (MUSCL slopes of the end faces)
constexpr int SX = TX + 2 * G, SY = TY + 2 * G;

// Limiter and stage count of a kernel instance: fixed at compile time for the
// default scheme (minmod, two stages: straight-line face code), read from the
// grid entry otherwise.
constexpr int kAnyLimiter = -1, kAnyStages = 0;

// Limited MUSCL slope from the one-sided differences a, b (zero where they
// differ in sign): minmod, MC, van Leer, superbee, or none.
template <class T, int LIM>
__device__ __forceinline__ T limited_slope(int rt_lim, T a, T b) {
    const int lim = LIM == kAnyLimiter ? rt_lim : LIM;
    if (lim == RH_LIMITER_NONE) return (T)0;
    if (!((a > (T)0 && b > (T)0) || (a < (T)0 && b < (T)0))) return (T)0;
    const T aa = fabs(a), ab = fabs(b);
    T m;
    if (lim == RH_LIMITER_MINMOD) m = min(aa, ab);
    else if (lim == RH_LIMITER_MC) m = min(min((T)2 * aa, (T)2 * ab), (T)0.5 * (aa + ab));
    else if (lim == RH_LIMITER_VANLEER) return (T)2 * a * b / (a + b);
    else m = max(min((T)2 * aa, ab), min(aa, (T)2 * ab));
    return a > (T)0 ? m : -m;
}

// Physical flux along DIR of a state (FP64 recovery for the fluid of EOS).
template <class T, int DIR, int EOS>
__device__ __forceinline__ void phys_flux(const T u[5], double gm1, T f[5], unsigned& cl) {
    double vd, p;
    if constexpr (EOS == EOS_CONFORMAL) {
        recover_vp<DIR>((double)u[0], (double)u[1], (double)u[2], (double)u[3], vd, p, cl);
    } else {
        double kap, Mxs, Mys, Mzs, e;
        recover_ideal((double)u[0], (double)u[1], (double)u[2], (double)u[3], (double)u[4], gm1, kap,
                      Mxs, Mys, Mzs, p, e, cl);
        vd = kap * (DIR == 0 ? Mxs : (DIR == 1 ? Mys : Mzs));
    }
    const T v = (T)vd, P = (T)p;
    f[0] = u[1 + DIR];
    f[1] = u[1] * v + (DIR == 0 ? P : (T)0);
    f[2] = u[2] * v + (DIR == 1 ? P : (T)0);
    f[3] = u[3] * v + (DIR == 2 ? P : (T)0);
    f[4] = u[4] * v;
}

// MUSCL + MUSTA flux of face i+1/2 from the cells i-1 .. i+2 (a, b, c, d).
template <class T, int DIR, int EOS, int LIM, int MK>
__device__ __forceinline__ void musta_face(const T a[5], const T b[5], const T c[5], const T d[5],
                                           const StageGrid<T>& Gr, T F[5], unsigned& cl) {
    T uL[5], uR[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const T si = limited_slope<T, LIM>(Gr.limiter, b[q] - a[q], c[q] - b[q]);
        const T sj = limited_slope<T, LIM>(Gr.limiter, c[q] - b[q], d[q] - c[q]);
        uL[q] = b[q] + (T)0.5 * si;
        uR[q] = c[q] - (T)0.5 * sj;
    }
    const T lam = Gr.lam, hlam = (T)0.5 * Gr.lam, q4 = (T)1 / ((T)4 * Gr.lam);
    const int mk = MK == kAnyStages ? Gr.mk : MK;
    constexpr int kUnroll = MK == kAnyStages ? 1 : MK;
#pragma unroll kUnroll
    for (int st = 1; st <= mk; ++st) {
        T fL[5], fR[5], uM[5], fM[5];
        phys_flux<T, DIR, EOS>(uL, Gr.gm1, fL, cl);
        phys_flux<T, DIR, EOS>(uR, Gr.gm1, fR, cl);
#pragma unroll
        for (int q = 0; q < 5; ++q) uM[q] = (T)0.5 * (uL[q] + uR[q]) - hlam * (fR[q] - fL[q]);
        phys_flux<T, DIR, EOS>(uM, Gr.gm1, fM, cl);
#pragma unroll
        for (int q = 0; q < 5; ++q) F[q] = (T)0.25 * (fL[q] + (T)2 * fM[q] + fR[q]) - (uR[q] - uL[q]) * q4;
        if (st < mk) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                uL[q] = uL[q] - lam * (F[q] - fL[q]);
                uR[q] = uR[q] - lam * (fR[q] - F[q]);
            }
        }
    }
}

}  // namespace

template <class T>
struct MustaMinBlocks {
    static constexpr int value = sizeof(T) == 4 ? 2 : 1;
};

template <class T, bool HUB, int EOS, int LIM, int MK>
__global__ void __launch_bounds__(256, (MustaMinBlocks<T>::value)) stage_musta(StageArgs<T> A) {
    __shared__ T su[5][SY][SX];           // staged plane: rows -2 .. TY+1, columns -2 .. TX+1
    __shared__ T fxs[5][TY][TX + 1];      // x faces: column f = face between tile columns f-1 and f
    __shared__ T fys[5][TY + 1][TX];      // y faces: row f = face between tile rows f-1 and f

    const int b = xcd_logical((int)blockIdx.x, (int)gridDim.x);
    const StageGrid<T> Gr = A.ngrid > 0 ? A.grids[stage_grid_of(A, b)] : A.one;
    const int lb = b - Gr.blk0;
    const int tpp = Gr.ntx * Gr.nty;
    const int zsg = lb / tpp, rem = lb - zsg * tpp;
    const int tyi = rem / Gr.ntx, txi = rem - tyi * Gr.ntx;
    const int nx = Gr.n[0], ny = Gr.n[1], nz = Gr.n[2];
    const int x0 = txi * TX, y0 = tyi * TY;
    const int xa = min(TX, nx - x0), ya = min(TY, ny - y0);
    const int k0 = zsg * Gr.seg, kend = min(k0 + Gr.seg, nz);
    const long long F = (long long)nx * ny * nz;
    const T* us = A.us + Gr.off;
    const T* u0 = A.u0 + Gr.off;
    T* out = A.out + Gr.off;
    const double t = A.t;
    const bool dox = nx > 1, doy = ny > 1, doz = nz > 1;

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;          // cell column of this lane (ly < TY for tid < 240)
    const bool act = ly < ya && lx < xa;
    const int cx = x0 + min(lx, xa - 1), cy = y0 + min(min(ly, TY - 1), ya - 1);
    const uint32_t sb = (uint32_t)sizeof(T) * (uint32_t)nx * (uint32_t)ny;
    const uint32_t cb = (uint32_t)sizeof(T) * ((uint32_t)cx + (uint32_t)nx * (uint32_t)cy);

    // halo job: x-halo cells (4 per row: columns -2, -1, xa, xa+1), then y-halo
    // cells (4 per column: rows -2, -1, ya, ya+1); staged indices are offset by 2
    const int nxh = 4 * ya, nyh = 4 * xa;
    int hkind = 0, hr = 0, hc = 0;
    if (tid < nxh) {
        const int j = tid & 3;
        hkind = 1;
        hr = tid >> 2;                      // tile row
        hc = j < 2 ? j - 2 : xa + j - 2;    // tile column
    } else if (tid < nxh + nyh) {
        const int s = tid - nxh, j = s & 3;
        hkind = 2;
        hc = s >> 2;
        hr = j < 2 ? j - 2 : ya + j - 2;
    }

    auto fetch_own = [&](int m, T u[5]) {
        if (m >= 0 && m < nz) {
            const uint32_t off = cb + (uint32_t)m * sb;
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = ld_off(us + f * F, off);
        } else {
            stage_load<T, HUB>(Gr, us, F, t, cx, cy, m, u);
        }
    };
    auto fetch_halo = [&](int m, T u[5]) {
        if (hkind) stage_load<T, HUB>(Gr, us, F, t, x0 + hc, y0 + hr, m, u);
    };

    const T ihx = Gr.inv_h[0], ihy = Gr.inv_h[1], ihz = Gr.inv_h[2];
    unsigned clamped = 0;

    T zw[4][5];                // planes m-3 .. m of this column
    T ring[3][5];              // x + y part of L of planes m-2, m-1, m
    T Fzl[5];                  // z face below the next cell to finish
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        Fzl[c] = (T)0;
#pragma unroll
        for (int j = 0; j < 4; ++j) zw[j][c] = (T)0;
#pragma unroll
        for (int j = 0; j < 3; ++j) ring[j][c] = (T)0;
    }

    const int mlo = k0 - G, mhi = kend + G - 1;
    T nu[5], nh[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
    fetch_own(mlo, nu);
    if (mlo >= k0) fetch_halo(mlo, nh);
    for (int m = mlo; m <= mhi; ++m) {
        const bool owned = m >= k0 && m < kend;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
            for (int j = 0; j < 3; ++j) zw[j][c] = zw[j + 1][c];
            zw[3][c] = nu[c];
        }
        T hu[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) hu[c] = nh[c];
        if (m + 1 <= mhi) fetch_own(m + 1, nu);
        if (m + 1 >= k0 && m + 1 < kend) fetch_halo(m + 1, nh);

        if (owned) {
            if (tid < TX * TY && act) {
#pragma unroll
                for (int c = 0; c < 5; ++c) su[c][ly + G][lx + G] = zw[3][c];
            }
            if (hkind) {
#pragma unroll
                for (int c = 0; c < 5; ++c) su[c][hr + G][hc + G] = hu[c];
            }
            __syncthreads();
            // x faces: job tid -> row r, face f (between tile columns f-1 and f)
            if (dox && tid < (TX + 1) * TY) {
                const int r = tid / (TX + 1), f = tid - r * (TX + 1);
                if (r < ya && f <= xa) {
                    T a[5], bb[5], c2[5], d[5], Fx[5];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        a[c] = su[c][r + G][f];
                        bb[c] = su[c][r + G][f + 1];
                        c2[c] = su[c][r + G][f + 2];
                        d[c] = su[c][r + G][f + 3];
                    }
                    unsigned cl = 0;
                    musta_face<T, 0, EOS, LIM, MK>(a, bb, c2, d, Gr, Fx, cl);
                    if (f > 0 || x0 == 0) clamped += cl;   // each face of the grid counted once
#pragma unroll
                    for (int c = 0; c < 5; ++c) fxs[c][r][f] = Fx[c];
                }
            }
            // y faces: job tid -> column c, face f (between tile rows f-1 and f)
            if (doy) {
                const int col = tid % TX, f = tid / TX;
                if (col < xa && f <= ya) {
                    T a[5], bb[5], c2[5], d[5], Fy[5];
#pragma unroll
                    for (int c = 0; c < 5; ++c) {
                        a[c] = su[c][f][col + G];
                        bb[c] = su[c][f + 1][col + G];
                        c2[c] = su[c][f + 2][col + G];
                        d[c] = su[c][f + 3][col + G];
                    }
                    unsigned cl = 0;
                    musta_face<T, 1, EOS, LIM, MK>(a, bb, c2, d, Gr, Fy, cl);
                    if (f > 0 || y0 == 0) clamped += cl;
#pragma unroll
                    for (int c = 0; c < 5; ++c) fys[c][f][col] = Fy[c];
                }
            }
            __syncthreads();
            if (act) {
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const T Lx = dox ? (fxs[c][ly][lx] - fxs[c][ly][lx + 1]) * ihx : (T)0;
                    const T Ly = doy ? (fys[c][ly][lx] - fys[c][ly + 1][lx]) * ihy : (T)0;
                    ring[2][c] = Lx + Ly;
                }
            }
        }
        // z face between planes m-2 and m-1 (cells m-3 .. m), for faces k0-1/2 .. kend-1/2
        if (m >= k0 + 1) {
            T Fz[5];
            if (doz) {
                unsigned cl = 0;
                musta_face<T, 2, EOS, LIM, MK>(zw[0], zw[1], zw[2], zw[3], Gr, Fz, cl);
                if (act && (m - 2 >= k0 || k0 == 0)) clamped += cl;
            } else {
#pragma unroll
                for (int c = 0; c < 5; ++c) Fz[c] = (T)0;
            }
            if (m >= k0 + 2) {
                // cell k = m - 2 is complete: its stage input is zw[1]
                const int k = m - 2;
                const uint32_t off = cb + (uint32_t)k * sb;
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const T L = ring[0][c] + (doz ? (Fzl[c] - Fz[c]) * ihz : (T)0);
                    T v;
                    if (A.stage == STAGE_WRITE_L) {
                        v = L;
                    } else {
                        v = zw[1][c] + A.dt * L;
                        if (A.stage == STAGE_2) v = (T)0.75 * ld_off(u0 + c * F, off) + (T)0.25 * v;
                        else if (A.stage == STAGE_3) v = rk3_last(ld_off(u0 + c * F, off), v);
                    }
                    if (act) st_off(out + c * F, off, v);
                }
            }
#pragma unroll
            for (int c = 0; c < 5; ++c) Fzl[c] = Fz[c];
        }
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            ring[0][c] = ring[1][c];
            ring[1][c] = ring[2][c];
        }
    }
    if (clamped) atomicAdd(A.clamps, clamped);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int musta_default_segment(const int n[3]) {
    // about 4096 blocks (several resident blocks per CU on 256 CUs), segments
    // of 8 to 64 planes (each segment re-enters 2G = 4 halo planes)
    const long long tiles = (long long)((n[0] + TX - 1) / TX) * ((n[1] + TY - 1) / TY);
    const long long target = 4096;
    long long nseg = (target + tiles - 1) / tiles;
    const long long max_seg = (n[2] + 7) / 8;
    if (nseg > max_seg) nseg = max_seg;
    if (nseg < 1) nseg = 1;
    int seg = (int)((n[2] + nseg - 1) / nseg);
    if (seg > 64) seg = 64;
    return seg;
}

template <class T>
void musta_shape(StageGrid<T>& g, int seg) {
    if (seg < 1) seg = 1;
    if (seg > g.n[2]) seg = g.n[2];
    g.ntx = (g.n[0] + TX - 1) / TX;
    g.nty = (g.n[1] + TY - 1) / TY;
    g.seg = seg;
    g.nseg = (g.n[2] + seg - 1) / seg;
}

template <class T, int LIM, int MK>
hipError_t launch_musta_t(bool hub, int eos, const StageArgs<T>& a, const dim3 grid, hipStream_t s) {
    if (eos == EOS_CONFORMAL) {
        if (hub) stage_musta<T, true, EOS_CONFORMAL, LIM, MK><<<grid, 256, 0, s>>>(a);
        else stage_musta<T, false, EOS_CONFORMAL, LIM, MK><<<grid, 256, 0, s>>>(a);
    } else if (eos == EOS_IDEAL && !hub) {
        stage_musta<T, false, EOS_IDEAL, LIM, MK><<<grid, 256, 0, s>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class T>
hipError_t launch_musta(bool hub, int eos, int limiter, int mk, const StageArgs<T>& a, long long nblocks,
                        hipStream_t s) {
    if (nblocks <= 0 || nblocks > 0x7fffffffLL || mk < 1) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nblocks);
    if (limiter == RH_LIMITER_MINMOD && mk == 2)
        return launch_musta_t<T, RH_LIMITER_MINMOD, 2>(hub, eos, a, grid, s);
    return launch_musta_t<T, kAnyLimiter, kAnyStages>(hub, eos, a, grid, s);
}

template void musta_shape<float>(StageGrid<float>&, int);
template void musta_shape<double>(StageGrid<double>&, int);
template hipError_t launch_musta<float>(bool, int, int, int, const StageArgs<float>&, long long, hipStream_t);
template hipError_t launch_musta<double>(bool, int, int, int, const StageArgs<double>&, long long, hipStream_t);

}  // namespace rh
