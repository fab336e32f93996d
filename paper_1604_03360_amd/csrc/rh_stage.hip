// rh_stage.hip -- one launch per SSP-RK3 stage for gfx950.
//
// stage_fused evaluates the whole operator L(u) of Eq. (2) (Sikorski et al.,
// arXiv:1604.03360) -- the x, y and z flux differences -- and applies the
// Runge-Kutta stage combine (Sec. 1) in a single launch, with no L accumulator
// in memory.  A work item is (grid, x-y tile of TX x TY = 256 cells, z segment):
// the block rolls along its z segment one plane at a time.  Each lane owns one
// (x, y) column of the tile and keeps a register window of 2R doubled split
// fluxes along z (as the rolling sweeps do); for every owned plane the block
// stages the tile's doubled x and y split fluxes in LDS, with R halo cells on
// each side along x and along y (no corners are needed), reconstructs every x
// and y face of the tile once and keeps the x + y part of L for R planes until
// the z face above the cell is known.  Every cell of the tile is loaded and
// recovered (FP64) once per plane; the halo cells of the tile are recovered
// again by the tiles that own them.
//
// The arithmetic of every face, flux difference and combine is that of the
// split sweeps, summed in the same order (x, then y, then z), so the result is
// bitwise that of the x, y and z sweeps run one after another.
//
// Ensembles use the same kernel: each block finds its grid in a table sorted
// by first block, so one launch covers every grid of the batch.
//
// Two generalisations of the flux step are instantiated here as well: local
// Lax-Friedrichs splitting (LOCAL: the block stages the physical flux and the
// state of each cell with its largest characteristic speed, and every face
// reconstructs F +- alpha u with alpha the largest speed of its 2R stencil
// cells), and the ideal-gas equation of state (EOS_IDEAL: a recovery pass
// solves for every cell's velocity and pressure once per evaluation of L, and
// the stage reads them with the state).  An axis of one cell contributes
// nothing to L.
#include "rh_internal.hpp"
#include "../../include/rh.h"

namespace rh {

namespace {

// One reconstruction from a window of 2R doubled split fluxes of cells
// i - R + 1 .. i + R (interface i + 1/2): plus = left-biased on f+, minus =
// mirrored on f-.  eps2 is the epsilon of the doubled data (4 eps); WENO5
// carries its smoothness indicators as 4 beta and takes 4 eps2.
template <class T, int ORDER>
__device__ __forceinline__ T stage_recon_plus(const T* w, T eps2) {
    if constexpr (ORDER == 5) return weno5<T>(w[0], w[1], w[2], w[3], w[4], (T)4 * eps2);
    else return weno7<T>(w[0], w[1], w[2], w[3], w[4], w[5], w[6], eps2);
}
template <class T, int ORDER>
__device__ __forceinline__ T stage_recon_minus(const T* w, T eps2) {
    if constexpr (ORDER == 5) return weno5<T>(w[5], w[4], w[3], w[2], w[1], (T)4 * eps2);
    else return weno7<T>(w[7], w[6], w[5], w[4], w[3], w[2], w[1], eps2);
}

}  // namespace

// Minimum resident blocks per CU (= waves per SIMD) for the register budget;
// FP64 blocks other than WENO5 16 x 16 with global splitting need more than
// half of the 160 KB LDS.
template <class T, int ORDER, int TX, bool LOCAL>
struct StageMinBlocks {
    static constexpr int value = sizeof(T) == 4 ? 3 : (ORDER == 5 && TX == 16 && !LOCAL ? 2 : 1);
};

// One face from the staged pairs of its 2R stencil cells: global splitting
// stages (F + u, F - u) and reconstructs them directly; local splitting stages
// (F, u) and reconstructs F +- alpha u with alpha the largest speed of the 2R
// cells.
template <class T, int ORDER>
__device__ __forceinline__ T recon_local(const T* wa, const T* wb, T alpha, T eps2) {
    constexpr int W = ORDER + 1;
    T wp[W], wm[W];
#pragma unroll
    for (int j = 0; j < W; ++j) {
        wp[j] = wa[j] + alpha * wb[j];
        wm[j] = wa[j] - alpha * wb[j];
    }
    return stage_recon_plus<T, ORDER>(wp, eps2) + stage_recon_minus<T, ORDER>(wm, eps2);
}

template <class T, int DIR, bool LOCAL>
__device__ __forceinline__ void stage_pair(const T u[5], T v, T P, T a[5], T b[5]) {
    if constexpr (LOCAL) {
        a[0] = u[1 + DIR];
        a[1] = u[1] * v + (DIR == 0 ? P : (T)0);
        a[2] = u[2] * v + (DIR == 1 ? P : (T)0);
        a[3] = u[3] * v + (DIR == 2 ? P : (T)0);
        a[4] = u[4] * v;
#pragma unroll
        for (int c = 0; c < 5; ++c) b[c] = u[c];
    } else {
        split_flux_vp<T, DIR>(u, v, P, a, b);
    }
}

template <class T, int ORDER, int TX, bool HUB, bool LOCAL, int EOS>
__global__ void __launch_bounds__(256, (StageMinBlocks<T, ORDER, TX, LOCAL>::value)) stage_fused(StageArgs<T> A) {
    constexpr int R = (ORDER + 1) / 2, W = 2 * R, TY = 256 / TX;
    static_assert(W * (TX + TY) <= 256, "one halo cell per lane and plane");
    static_assert(5 * (TX + TY) <= 256, "one edge face (all components) per lane");
    constexpr int SX = TX + 2 * R;            // staged x row: R ghosts, TX cells, R ghosts
    constexpr int SY = TY + 2 * R;
    constexpr int SPX = LOCAL ? TY : 1, SPY = LOCAL ? SY : 1;
    __shared__ T sx[2][5][TY][SX];            // doubled x split fluxes (plus, minus), or (F, u) with LOCAL
    __shared__ T sy[2][5][SY][TX];            // the same along y
    __shared__ T ssx[SPX][LOCAL ? SX : 1];    // LOCAL: largest speed along x of the staged cells
    __shared__ T ssy[SPY][LOCAL ? TX : 1];    // LOCAL: largest speed along y
    __shared__ T fx[5][TY][TX + 1];           // x face fluxes: column 0 = left face of the tile, 1 + i = right face of cell i
    __shared__ T fy[5][TY + 1][TX];           // y face fluxes: row 0 = lower face of the tile, 1 + j = upper face of row j

    const int b = xcd_logical((int)blockIdx.x, (int)gridDim.x);
    const StageGrid<T> G = A.ngrid > 0 ? A.grids[stage_grid_of(A, b)] : A.one;
    const int lb = b - G.blk0;
    const int tpp = G.ntx * G.nty;
    const int zs = lb / tpp, rem = lb - zs * tpp;
    const int tyi = rem / G.ntx, txi = rem - tyi * G.ntx;
    const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
    const int x0 = txi * TX, y0 = tyi * TY;
    const int xa = min(TX, nx - x0), ya = min(TY, ny - y0);
    const int k0 = zs * G.seg, kend = min(k0 + G.seg, nz);
    const long long F = (long long)nx * ny * nz;
    const T* us = A.us + G.off;
    const T* u0 = A.u0 + G.off;
    T* out = A.out + G.off;
    const double t = A.t;
    // an axis of one cell contributes nothing to L
    const bool dox = nx > 1, doy = ny > 1, doz = nz > 1;

    const int tid = threadIdx.x, lx = tid % TX, ly = tid / TX;
    const bool act = lx < xa && ly < ya;
    // lanes outside a ragged tile follow the loop on a valid cell and store nothing
    const int cx = x0 + min(lx, xa - 1), cy = y0 + min(ly, ya - 1);
    const uint32_t sb = (uint32_t)sizeof(T) * (uint32_t)nx * (uint32_t)ny;   // z plane, bytes
    const uint32_t cb = (uint32_t)sizeof(T) * ((uint32_t)cx + (uint32_t)nx * (uint32_t)cy);

    // halo job of this lane: one x-halo cell (row r, staged column p; cell x0 - R + p)
    // or one y-halo cell (column c, staged row q; cell y0 - R + q), the same every plane
    const int nxh = W * ya, nyh = W * xa;
    int hkind = 0, hr = 0, hc = 0, hxc = 0, hyc = 0;
    if (tid < nxh) {
        const int j = tid % W;
        hkind = 1;
        hr = tid / W;
        hc = j < R ? j : xa + j;
        hxc = x0 - R + hc;
        hyc = y0 + hr;
    } else if (tid < nxh + nyh) {
        const int s = tid - nxh, j = s % W;
        hkind = 2;
        hc = s / W;
        hr = j < R ? j : ya + j;
        hxc = x0 + hc;
        hyc = y0 - R + hr;
    }

    auto fetch_own = [&](int m, T u[5]) {
        if (m >= 0 && m < nz) {
            const uint32_t off = cb + (uint32_t)m * sb;
#pragma unroll
            for (int f = 0; f < 5; ++f) u[f] = ld_off(us + f * F, off);
        } else {
            stage_load<T, HUB>(G, us, F, t, cx, cy, m, u);
        }
    };
    auto fetch_halo = [&](int m, T u[5]) {
        if (hkind) stage_load<T, HUB>(G, us, F, t, hxc, hyc, m, u);
    };
    // ideal gas: the recovery pass's (vx, vy, vz, p, c_s^2) of the same cells
    const T* pr = EOS == EOS_IDEAL ? A.prim + G.off : nullptr;
    auto fetch_own_prim = [&](int m, T q[5]) {
        if constexpr (EOS == EOS_IDEAL) stage_load<T, false>(G, pr, F, t, cx, cy, m, q);
    };
    auto fetch_halo_prim = [&](int m, T q[5]) {
        if constexpr (EOS == EOS_IDEAL) {
            if (hkind) stage_load<T, false>(G, pr, F, t, hxc, hyc, m, q);
        }
    };

    const T eps2 = (T)4 * G.eps;   // epsilon of the doubled split fluxes
    const T hxinv = (T)0.5 * G.inv_h[0], hyinv = (T)0.5 * G.inv_h[1], hzinv = (T)0.5 * G.inv_h[2];
    unsigned clamped = 0;

    T zp[5][W], zm[5][W];     // z window: staged pairs of cells k - R .. k + R - 1
    T zsp[LOCAL ? W : 1];     // LOCAL: their largest speeds along z
    T ring[R][5];             // x + y part of L of the last R owned planes, oldest first
#pragma unroll
    for (int c = 0; c < 5; ++c) {
#pragma unroll
        for (int j = 0; j < W; ++j) zp[c][j] = zm[c][j] = (T)0;
#pragma unroll
        for (int j = 0; j < R; ++j) ring[j][c] = (T)0;
    }
#pragma unroll
    for (int j = 0; j < (LOCAL ? W : 1); ++j) zsp[j] = (T)0;

    // Enter plane m: recover the own cell, shift its z split fluxes into the
    // window and, for an owned plane, stage the x / y split fluxes of the own
    // and halo cells.
    auto enter = [&](int m, const T u[5], const T hu[5], bool owned) {
        // velocity, pressure (and, for the local splitting, v^2 and c_s^2) of the
        // own cell: FP64 closed-form recovery, or read from the recovery pass
        // (loaded here, not a plane ahead: the registers of a prefetch spill)
        T VX, VY, VZ, P;
        double vxd, vyd, vzd, v2 = 0.0, cs2 = 0.0;
        unsigned c0 = 0;
        if constexpr (EOS == EOS_IDEAL) {
            T pu[5];
            fetch_own_prim(m, pu);
            VX = pu[0];
            VY = pu[1];
            VZ = pu[2];
            P = pu[3];
            vxd = (double)VX;
            vyd = (double)VY;
            vzd = (double)VZ;
            if constexpr (LOCAL) {
                v2 = vxd * vxd + vyd * vyd + vzd * vzd;
                cs2 = (double)pu[4];
            }
        } else {
            double kap, Mxs, Mys, Mzs, p;
            recover_kp3((double)u[0], (double)u[1], (double)u[2], (double)u[3], kap, Mxs, Mys, Mzs, p, c0);
            vxd = kap * Mxs;
            vyd = kap * Mys;
            vzd = kap * Mzs;
            VX = (T)vxd;
            VY = (T)vyd;
            VZ = (T)vzd;
            P = (T)p;
            cs2 = 1.0 / 3.0;
            if constexpr (LOCAL) v2 = kap * kap * (Mxs * Mxs + Mys * Mys + Mzs * Mzs);
        }
        T fp[5], fm[5];
        stage_pair<T, 2, LOCAL>(u, VZ, P, fp, fm);
#pragma unroll
        for (int c = 0; c < 5; ++c) {
#pragma unroll
            for (int j = 0; j < W - 1; ++j) {
                zp[c][j] = zp[c][j + 1];
                zm[c][j] = zm[c][j + 1];
            }
            zp[c][W - 1] = fp[c];
            zm[c][W - 1] = fm[c];
        }
        if constexpr (LOCAL) {
#pragma unroll
            for (int j = 0; j < W - 1; ++j) zsp[j] = zsp[j + 1];
            zsp[W - 1] = (T)max_char_speed(vzd, v2, cs2);
        }
        if (!owned) return;
        if (act) {
            clamped += c0;   // floors counted once per owned cell and evaluation of L
            stage_pair<T, 0, LOCAL>(u, VX, P, fp, fm);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                sx[0][c][ly][R + lx] = fp[c];
                sx[1][c][ly][R + lx] = fm[c];
            }
            stage_pair<T, 1, LOCAL>(u, VY, P, fp, fm);
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                sy[0][c][R + ly][lx] = fp[c];
                sy[1][c][R + ly][lx] = fm[c];
            }
            if constexpr (LOCAL) {
                ssx[ly][R + lx] = (T)max_char_speed(vxd, v2, cs2);
                ssy[R + ly][lx] = (T)max_char_speed(vyd, v2, cs2);
            }
        }
        if (hkind) {
            T HX, HY, HP;
            double hxd, hyd, hv2 = 0.0, hcs2 = 0.0;
            if constexpr (EOS == EOS_IDEAL) {
                T phu[5];
                fetch_halo_prim(m, phu);
                HX = phu[0];
                HY = phu[1];
                HP = phu[3];
                hxd = (double)HX;
                hyd = (double)HY;
                if constexpr (LOCAL) {
                    const double hzd = (double)phu[2];
                    hv2 = hxd * hxd + hyd * hyd + hzd * hzd;
                    hcs2 = (double)phu[4];
                }
            } else {
                double hk, hMx, hMy, hp;
                unsigned hcl = 0;
                if constexpr (!LOCAL) {
                    recover_kp((double)hu[0], (double)hu[1], (double)hu[2], (double)hu[3], hk, hMx, hMy, hp, hcl);
                } else {
                    double hMz;
                    recover_kp3((double)hu[0], (double)hu[1], (double)hu[2], (double)hu[3], hk, hMx, hMy, hMz, hp,
                                hcl);
                    hv2 = hk * hk * (hMx * hMx + hMy * hMy + hMz * hMz);
                    hcs2 = 1.0 / 3.0;
                }
                hxd = hk * hMx;
                hyd = hk * hMy;
                HX = (T)hxd;
                HY = (T)hyd;
                HP = (T)hp;
            }
            if (hkind == 1) {
                stage_pair<T, 0, LOCAL>(hu, HX, HP, fp, fm);
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    sx[0][c][hr][hc] = fp[c];
                    sx[1][c][hr][hc] = fm[c];
                }
                if constexpr (LOCAL) ssx[hr][hc] = (T)max_char_speed(hxd, hv2, hcs2);
            } else {
                stage_pair<T, 1, LOCAL>(hu, HY, HP, fp, fm);
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    sy[0][c][hr][hc] = fp[c];
                    sy[1][c][hr][hc] = fm[c];
                }
                if constexpr (LOCAL) ssy[hr][hc] = (T)max_char_speed(hyd, hv2, hcs2);
            }
        }
    };

    // x + y part of L of the staged (owned) plane, pushed into the ring
    auto plane_xy = [&]() {
        __syncthreads();
        if (act) {
            T ax = (T)0, ay = (T)0;
            if constexpr (LOCAL) {
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    ax = max(ax, ssx[ly][lx + 1 + j]);
                    ay = max(ay, ssy[ly + 1 + j][lx]);
                }
            }
            // one component at a time: unrolled, the LDS reads of all five
            // windows would be hoisted and raise the register peak
#pragma unroll 1
            for (int c = 0; c < 5; ++c) {
                // window of face x + 1/2: staged columns lx + 1 .. lx + 2R
                if constexpr (LOCAL) {
                    T wa[W], wb[W];
#pragma unroll
                    for (int j = 0; j < W; ++j) {
                        wa[j] = sx[0][c][ly][lx + 1 + j];
                        wb[j] = sx[1][c][ly][lx + 1 + j];
                    }
                    fx[c][ly][lx + 1] = recon_local<T, ORDER>(wa, wb, ax, eps2);
                } else {
                    fx[c][ly][lx + 1] = stage_recon_plus<T, ORDER>(&sx[0][c][ly][lx + 1], eps2) +
                                        stage_recon_minus<T, ORDER>(&sx[1][c][ly][lx + 1], eps2);
                }
                T wp[W], wm[W];
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    wp[j] = sy[0][c][ly + 1 + j][lx];
                    wm[j] = sy[1][c][ly + 1 + j][lx];
                }
                if constexpr (LOCAL) fy[c][ly + 1][lx] = recon_local<T, ORDER>(wp, wm, ay, eps2);
                else fy[c][ly + 1][lx] = stage_recon_plus<T, ORDER>(wp, eps2) + stage_recon_minus<T, ORDER>(wm, eps2);
            }
        }
        // faces on the lower edges of the tile, one (line, component) per lane:
        // 5 ya x jobs (window at staged column 0), then 5 xa y jobs (staged row 0)
        if (tid < 5 * ya) {
            const int r = tid / 5, c = tid - 5 * r;
            if constexpr (LOCAL) {
                T wa[W], wb[W], al = (T)0;
#pragma unroll
                for (int j = 0; j < W; ++j) {
                    wa[j] = sx[0][c][r][j];
                    wb[j] = sx[1][c][r][j];
                    al = max(al, ssx[r][j]);
                }
                fx[c][r][0] = recon_local<T, ORDER>(wa, wb, al, eps2);
            } else {
                fx[c][r][0] = stage_recon_plus<T, ORDER>(&sx[0][c][r][0], eps2) +
                              stage_recon_minus<T, ORDER>(&sx[1][c][r][0], eps2);
            }
        } else if (tid < 5 * (ya + xa)) {
            const int s = tid - 5 * ya, col = s / 5, c = s - 5 * col;
            T wp[W], wm[W];
#pragma unroll
            for (int j = 0; j < W; ++j) {
                wp[j] = sy[0][c][j][col];
                wm[j] = sy[1][c][j][col];
            }
            if constexpr (LOCAL) {
                T al = (T)0;
#pragma unroll
                for (int j = 0; j < W; ++j) al = max(al, ssy[j][col]);
                fy[c][0][col] = recon_local<T, ORDER>(wp, wm, al, eps2);
            } else {
                fy[c][0][col] = stage_recon_plus<T, ORDER>(wp, eps2) + stage_recon_minus<T, ORDER>(wm, eps2);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < R - 1; ++j)
#pragma unroll
            for (int c = 0; c < 5; ++c) ring[j][c] = ring[j + 1][c];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T Lx = dox ? (fx[c][ly][lx] - fx[c][ly][lx + 1]) * hxinv : (T)0;
            const T Ly = doy ? (fy[c][ly][lx] - fy[c][ly + 1][lx]) * hyinv : (T)0;
            ring[R - 1][c] = Lx + Ly;
        }
    };
    auto push_none = [&]() {
#pragma unroll
        for (int j = 0; j < R - 1; ++j)
#pragma unroll
            for (int c = 0; c < 5; ++c) ring[j][c] = ring[j + 1][c];
    };
    // z face above the window's centre, component c
    auto zface = [&](int c) {
        if constexpr (LOCAL) {
            T al = (T)0;
#pragma unroll
            for (int j = 0; j < W; ++j) al = max(al, zsp[j]);
            return recon_local<T, ORDER>(zp[c], zm[c], al, eps2);
        } else {
            return stage_recon_plus<T, ORDER>(zp[c], eps2) + stage_recon_minus<T, ORDER>(zm[c], eps2);
        }
    };

    // fill: planes k0 - R .. k0 + R - 1 (the z window of face k0 - 1/2)
    T nu[5], nh[5] = {(T)0, (T)0, (T)0, (T)0, (T)0};
    fetch_own(k0 - R, nu);
    for (int m = k0 - R; m < k0 + R; ++m) {
        T u[5], hu[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            u[f] = nu[f];
            hu[f] = nh[f];
        }
        const bool owned = m >= k0 && m < kend;
        fetch_own(m + 1, nu);
        if (m + 1 >= k0 && m + 1 < kend) fetch_halo(m + 1, nh);
        enter(m, u, hu, owned);
        if (owned) plane_xy();
        else if (m >= k0) push_none();
    }
    T Fl[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) Fl[c] = zface(c);

    // main loop: plane m = k + R enters, cell k is finished
    for (int k = k0; k < kend; ++k) {
        const int m = k + R;
        T u[5], hu[5];
#pragma unroll
        for (int f = 0; f < 5; ++f) {
            u[f] = nu[f];
            hu[f] = nh[f];
        }
        const bool owned = m < kend;
        if (k + 1 < kend) fetch_own(m + 1, nu);
        if (m + 1 < kend) fetch_halo(m + 1, nh);
        const uint32_t off = cb + (uint32_t)k * sb;
        enter(m, u, hu, owned);
        T Lk[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            // the z face is reconstructed for every grid (on ghost copies where nz is
            // 1) and discarded by a select, which keeps it out of a branch
            const T Fr = zface(c);
            const T Lz = doz ? (Fl[c] - Fr) * hzinv : (T)0;
            Fl[c] = Fr;
            Lk[c] = ring[0][c] + Lz;
        }
        // the stage input and u^n of cell k, loaded after the reconstructions
        // to keep them out of the register peak
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T L = Lk[c];
            const T usk = A.stage != STAGE_WRITE_L ? ld_off(us + c * F, off) : (T)0;
            const T u0k = A.stage >= STAGE_2 ? ld_off(u0 + c * F, off) : (T)0;
            T v;
            if (A.stage == STAGE_WRITE_L) {
                v = L;
            } else {
                v = usk + A.dt * L;
                if (A.stage == STAGE_2) v = (T)0.75 * u0k + (T)0.25 * v;
                else if (A.stage == STAGE_3) v = rk3_last(u0k, v);
            }
            if (act) st_off(out + c * F, off, v);
        }
        if (owned) plane_xy();
        else push_none();
    }
    if (clamped) atomicAdd(A.clamps, clamped);
}

// Ideal-gas recovery pass: every cell of every grid once per evaluation of L
// (the stage kernel reads the result for its own and halo cells, so the Newton
// iteration runs once per cell instead of once per staging).
template <class T>
__global__ void __launch_bounds__(256) recover_ideal_cells(StageArgs<T> A) {
    const int b = (int)blockIdx.x;
    int g = 0;
    if (A.ngrid > 0) {
        int lo = 0, hi = A.ngrid - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.grids[mid].rblk0 <= b) lo = mid;
            else hi = mid - 1;
        }
        g = lo;
    }
    const StageGrid<T>& G = A.ngrid > 0 ? A.grids[g] : A.one;
    const long long n = (long long)G.n[0] * G.n[1] * G.n[2];
    const long long i = (long long)(b - G.rblk0) * 256 + threadIdx.x;
    unsigned cl = 0;
    if (i < n) {
        const T* u = A.us + G.off;
        T* q = A.prim + G.off;
        double kap, Mxs, Mys, Mzs, p, e;
        recover_ideal((double)u[i], (double)u[n + i], (double)u[2 * n + i], (double)u[3 * n + i],
                      (double)u[4 * n + i], G.gm1, kap, Mxs, Mys, Mzs, p, e, cl);
        q[i] = (T)(kap * Mxs);
        q[n + i] = (T)(kap * Mys);
        q[2 * n + i] = (T)(kap * Mzs);
        q[3 * n + i] = (T)p;
        q[4 * n + i] = (T)(e + p > 0.0 ? (G.gm1 + 1.0) * p / (e + p) : 0.0);
    }
    if (cl) atomicAdd(A.clamps, cl);
}

template <class T>
hipError_t launch_recover_ideal(const StageArgs<T>& a, long long nblocks, hipStream_t s) {
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    recover_ideal_cells<T><<<dim3((unsigned)nblocks), 256, 0, s>>>(a);
    return hipGetLastError();
}

template hipError_t launch_recover_ideal<float>(const StageArgs<float>&, long long, hipStream_t);
template hipError_t launch_recover_ideal<double>(const StageArgs<double>&, long long, hipStream_t);

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
int stage_default_segment(const int n[3], int tx) {
    // enough blocks to fill the chip several times over (about 3 x 256 x 4
    // resident blocks), segments of 16 to 64 planes (each segment re-enters
    // 2R halo planes)
    const int ty = 256 / tx;
    const long long tiles = (long long)((n[0] + tx - 1) / tx) * ((n[1] + ty - 1) / ty);
    const long long target = 4096;
    long long nseg = (target + tiles - 1) / tiles;
    const long long max_seg = (n[2] + 15) / 16;
    if (nseg > max_seg) nseg = max_seg;
    if (nseg < 1) nseg = 1;
    int seg = (int)((n[2] + nseg - 1) / nseg);
    if (seg > 64) seg = 64;
    return seg;
}

template <class T>
void stage_shape(StageGrid<T>& g, int tx, int seg) {
    const int ty = 256 / tx;
    if (seg < 1) seg = 1;
    if (seg > g.n[2]) seg = g.n[2];
    g.ntx = (g.n[0] + tx - 1) / tx;
    g.nty = (g.n[1] + ty - 1) / ty;
    g.seg = seg;
    g.nseg = (g.n[2] + seg - 1) / seg;
}

template <class T, int ORDER, int TX>
static hipError_t launch_stage_t(bool hub, bool local, int eos, const StageArgs<T>& a, dim3 grid, hipStream_t s) {
    if (eos == EOS_CONFORMAL) {
        if (hub && local) stage_fused<T, ORDER, TX, true, true, EOS_CONFORMAL><<<grid, 256, 0, s>>>(a);
        else if (hub) stage_fused<T, ORDER, TX, true, false, EOS_CONFORMAL><<<grid, 256, 0, s>>>(a);
        else if (local) stage_fused<T, ORDER, TX, false, true, EOS_CONFORMAL><<<grid, 256, 0, s>>>(a);
        else stage_fused<T, ORDER, TX, false, false, EOS_CONFORMAL><<<grid, 256, 0, s>>>(a);
    } else if (eos == EOS_IDEAL && !hub) {
        // analytic boundaries are the conformal fluid's
        if (local) stage_fused<T, ORDER, TX, false, true, EOS_IDEAL><<<grid, 256, 0, s>>>(a);
        else stage_fused<T, ORDER, TX, false, false, EOS_IDEAL><<<grid, 256, 0, s>>>(a);
    } else {
        return hipErrorInvalidValue;
    }
    return hipSuccess;
}

template <class T>
hipError_t launch_stage(int order, int tx, bool hub, bool local, int eos, const StageArgs<T>& a,
                        long long nblocks, hipStream_t s) {
    if (nblocks <= 0 || nblocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nblocks);
    hipError_t e;
    if (order == 5) {
        if (tx == 16) e = launch_stage_t<T, 5, 16>(hub, local, eos, a, grid, s);
        else if (tx == 32) e = launch_stage_t<T, 5, 32>(hub, local, eos, a, grid, s);
        else return hipErrorInvalidValue;
    } else if (order == 7) {
        // WENO7 tiles are 16 x 16 (a 32 x 8 tile has 320 halo cells per plane)
        if (tx == 16) e = launch_stage_t<T, 7, 16>(hub, local, eos, a, grid, s);
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    return e != hipSuccess ? e : hipGetLastError();
}

template void stage_shape<float>(StageGrid<float>&, int, int);
template void stage_shape<double>(StageGrid<double>&, int, int);
template hipError_t launch_stage<float>(int, int, bool, bool, int, const StageArgs<float>&, long long, hipStream_t);
template hipError_t launch_stage<double>(int, int, bool, bool, int, const StageArgs<double>&, long long, hipStream_t);

}  // namespace rh
