// rh_internal.hpp -- host-side interface between the plan runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rh_device.hpp"
#include "../../include/rh.h"

namespace rh {

// Epilogue of the last directional sweep of an evaluation of L:
//   0: write L (accumulated over the directions done so far) to `lacc`;
//   1..3: fuse the SSP-RK3 stage combine and write the new state to `uout`.
enum { STAGE_WRITE_L = 0, STAGE_1 = 1, STAGE_2 = 2, STAGE_3 = 3 };

// Equations of state of the kernels (the values of RH_EOS_*).
enum { EOS_CONFORMAL = 0, EOS_IDEAL = 1 };

template <class T>
struct SweepArgs {
    const T* us;        // stage input (stencil source)
    const T* u0;        // u^n (stages 2 and 3 read it pointwise)
    T* lacc;            // L accumulator: read unless `first`, written when stage == 0
    T* uout;            // new state when stage > 0 (may alias u0: read pointwise first)
    long long fstride;  // elements per field (nx*ny*nz)
    int n[3];           // nx, ny, nz
    int bc;             // boundary condition of the sweep axis
    int first;          // this sweep starts L (no accumulator read)
    int stage;          // STAGE_*
    int seg;            // rolling segment length (y/z sweeps)
    T inv_h;            // 1 / cell width along the sweep axis
    T dt;               // Runge-Kutta step
    T eps;              // WENO epsilon
    HubbleBC hb;        // analytic boundary data (bc == HUBBLE)
    unsigned* clamps;   // floor counter
};

// One grid of a batched (event-ensemble) launch.  All of the grid's fields live
// at element offset `off` of every batched buffer, in the single-grid layout.
template <class T>
struct BatchGrid {
    long long off;
    int n[3];
    int bc[3];
    T inv_h[3];
    int blk0[3];     // first block of this grid in the launch of sweep class 0/1/2
    int seg[3];      // rolling segment length along y (1) and z (2)
    int nchunk[3];   // 256-lane chunks of the (x, w) plane for y (1) and z (2)
    T eps;           // WENO epsilon of this grid
    double c0[3];
    double h[3];
    double t0, e0, n0;   // analytic (HUBBLE) boundary parameters of this grid
};

template <class T>
struct BatchArgs {
    SweepArgs<T> base;            // buffers (batch bases), eps, dt, stage, first, time
    const BatchGrid<T>* grids;    // device array
    int ngrid;
};

// Adjoint sweep along one axis: ub += (dL_axis/du)(u)^T w.
template <class T>
struct AdjArgs {
    const T* u;         // state at which the Jacobian is taken
    const T* w;         // weights (adjoint of L)
    T* ub;              // accumulated adjoint of u (read-modify-write)
    long long fstride;
    int n[3];
    int bc;             // boundary condition of the sweep axis
    int seg;            // owned segment length along the axis
    T inv_h;
    T eps;
    T scale;            // ub += scale * (J^T w) of this axis
    T* pk;              // per-cell recovery pack (kappa, p, dkappa/dE, dkappa/dM2, dp/dE, dp/dM2) or null;
                        // the whole-row x adjoint writes it, the other sweeps read it
    HubbleBC hb;
};

// y (dir 1) or z (dir 2) axis of the adjoint: a.ub += a.scale J_dir^T w.
// a.pk (required) holds the recovery and its derivatives for every cell.
template <class T>
hipError_t launch_adjoint_sweep(int dir, int order, AdjArgs<T> a, hipStream_t s);
// Fill the six-field recovery pack of state u (layout [5][ncell] -> [6][ncell]).
template <class T>
hipError_t launch_adjoint_pack(const T* u, T* pk, long long ncell, hipStream_t s);

// Linear combination a1 X1 + a2 X2 + a3 X3 of state-layout buffers (null X
// terms are skipped; they may alias the output).
template <class T>
struct Lin3 {
    T a1, a2, a3;
    const T *X1, *X2, *X3;
};
// x axis of the adjoint (LDS tiles or whole rows): a.ub = init + a.scale J_x^T w,
// written without reading a.ub.  a.pk (required) holds the recovery pack, or,
// where adjoint_x_rows() holds, receives it from this launch (whole-row kernel).
template <class T>
hipError_t launch_adjoint_x(int order, AdjArgs<T> a, Lin3<T> init, hipStream_t s);
// True where the x adjoint takes whole periodic rows and writes the pack itself.
bool adjoint_x_rows(const int n[3], int bc_x);
template <class T>
hipError_t launch_fill_zero(T* p, long long n, hipStream_t s);
template <class T>
hipError_t launch_lincomb(T* out, long long n, T a, const T* X, T b, const T* Y, T c, const T* Z, T d,
                          const T* V, hipStream_t s);

// Launchers (return hipGetLastError() of the launch).
template <class T>
hipError_t launch_sweep(int dir, int order, const SweepArgs<T>& a, hipStream_t s);
template <class T>
hipError_t launch_combine(const SweepArgs<T>& a, hipStream_t s);
template <class T>
hipError_t launch_sweep_batch(int dir, int order, int tx, const BatchArgs<T>& b, int nblocks,
                              hipStream_t s);
void batch_blocks(const int n[3], int tx, const int seg[3], int blocks[3], int nchunk[3]);
// Field conversion for the equation of state eos (EOS_*; gm1 = gamma - 1 of the ideal gas).
template <class T>
hipError_t launch_set_fields(T* state, const double* src, int kind, long long ncell, int eos, double gm1,
                             hipStream_t s);
template <class T>
hipError_t launch_get_fields(const T* state, double* dst, int kind, long long ncell,
                             unsigned* clamps, int eos, double gm1, hipStream_t s);
template <class T>
hipError_t launch_totals(const T* state, long long ncell, double* partials, int nblk,
                         double* out, hipStream_t s);

constexpr int kTotalsBlocks = 512;

// x-sweep tile width chosen for nx (64, 32 or 16 cells; 256 threads per block).
int choose_tile_x(int nx, int ghosts);
// rolling segment length along y or z
int choose_segment(int n, int ncols);

// Fused x and y sweeps (one launch doing both axes, bitwise the result of the
// x sweep followed by the y sweep): applies to WENO5 and WENO7 grids with a
// periodic x axis of 64, 128, 192 or 256 cells and more than one cell along y.
bool sweep_xy_applies(int order, const int n[3], int bc_x);
// a: the y sweep's arguments (first = 1; bc, inv_h of y); inv_hx = 1 / dx.
template <class T>
hipError_t launch_sweep_xy(int order, SweepArgs<T> a, T inv_hx, hipStream_t s);

// ---------------------------------------------------------------------------
// Fused stage: one launch evaluates L along x, y and z and applies the stage
// combine (or stores L).  Work items are (grid, x-y tile, z segment).
// ---------------------------------------------------------------------------
template <class T>
struct StageGrid {
    long long off;          // element offset of this grid in every buffer
    int n[3];
    int bc[3];
    T inv_h[3];
    T eps;
    int ntx, nty;           // tiles along x and y
    int seg, nseg;          // z segment length and number of segments
    int blk0;               // first (logical) block of this grid
    double c0[3], h[3];     // cell-0 centre and widths (analytic boundaries)
    double t0, e0, n0;      // analytic boundary parameters
    double gm1;             // ideal gas: gamma - 1 (unused for the conformal fluid)
    int limiter;            // MUSTA-FORCE: MUSCL slope limiter (RH_LIMITER_*)
    int mk;                 // MUSTA-FORCE: FORCE evaluations per face
    T lam;                  // MUSTA-FORCE: dt/dx of the local predictor-corrector
    int rblk0;              // ideal gas: first block of this grid in the recovery pass
};

template <class T>
struct StageArgs {
    const T* us;            // stage input
    const T* u0;            // u^n (stages 2 and 3 read it pointwise)
    T* out;                 // new state (stage > 0; may alias u0) or L (STAGE_WRITE_L)
    T dt;
    int stage;              // STAGE_*
    double t;               // stage time (analytic boundaries)
    unsigned* clamps;       // floor counter
    const StageGrid<T>* grids;   // device table (ngrid > 0), sorted by blk0
    int ngrid;              // 0: single grid in `one`
    StageGrid<T> one;
    T* prim;                // ideal gas: per-cell (vx, vy, vz, p, c_s^2) of the stage input, in
                            // the state layout (written by the recovery pass, read by the stage)
};

// Blocks of 256 cells of the ideal-gas recovery pass for one grid.
template <class T>
long long recover_blocks(const StageGrid<T>& g) {
    return ((long long)g.n[0] * g.n[1] * g.n[2] + 255) / 256;
}
// The ideal-gas recovery pass: A.prim <- (vx, vy, vz, p, c_s^2) of every cell of
// A.us (FP64 Newton recovery, stored in the plan precision), floors counted once
// per cell; nblocks is the sum of recover_blocks over the grids (ordered by rblk0).
template <class T>
hipError_t launch_recover_ideal(const StageArgs<T>& a, long long nblocks, hipStream_t s);

// Tile width along x of the fused stage (16 or 32; 256 / tx rows along y).
constexpr int kStageTiles[2] = {16, 32};
// Fill ntx, nty, nseg (and seg, clamped to nz) of g for tile width tx and z segment seg.
template <class T>
void stage_shape(StageGrid<T>& g, int tx, int seg);
template <class T>
long long stage_blocks(const StageGrid<T>& g) {
    return (long long)g.ntx * g.nty * g.nseg;
}
// Launch the fused stage over nblocks blocks (tile width tx in {16, 32}); hub
// selects the instantiation with analytic (HUBBLE) ghost cells, local the
// Lax-Friedrichs splitting with alpha per interface, eos the equation of state.
template <class T>
hipError_t launch_stage(int order, int tx, bool hub, bool local, int eos, const StageArgs<T>& a,
                        long long nblocks, hipStream_t s);
// Default z segment of the fused stage for a grid of n cells (tiles of tx).
int stage_default_segment(const int n[3], int tx);

// MUSTA-FORCE stage (the same work items, with x-y tiles of kMustaTX x
// kMustaTY cells): one launch evaluates the MUSCL + MUSTA face fluxes of x, y
// and z and applies the stage combine.
constexpr int kMustaTX = 16, kMustaTY = 15;
template <class T>
void musta_shape(StageGrid<T>& g, int seg);
int musta_default_segment(const int n[3]);
template <class T>
// limiter (RH_LIMITER_*) and mk (FORCE evaluations per face) are those of
// every grid of the launch (they select the kernel instance).
hipError_t launch_musta(bool hub, int eos, int limiter, int mk, const StageArgs<T>& a, long long nblocks,
                        hipStream_t s);

// The chip hands consecutive blocks of a launch to its eight XCDs in turn
// (block b to XCD b mod 8).  Renumbering gives every XCD a contiguous range of
// logical blocks, so tiles that share halo cells meet in the same L2.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

// Grid of a fused-stage block: binary search of the block table sorted by
// first block (ngrid > 0), or the single grid.
template <class T>
__device__ __forceinline__ int stage_grid_of(const StageArgs<T>& A, int b) {
    int g = 0;
    if (A.ngrid > 0) {
        int lo = 0, hi = A.ngrid - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (A.grids[mid].blk0 <= b) lo = mid;
            else hi = mid - 1;
        }
        g = lo;
    }
    return g;
}

__device__ __forceinline__ int ghost_index(int m, int nd, int bc) {
    if (bc == RH_BC_PERIODIC) {
        m %= nd;
        return m < 0 ? m + nd : m;
    }
    return m < 0 ? 0 : nd - 1;   // outflow: zero-gradient copy of the edge cell
}

// Load / store through a uniform base pointer and a 32-bit byte offset (the
// plan limits one field to < 4 GiB), so that address arithmetic stays 32-bit
// per lane and the base lives in scalar registers.
template <class T>
__device__ __forceinline__ T ld_off(const T* base, uint32_t off) {
    return *(const T*)((const char*)base + off);
}
template <class T>
__device__ __forceinline__ void st_off(T* base, uint32_t off, T v) {
    *(T*)((char*)base + off) = v;
}

// State of cell (x, y, z) of grid G, of which at most one coordinate lies
// outside the grid; ghost cells follow the boundary condition of that axis
// (analytic ones are evaluated at the stage time t).  The analytic branch is
// compiled only where HUB is set: inlined into a rolling loop its FP64
// temporaries cost about 30 registers per lane even when never taken.
template <class T, bool HUB>
__device__ __forceinline__ void stage_load(const StageGrid<T>& G, const T* us, long long F, double t,
                                           int x, int y, int z, T u[5]) {
    bool analytic = false;
    if (x < 0 || x >= G.n[0]) {
        if (HUB && G.bc[0] == RH_BC_HUBBLE) analytic = true;
        else x = ghost_index(x, G.n[0], G.bc[0]);
    }
    if (y < 0 || y >= G.n[1]) {
        if (HUB && G.bc[1] == RH_BC_HUBBLE) analytic = true;
        else y = ghost_index(y, G.n[1], G.bc[1]);
    }
    if (z < 0 || z >= G.n[2]) {
        if (HUB && G.bc[2] == RH_BC_HUBBLE) analytic = true;
        else z = ghost_index(z, G.n[2], G.bc[2]);
    }
    if (HUB && analytic) {
        HubbleBC hb;
        hb.t = t;
        hb.t0 = G.t0;
        hb.e0 = G.e0;
        hb.n0 = G.n0;
        double uh[5];
        hubble_conserved(hb, G.c0[0] + x * G.h[0], G.c0[1] + y * G.h[1], G.c0[2] + z * G.h[2], uh);
#pragma unroll
        for (int f = 0; f < 5; ++f) u[f] = (T)uh[f];
        return;
    }
    const uint32_t off = (uint32_t)sizeof(T) * ((uint32_t)x + (uint32_t)G.n[0] * ((uint32_t)y + (uint32_t)G.n[1] * (uint32_t)z));
#pragma unroll
    for (int f = 0; f < 5; ++f) u[f] = ld_off(us + f * F, off);
}

}  // namespace rh
