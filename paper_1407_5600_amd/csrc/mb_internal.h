// Internal state of the multiblob library: grid handle, spring table, FFT
// plans, tile geometry and the per-kernel timing hooks.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/multiblob.h"

namespace mb {

// Stable kernel ids (reported by the timing interface).
enum KernelId : int {
    K_BIN_COUNT = 0,
    K_SCAN_REDUCE,
    K_SCAN_APPLY,
    K_SPRINGS_SCATTER,
    K_BIN_SCATTER,
    K_SPRINGS,
    K_SPREAD,
    K_FFT_X_FWD,
    K_FFT_Y_FWD,
    K_FFT_Z_SPECTRAL,
    K_FFT_Y_INV,
    K_FFT_X_INV,
    K_INTERP,
    K_INTERP_STEP,
    K_U0,
    K_DIAG,
    K_FOLD,
    K_INTERP_GRAD,
    K_SPRINGS_ADJ,
    K_FFT_XY_INV,
    K_NUM
};

// Spring table of the particle template on the device: the pair list and,
// per blob, its incident pairs with the pair's other blob.
struct SpringsDev {
    const int* pa;          // [npairs]
    const int* pb;          // [npairs]
    const double* r0;       // [npairs]
    const int* adj_start;   // [nb + 1]
    const int* adj_pair;    // [2 * npairs] pair << 8 | other blob of the pair
    double k;
    int nb;
    int npairs;
    int ppb;                // particles per block of the springs kernels
};

// Tile geometry for spreading and interpolation.
// Tiles are numbered box-tile major: the 2^(lfx+lfy+lfz) tiles of one
// spreading box tile (2^lfx along x, ...) are consecutive, x fastest within
// it, and the box tiles (nbx x nby x ...) follow one another x fastest, so a
// box tile's blobs form one range of the tile-sorted records.  For the box
// tiles themselves (and any tiles not grouped) lfx = lfy = lfz = 0, nbx =
// ntx, nby = nty: plain x-fastest order.
struct Tiles {
    int tx, ty, tz;     // tile extent in cells
    int ntx, nty, ntz;  // tiles per axis
    int n;              // tiles per box
    int remap;          // 1: XCD-aware block -> tile mapping
    int nbox;           // boxes of the grid (a batch of equal boxes)
    int lfx, lfy, lfz;  // log2 of the tiles per box tile along each axis
    int nbx, nby;       // box tiles along x and y
};


// Tile shapes (tx, ty, tz) with instantiated spreading and interpolation
// kernels: the LDS of the float32 interpolation (three components of the
// (tx+3)(ty+3)(tz+3) box) stays under 64 KB.
#define MB_TILE_SHAPES(X) X(16, 8, 8) X(8, 8, 8) X(32, 8, 8) X(16, 16, 8) X(16, 8, 16) X(8, 16, 16)

bool tile_shape_supported(int tx, int ty, int tz);
// A spreading kernel exists for box tiles of sx x sy x sz cells made of
// binning tiles of tx x ty x tz.
bool box_shape_supported(int sx, int sy, int sz, int tx, int ty, int tz);

struct TimerPair {
    hipEvent_t a, b;
    int id;
};

}  // namespace mb

struct mb_springs {
    int nb;
    int npairs;
    int ppb;
    double k;
    int device;
    int* d_pa;
    int* d_pb;
    double* d_r0;
    int* d_adj_start;
    int* d_adj_pair;
};

struct mb_grid {
    mb_grid_desc d;
    int device;
    // workspace: every O(N) and O(M) scratch buffer below (tables to force
    // partials and the non-finite flag) lies in this one region
    void* ws;           // null until a workspace is set (external_workspace)
    size_t ws_bytes;
    bool ws_owned;      // allocated by the library (freed at destroy)
    int* d_flag;        // [0] non-finite flag (check_finite; bit 2: a springs
                        // block gave up waiting for the offsets), [1] the
                        // fused scan's published launch number
    uint32_t scan_epoch;  // launches of the springs kernel with the fused scan
    double* d_qint;     // [max_blobs][3] positions in the step calls' particle order
    double* d_pint;     // [max_blobs][3] per-particle forces, then velocities, same order
    int* d_order;       // [max_blobs] caller's particle of each internal particle
    int ntiles_cap;     // tiles per box the workspace holds (all shapes)
    int L, NC;          // cells per side, complex columns L/2 + 1
    int64_t N;          // L^3 (cells of one box)
    size_t fsz;         // bytes per scalar (8 or 4)
    // FFT
    void* d_tw;         // twiddles W_L^k, k < L (cplx<T>)
    void* d_dsym;       // D symbol per mode index: (1 - e^{-2 pi i m / L}) / h
    void* d_d2;         // |D symbol|^2 per mode index (T)
    void* d_spec;       // [3][L(z)][NC(kx)][L(ky)] cplx<T>
    int nblk_x;         // blocks of an x pass
    double* d_psum;     // [nblk_x][2] per-block sums of v and f (float64)
    // binning (by tile)
    int* d_count;       // [tiles] (kept zeroed between uses)
    int* d_offs;        // [tiles + 1]
    int* d_bsum;        // scan block sums
    int nscan;          // scan blocks
    int* d_tile;        // [max_blobs] tile of each blob
    int* d_rank;        // [max_blobs] place among its tile's blobs
    int* d_perm;        // [max_blobs] blob of each sorted record
    int64_t perm_m;     // d_perm is a permutation of [0, perm_m) (-1: none)
    void* d_rec;        // [max_blobs] records
    size_t rec_size;
    mb::Tiles tiles;       // binning, spreading and interpolation tiles
    mb::Tiles btiles;      // spread box tiles: whole numbers of tiles per axis
    void* d_box;           // [3][tiles][box nodes] spread boxes of the step
    double* d_u;           // [max_blobs][3] blob velocities of the last step
    double* d_adj;         // reverse-step scratch (allocated on first use)
    double* d_adj_part;    // per-block k / r0 derivative sums (deterministic)
    size_t adj_part_cap;   // doubles in d_adj_part
    void* d_ffield;        // force field of forced steps (allocated on first use)
    double* d_mid;         // midpoint scheme: q* and a velocity per blob (first use)
    int scheme;            // mb_scheme of the steps
    double* d_tile_part;   // [tiles][4]  (sum v_a, max |Dv|)
    double* d_force_part;  // [force blocks][3]
    int force_blocks_cap;
    // timing
    uint32_t timing;    // bit mask of timed kernel ids
    std::vector<mb::TimerPair> pending;
    std::vector<hipEvent_t> free_events;
    double acc_ms[mb::K_NUM];
    int64_t acc_n[mb::K_NUM];
};

namespace mb {

// Timing of a launch of kernel `id` (when timing is enabled for it): two
// events, queued for mb_grid_kernel_times, that the launch itself records
// at its start and end (hipExtLaunchKernel), so the duration is the
// kernel's execution without the gaps around it.  False: not timed.
bool timer_pair(mb_grid* g, int id, hipEvent_t* start, hipEvent_t* stop);

#define MB_LAUNCH(g, id, s, kern, grid, block, shm, ...)                          \
    do {                                                                          \
        hipEvent_t a_ = nullptr, b_ = nullptr;                                    \
        if (::mb::timer_pair((g), (id), &a_, &b_))                                \
            hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), (shm), (s), a_, b_, \
                                  0, __VA_ARGS__);                                \
        else                                                                      \
            hipLaunchKernelGGL(kern, dim3(grid), dim3(block), (shm), (s),         \
                               __VA_ARGS__);                                      \
    } while (0)

// Blocks of an x pass of the FFT solve (one float64 partial sum pair each).
int fft_x_blocks(int L, int precision);

// Workspace set-up on stream s: the FFT twiddle and symbol tables (computed
// on the device), zeroed tile counts, partial sums and non-finite flag.
hipError_t init_workspace(mb_grid* g, hipStream_t s);
// Zero n 32-bit words at p (a kernel, never a memset node in a graph).
hipError_t zero_words(void* p, size_t n, hipStream_t s);

// Launchers (templated on the field scalar type, float or double).  Each
// returns hipSuccess or the launch error.
// Tile, rank and counting sort of the blobs at q; with counted the counts,
// tiles and ranks are already in place (the previous step's interpolation
// binned these positions) and only the scan runs.
// scan: also the scan of the counts into offsets (else the springs kernel
// of the step does it: scatter_springs with scan).
template <typename T>
hipError_t bin_blobs(mb_grid* g, int64_t M, const double* q, hipStream_t s,
                     bool counted = false, bool scan = true);
// Records of the binned blobs with forces F scaled by fscale (h^-3 when
// fscale <= 0: a force density).
template <typename T>
hipError_t scatter_records(mb_grid* g, int64_t M, const double* q,
                           const double* F, hipStream_t s, double fscale = 0.0);
// Non-finite flag of the grid's checks (null unless check_finite).
inline int* finite_flag(mb_grid* g) { return g->d.check_finite ? g->d_flag : nullptr; }
// Springs and records; force_sums: also the per-block sums of the blob
// forces read by the diagnostics.
// scan: block 0 of the kernel first scans the tile counts (left by the
// binning, bin_blobs with scan = false) into the offsets the others wait for;
// only where fused_scan_ok.
template <typename T>
hipError_t scatter_springs(mb_grid* g, const SpringsDev& sp, int64_t P,
                           const double* q, const double* Fext, hipStream_t s,
                           const double* Gblob = nullptr, bool force_sums = true,
                           bool scan = false);
// The scan can ride in the springs kernel: a single scan block's worth of
// tiles and a stream not being captured (a captured launch would replay its
// launch number; d_flag[1] is zeroed with the workspace, launch numbers
// start at 1).
bool fused_scan_ok(mb_grid* g, hipStream_t s);
hipError_t spring_forces(const SpringsDev& sp, int64_t P, const double* q,
                         const double* Fext, double* F, hipStream_t s,
                         mb_grid* timing_grid, const double* Gblob = nullptr);
// qbar += (dF/dq)^T Fbar; kbar, r0bar (nullable) accumulate the k and rest
// length parts.
hipError_t springs_adjoint(const SpringsDev& sp, int64_t P, const double* q,
                           const double* Fbar, double* qbar, double* kbar,
                           double* r0bar, hipStream_t s, mb_grid* timing_grid,
                           double* part = nullptr);
// Doubles of per-block partial sums springs_adjoint writes to `part`
// (then summed in block order) instead of its float64 atomics.
size_t springs_adjoint_part_size(const SpringsDev& sp, int64_t P);
// out = (a ? a : 0) + sc b; y += x (n doubles).
hipError_t blob_axpy(int64_t n, const double* a, double sc, const double* b, double* out,
                     hipStream_t s);
hipError_t blob_add(int64_t n, const double* x, double* y, hipStream_t s);
// y = (rho/dt) x + (eta/2) L_h x (explicit half of Crank-Nicolson).
template <typename T>
hipError_t apply_cn(mb_grid* g, const T* x, T* y, hipStream_t s);
// Spreading into the per-tile boxes (g->d_box), and the field from them.
template <typename T>
hipError_t spread_boxes(mb_grid* g, hipStream_t s);
template <typename T>
hipError_t fold_boxes(mb_grid* g, T* f, hipStream_t s, const T* add = nullptr);
// Fluid solve; the force is f, or the boxes of the last spreading when
// boxed is set (f unused).
template <typename T>
hipError_t fluid_solve(mb_grid* g, const T* v_in, const T* f, T* v_out,
                       hipStream_t s, bool boxed = false);
// Elements of the box array: 3 components x tiles x (tx+3)(ty+3)(tz+3).
size_t box_elems(const Tiles& t);
// Interpolation of v at the binned blobs (u_out, q_update += dt u, both
// nullable; diag: per-tile partial sums); bin_next (with q_update): also
// bin the moved blobs into the counts of the next binning.
template <typename T>
hipError_t interpolate(mb_grid* g, int64_t M, const T* v, double* u_out,
                       double* q_update, int diag, hipStream_t s, double uscale = 1.0,
                       bool bin_next = false);
// gout += wscale sum_a W_a grad_q (J v)_a per blob, on the binned records.
template <typename T>
hipError_t interpolate_grad(mb_grid* g, const T* v, const double* W, double wscale,
                            double* gout, hipStream_t s);
hipError_t particle_means(mb_grid* g, int64_t P, int nb, const double* u,
                          double* U0, hipStream_t s);
hipError_t diagnostics(mb_grid* g, int force_blocks, double* diag,
                       hipStream_t s);
// Particle order of a step call: particles counting-sorted by the tile of
// their last blob (the centre of the icosahedral template) into d_order
// (internal particle -> caller's particle), and the positions q and forces
// Fext (nullable) gathered into d_qint and d_pint in that order.
hipError_t order_particles(mb_grid* g, int64_t P, int nb, const double* q,
                           const double* Fext, hipStream_t s);
// Back to the caller's order: positions into q, and (each nullable) the blob
// velocities u_int into u_out and particle velocities U0_int into U0_out.
hipError_t unorder_particles(mb_grid* g, int64_t P, int nb, double* q, const double* u_int,
                             double* u_out, const double* U0_int, double* U0_out,
                             hipStream_t s);
size_t record_size(int precision);
// Blocks and dynamic LDS bytes of the springs kernels for P particles.
int springs_blocks(const SpringsDev& sp, int64_t P);
size_t springs_lds(const SpringsDev& sp);

}  // namespace mb
