// HIP kernels of the multiblob step for gfx950 and their launchers.
//
// Per step: blobs are counting-sorted by cell (count, scan, scatter with the
// spring forces), spread tile by tile with LDS accumulation, the fluid is
// solved by a hand-written 3-D FFT (x pass with the Crank-Nicolson
// right-hand side fused in, y pass, z pass fused with the projection and
// the viscous divide, inverse y, inverse x), and the new velocity is
// interpolated tile by tile from an LDS copy of the field, moving the blobs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "mb_box.h"
#include "mb_device.h"
#include "mb_internal.h"

namespace mb {

// Sorted-blob records, in two arrays.  The geometry record holds the
// position's fraction of its cell per axis, s = x/h - floor(x/h) in [0, 1),
// and the packed cell: bits 0-8 x, 9-17 y, 18-26 z, 27-29 the "rounds up"
// bit per axis (s >= 1/2).  The kernel offset of the cell-centred node set
// is t = s - bit (nearest node c + bit), that of the component's own,
// half-cell shifted set t = s - 1/2 (nearest node c); rec_t forms them.
// The force record (F h^-3 per component, [pos][3]) is a separate array:
// the interpolation reads only the geometry.
template <typename T>
struct __align__(16) RecG {
    T s[3];
    uint32_t cell;
};

// Kernel offset of a record for velocity component a along axis b.
template <typename T>
__device__ __forceinline__ T rec_t(const RecG<T>& r, int a, int b) {
    return a == b ? r.s[b] - T(0.5) : r.s[b] - T((r.cell >> (27 + b)) & 1u);
}

constexpr int BLK = 256;

struct Geom {
    int c[3];
    int up[3];
    double s[3];
};

// Cell, rounding bits and kernel offsets of a position (float64).  For the
// node set of velocity component a along axis b the node coordinate is
// x = q_b/h - (1/2) delta_ab; the nearest node is i0 = floor(x + 1/2) and
// t = x - i0 in [-1/2, 1/2).  q_b/h is formed as q_b (1/h) (exact for h a
// power of two, else within an ulp; at a tie of the rounding either node
// set gives the same sums, the kernel vanishing at 3/2).
__device__ __forceinline__ Geom blob_geom(const double* __restrict__ q,
                                          int64_t i, double inv_h, int L) {
    Geom g;
    const double Ld = (double)L;
    const double invL = 1.0 / Ld;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double x = q[3 * i + b] * inv_h;
        const double fl = floor(x);
        const double s = x - fl;  // [0, 1)
        // fl mod L without integer division: exact for |fl| < 2^53, the
        // rounded quotient is off by at most one and corrected
        double c = fl - floor(fl * invL) * Ld;
        if (c < 0.0) c += Ld;
        if (c >= Ld) c -= Ld;
        // non-finite or beyond 2^53 cells: any in-range cell (such input
        // has no meaningful result; no index may leave the grid)
        if (!(c >= 0.0 && c < Ld)) c = 0.0;
        g.c[b] = (int)c;
        g.up[b] = s >= 0.5 ? 1 : 0;
        g.s[b] = s;
    }
    return g;
}

// Index of the tile with tile coordinates tc (box-tile major, see Tiles).
__device__ __forceinline__ int tile_index(const int tc[3], const Tiles& tl) {
    const int bt = ((tc[2] >> tl.lfz) * tl.nby + (tc[1] >> tl.lfy)) * tl.nbx + (tc[0] >> tl.lfx);
    const int lx = tc[0] & ((1 << tl.lfx) - 1), ly = tc[1] & ((1 << tl.lfy) - 1),
              lz = tc[2] & ((1 << tl.lfz) - 1);
    return (bt << (tl.lfx + tl.lfy + tl.lfz)) + (((lz << tl.lfy) + ly) << tl.lfx) + lx;
}
// Tile coordinates of tile index t (the inverse of tile_index).
__device__ __forceinline__ void tile_coords(int t, const Tiles& tl, int tc[3]) {
    const int nl = tl.lfx + tl.lfy + tl.lfz;
    const int loc = t & ((1 << nl) - 1);
    int bt = t >> nl;
    const int bx = bt % tl.nbx;
    bt /= tl.nbx;
    const int by = bt % tl.nby;
    const int bz = bt / tl.nby;
    tc[0] = (bx << tl.lfx) + (loc & ((1 << tl.lfx) - 1));
    tc[1] = (by << tl.lfy) + ((loc >> tl.lfx) & ((1 << tl.lfy) - 1));
    tc[2] = (bz << tl.lfz) + (loc >> (tl.lfx + tl.lfy));
}

// Tile of a cell: blobs are sorted by the tiles of spreading and
// interpolation (extents powers of two).
__device__ __forceinline__ int tile_linear(const int c[3], const Tiles& tl) {
    const int tc[3] = {c[0] >> (__ffs(tl.tx) - 1), c[1] >> (__ffs(tl.ty) - 1),
                       c[2] >> (__ffs(tl.tz) - 1)};
    return tile_index(tc, tl);
}

// 1 when any of the n values is NaN or infinite.
__device__ __forceinline__ int nonfinite(const double* x, int n) {
    int bad = 0;
    for (int k = 0; k < n; ++k) bad |= !isfinite(x[k]);
    return bad;
}

__device__ __forceinline__ uint32_t cell_pack(const Geom& g) {
    return (uint32_t)g.c[0] | ((uint32_t)g.c[1] << 9) | ((uint32_t)g.c[2] << 18) |
           ((uint32_t)g.up[0] << 27) | ((uint32_t)g.up[1] << 28) |
           ((uint32_t)g.up[2] << 29);
}

// ---------------------------------------------------------------------------
// Block scan helpers.
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = BLK * SCAN_ITEMS;  // 4096

__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

// Exclusive scan of `vals` (n entries) held in LDS tile `s` of SCAN_TILE
// entries (padded indexing); returns the tile total.
__device__ int scan_tile_lds(int* s, int* scratch) {
    int local[SCAN_ITEMS];
    int sum = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        local[k] = s[scan_pad(threadIdx.x * SCAN_ITEMS + k)];
        sum += local[k];
    }
    int total;
    int run = block_exclusive_scan(sum, scratch, &total);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        s[scan_pad(threadIdx.x * SCAN_ITEMS + k)] = run;
        run += local[k];
    }
    __syncthreads();
    return total;
}

// ---------------------------------------------------------------------------
// Binning: counting sort of blobs by tile.  Blobs are taken in `order` (the
// sorted order of the previous binning when it covered the same blobs, so
// that a block's blobs fall in a few consecutive tiles; the identity
// otherwise): a block counts its blobs of tiles [t0, t0 + 64) in LDS (t0 the
// tile of its first blob) and adds each such count to the global count with
// one atomic; other blobs take a global atomic each.  rank is the blob's
// place among its tile's blobs, in no particular order.  With a batch of
// boxes, blob i belongs to box i / mbox and tiles are numbered box by box.
constexpr int TILE_WIN = 64;

__global__ void __launch_bounds__(BLK)
k_tile_count(const double* __restrict__ q, const int* __restrict__ order,
             int64_t M, int64_t mbox, double inv_h, int L, Tiles tl, int* __restrict__ count,
             int* __restrict__ tile_of, int* __restrict__ rank) {
    __shared__ int lcount[TILE_WIN];
    __shared__ int lbase[TILE_WIN];
    __shared__ int t0s;
    const int64_t j = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (threadIdx.x < TILE_WIN) lcount[threadIdx.x] = 0;
    int64_t i = -1;
    int t = 0;
    if (j < M) {
        i = order ? order[j] : j;
        const Geom g = blob_geom(q, i, inv_h, L);
        t = (int)(i / mbox) * tl.n + tile_linear(g.c, tl);  // box i / mbox
    }
    if (threadIdx.x == 0) t0s = t;  // block 0's first blob exists (M > 0)
    __syncthreads();
    const int k = t - t0s;
    const bool local = i >= 0 && k >= 0 && k < TILE_WIN;
    int r = 0;
    if (local) r = atomicAdd(&lcount[k], 1);
    else if (i >= 0) r = atomicAdd(&count[t], 1);
    __syncthreads();
    if (threadIdx.x < TILE_WIN) {
        const int c = lcount[threadIdx.x];
        lbase[threadIdx.x] = c > 0 ? atomicAdd(&count[t0s + threadIdx.x], c) : 0;
    }
    __syncthreads();
    if (i >= 0) {
        tile_of[i] = t;
        rank[i] = local ? lbase[k] + r : r;
    }
}

// Per-block sums of the counts.
__global__ void __launch_bounds__(BLK)
k_scan_reduce(const int* __restrict__ count, int64_t n, int* __restrict__ bsum) {
    __shared__ double red[16];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int s = 0;
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t i = base + k * BLK + threadIdx.x;
        if (i < n) s += count[i];
    }
    const double tot = block_reduce<false>((double)s, red);
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int)tot;
}

// offs[i] = exclusive prefix of count; offs[n] = total; count reset to 0.
// Each block adds the sums of the blocks before it (a few hundred at most).
__global__ void __launch_bounds__(BLK)
k_scan_apply(int* __restrict__ count, int64_t n, const int* __restrict__ bsum,
             int* __restrict__ offs) {
    __shared__ int s[SCAN_TILE + SCAN_TILE / 32];
    __shared__ int scratch[16];
    __shared__ double red[16];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int off = 0;  // the counts of the blocks before this one
    if (gridDim.x > 1) {
        int before = 0;
        for (int b = threadIdx.x; b < (int)blockIdx.x; b += BLK) before += bsum[b];
        off = (int)block_reduce<false>((double)before, red);
    }
    {
        int c[SCAN_ITEMS];  // all loads before the LDS stores
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const int i = k * BLK + threadIdx.x;
            c[k] = count[base + i < n ? base + i : 0];
        }
#pragma unroll
        for (int k = 0; k < SCAN_ITEMS; ++k) {
            const int i = k * BLK + threadIdx.x;
            s[scan_pad(i)] = (base + i < n) ? c[k] : 0;
        }
    }
    __syncthreads();
    const int total = scan_tile_lds(s, scratch);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int i = k * BLK + threadIdx.x;
        if (base + i < n) {
            offs[base + i] = s[scan_pad(i)] + off;
            count[base + i] = 0;
        }
    }
    if (base + SCAN_TILE >= n && threadIdx.x == 0) offs[n] = off + total;
}

// Exclusive scan of n <= BLK * SCAN_ITEMS tile counts into offs (offs[n]
// = their total) by one block of BLK threads, the counts reset to zero:
// thread t takes the counts [t K, t K + K) in registers (K = ceil(n / BLK)),
// a wave scan of the thread sums and the sums of the waves before (wsum,
// BLK / WAVE ints of LDS) give its exclusive prefix.
__device__ void block_scan_counts(int* __restrict__ count, int n, int* __restrict__ offs,
                                  int* wsum) {
    const int t = threadIdx.x, lane = t % WAVE, wave = t / WAVE;
    const int K = (n + BLK - 1) / BLK;
    int c[SCAN_ITEMS];
    int sum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int idx = t * K + j;
        c[j] = (j < K && idx < n) ? count[idx] : 0;
        sum += c[j];
    }
    int x = sum;  // inclusive scan over the wave
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == WAVE - 1) wsum[wave] = x;
    __syncthreads();
    int run = x - sum, total = 0;
#pragma unroll
    for (int w = 0; w < BLK / WAVE; ++w) {
        if (w < wave) run += wsum[w];
        total += wsum[w];
    }
#pragma unroll
    for (int j = 0; j < SCAN_ITEMS; ++j) {
        const int idx = t * K + j;
        if (j < K && idx < n) {
            offs[idx] = run;
            count[idx] = 0;
        }
        run += c[j];
    }
    if (t == 0) offs[n] = total;
}

// Spins (thread 0) until *flag == want, reading it where all XCDs see the
// same value; gives up after 2^20 polls (each a device-memory round trip
// and a short sleep: one to two seconds) and returns false, so that a wait
// never hangs.
__device__ bool wait_flag(const int* flag, int want) {
    for (int it = 0; it < (1 << 20); ++it) {
        if (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == want)
            return true;
        __builtin_amdgcn_s_sleep(4);
    }
    return false;
}

// Writes the records of blob i at sorted position pos (recf may be null:
// no forces).
template <typename T>
__device__ __forceinline__ void write_record(RecG<T>* __restrict__ rec, T* __restrict__ recf,
                                             int* __restrict__ perm, int64_t pos,
                                             int64_t i, const Geom& g,
                                             const double F[3], double inv_vol) {
    RecG<T> r;
#pragma unroll
    for (int b = 0; b < 3; ++b) r.s[b] = (T)g.s[b];
    r.cell = cell_pack(g);
    rec[pos] = r;
    if (recf) {
#pragma unroll
        for (int b = 0; b < 3; ++b) recf[3 * pos + b] = (T)(F[b] * inv_vol);
    }
    perm[pos] = (int)i;
}

// Records in tile order for given forces (F may be null: interpolation).
template <typename T>
__global__ void __launch_bounds__(BLK)
k_bin_scatter(const double* __restrict__ q, const double* __restrict__ F,
              int64_t M, double inv_h, int L, double inv_vol,
              const int* __restrict__ offs, const int* __restrict__ tile_of,
              const int* __restrict__ rank, RecG<T>* __restrict__ rec,
              T* __restrict__ recf, int* __restrict__ perm, int* __restrict__ flag) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i >= M) return;
    const Geom g = blob_geom(q, i, inv_h, L);
    double f[3] = {0.0, 0.0, 0.0};
    if (F) {
        f[0] = F[3 * i];
        f[1] = F[3 * i + 1];
        f[2] = F[3 * i + 2];
    }
    if (flag && (nonfinite(q + 3 * i, 3) | nonfinite(f, 3))) atomicOr(flag, 1);
    const int64_t pos = (int64_t)offs[tile_of[i]] + rank[i];
    write_record<T>(rec, F ? recf : nullptr, perm, pos, i, g, f, inv_vol);
}

// Spring forces of the sp.ppb particles of a block (float64), in two
// parts.  springs_stage loads the blob positions and the incidence lists
// into LDS (and each blob's external force, its share Fext_p / nb of its
// particle's force plus its own G_i, into registers); springs_forces then has thread j (< nblob) sum over the pairs
// incident to its blob the pair force on it, k (|d| - r0) d / |d| with
// d = q_other - q_self (the two blobs of a pair get exactly opposite
// forces), plus the external force.
struct SpringsBlk {
    int64_t p0;    // first particle
    int npart;     // particles of the block
    int nblob;     // blobs of the block (thread j < nblob owns blob p0 nb + j)
    double* qs;    // [ppb * nb][3] positions
    double* r0s;   // [np] rest lengths times r0scale
    int* adj;      // [nb + 1] incidence starts, then [2 np] (pair << 8 | other)
};

// after_loads runs once the position loads are issued (more loads of the
// caller, in flight with them).
template <typename AfterLoads = NoOp>
__device__ __forceinline__ SpringsBlk springs_stage(const SpringsDev& sp,
                                                    const double* __restrict__ q,
                                                    const double* __restrict__ Fext,
                                                    const double* __restrict__ Gblob,
                                                    int64_t P, double* smem,
                                                    double fe[3], double r0scale,
                                                    AfterLoads after_loads = NoOp{}) {
    SpringsBlk B;
    const int nb = sp.nb, np = sp.npairs;
    B.p0 = (int64_t)blockIdx.x * sp.ppb;
    B.npart = (int)(P - B.p0 < sp.ppb ? P - B.p0 : sp.ppb);
    B.nblob = B.npart * nb;
    B.qs = smem;
    B.r0s = smem + 3 * sp.ppb * nb;
    B.adj = (int*)(B.r0s + np);
    const double* qg = q + 3 * B.p0 * nb;  // contiguous blobs of the block
    // every load is issued before any result is used (one round trip): the
    // positions (a block holds at most BLK blobs: springs_blocks), the
    // external force of the thread's particle and its blob's own force
    // (indices clamped into the block, values dropped below), the tables;
    // then the LDS stores
    double ld[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = threadIdx.x + k * BLK;
        ld[k] = qg[i < 3 * B.nblob ? i : 0];
    }
    after_loads();
    const bool mine = (int)threadIdx.x < B.nblob;
    const int j = mine ? (int)threadIdx.x : 0;
    double fx[3] = {0.0, 0.0, 0.0}, gx[3] = {0.0, 0.0, 0.0};
    if (Fext) {  // (a kernel argument: uniform over the block)
        const double* f = Fext + 3 * (B.p0 + j / nb);
        fx[0] = f[0];
        fx[1] = f[1];
        fx[2] = f[2];
    }
    if (Gblob) {
        const double* gb = Gblob + 3 * (B.p0 * nb + j);
        gx[0] = gb[0];
        gx[1] = gb[1];
        gx[2] = gb[2];
    }
    // tables (each at least one entry): the first BLK rest lengths and 2 BLK
    // incidence codes through registers, any beyond (more than 128 pairs) in
    // loops
    const int t = threadIdx.x;
    const double tr0 = sp.r0[t < np ? t : 0];
    const int tas = sp.adj_start[t <= nb ? t : 0];  // nb <= 64 < BLK
    const int tap0 = sp.adj_pair[t < 2 * np ? t : 0];
    const int tap1 = sp.adj_pair[t + BLK < 2 * np ? t + BLK : 0];
    if (t < np) B.r0s[t] = r0scale * tr0;
    if (t <= nb) B.adj[t] = tas;
    if (t < 2 * np) B.adj[nb + 1 + t] = tap0;
    if (t + BLK < 2 * np) B.adj[nb + 1 + t + BLK] = tap1;
    for (int e = t + BLK; e < np; e += BLK) B.r0s[e] = r0scale * sp.r0[e];
    for (int e = t + 2 * BLK; e < 2 * np; e += BLK) B.adj[nb + 1 + e] = sp.adj_pair[e];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int i = threadIdx.x + k * BLK;
        if (i < 3 * B.nblob) B.qs[i] = ld[k];
    }
    __syncthreads();
    const double inv_nb = 1.0 / (double)nb;
#pragma unroll
    for (int b = 0; b < 3; ++b) fe[b] = mine ? fx[b] * inv_nb + gx[b] : 0.0;
    return B;
}

// NEWTON: Newton steps of the reciprocal square root (two for float64
// results; one for forces that are rounded to float32 records, whose
// relative error it leaves far below float32 rounding).  B.r0s holds k r0
// (springs_stage with r0scale = k).
template <int NEWTON = 2>
__device__ __forceinline__ void springs_forces(const SpringsDev& sp, const SpringsBlk& B,
                                               const double fe[3], double F[3],
                                               int64_t* blob) {
    const int nb = sp.nb;
    F[0] = F[1] = F[2] = 0.0;
    *blob = -1;
    const int j = threadIdx.x;
    if (j >= B.nblob) return;
    const int pl = j / nb;
    const int b = j - pl * nb;
    const double* qp = B.qs + 3 * pl * nb;  // the particle's blobs
    const double qx = qp[3 * b], qy = qp[3 * b + 1], qz = qp[3 * b + 2];
    double fx = fe[0], fy = fe[1], fz = fe[2];
    const int* inc = B.adj + nb + 1;
    const int e0 = B.adj[b], e1 = B.adj[b + 1];
    auto pair = [&](int code) {
        const int o = code & 0xff;
        const double* qo = qp + 3 * o;
        const double dx = qo[0] - qx, dy = qo[1] - qy, dz = qo[2] - qz;
        // k (|d| - r0) / |d| = k - k r0 / |d|
        const double inv_len = rsqrt_nr<NEWTON>(dx * dx + dy * dy + dz * dz);
        const double s = fma(-B.r0s[code >> 8], inv_len, sp.k);
        fx += s * dx;
        fy += s * dy;
        fz += s * dz;
    };
    constexpr int DMAX = 16;  // incident pairs held in registers
    if (e1 - e0 <= DMAX) {
        // all incidence codes read at once, then the pairs four at a time
        // (their position reads independent of one another)
        int codes[DMAX];
#pragma unroll
        for (int x = 0; x < DMAX; ++x) codes[x] = e0 + x < e1 ? inc[e0 + x] : -1;
#pragma clang loop unroll(full)
        for (int x = 0; x < DMAX; ++x)
            if (codes[x] >= 0) pair(codes[x]);
    } else {
        for (int x = e0; x < e1; ++x) pair(inc[x]);
    }
    F[0] = fx;
    F[1] = fy;
    F[2] = fz;
    *blob = B.p0 * nb + j;
}

// Spring forces fused with the scatter of the records; also the per-block
// float64 sums of the blob forces (momentum diagnostics).  The blob's tile,
// rank and the tile's offset are fetched while the forces are computed, and
// its record geometry comes from the LDS copy of the positions.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_springs_scatter(SpringsDev sp, const double* __restrict__ q,
                  const double* __restrict__ Fext, const double* __restrict__ Gblob,
                  int64_t P, double inv_h, int L,
                  double inv_vol, int* __restrict__ offs,
                  const int* __restrict__ tile_of, const int* __restrict__ rank,
                  RecG<T>* __restrict__ rec, T* __restrict__ recf, int* __restrict__ perm,
                  double* __restrict__ fpart, int* __restrict__ flag, int* __restrict__ count,
                  int scan_n, int* __restrict__ sflag, int epoch, int* __restrict__ err) {
    extern __shared__ double smem[];
    __shared__ double red[16 * 3];
    __shared__ int scan_ok;
    const int64_t p0 = (int64_t)blockIdx.x * sp.ppb;
    // scan_n > 0: block 0 first scans the tile counts into offs (there is
    // then no scan kernel ahead of this one) and publishes them by setting
    // *sflag = epoch after a device-scope fence; every block reads its
    // offsets only after seeing that (block 0 is dispatched first, so the
    // others' bounded wait ends)
    if (scan_n > 0 && blockIdx.x == 0) {
        block_scan_counts(count, scan_n, offs, reinterpret_cast<int*>(red));
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // offsets out of this XCD's L2
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(sflag, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const int nblob = (int)((P - p0 < sp.ppb ? P - p0 : sp.ppb) * sp.nb);
    const bool own = (int)threadIdx.x < nblob;
    const int64_t ib = p0 * sp.nb + threadIdx.x;
    const int64_t ibc = own ? ib : p0 * sp.nb;  // loads without branches
    const int tl = tile_of[ibc];
    const int rk = rank[ibc];
    int off = 0;
    double fe[3];
    // the block's positions are requested before the tile's offset, which
    // waits for the tile; both arrive while the block stages its positions
    const SpringsBlk B = springs_stage(sp, q, Fext, Gblob, P, smem, fe, sp.k,
                                       [&] { if (scan_n == 0) off = offs[tl]; });
    double F[3];
    int64_t i;
    springs_forces<sizeof(T) == 4 ? 1 : 2>(sp, B, fe, F, &i);
    if (scan_n > 0) {
        // the offsets as block 0 left them in memory (past any stale copy
        // in this XCD's L2)
        if (threadIdx.x == 0) scan_ok = wait_flag(sflag, epoch);
        __syncthreads();
        if (!scan_ok) {
            if (threadIdx.x == 0) atomicOr(err, 2);
            i = -1;  // no offsets: no records written (the error bit is set)
        }
        off = __hip_atomic_load(&offs[tl], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (i >= 0) {
        const Geom g = blob_geom(B.qs, threadIdx.x, inv_h, L);
        write_record<T>(rec, recf, perm, (int64_t)off + rk, i, g, F, inv_vol);
        if (flag && (nonfinite(B.qs + 3 * threadIdx.x, 3) | nonfinite(F, 3)))
            atomicOr(flag, 1);
    }
    if (fpart) {  // (a kernel argument: uniform over the block)
        double tot[3] = {F[0], F[1], F[2]};
        block_reduce3(tot, red);
        if (threadIdx.x == 0) {
            fpart[3 * blockIdx.x] = tot[0];
            fpart[3 * blockIdx.x + 1] = tot[1];
            fpart[3 * blockIdx.x + 2] = tot[2];
        }
    }
}

__global__ void __launch_bounds__(BLK)
k_springs(SpringsDev sp, const double* __restrict__ q,
          const double* __restrict__ Fext, const double* __restrict__ Gblob, int64_t P,
          double* __restrict__ Fout) {
    extern __shared__ double smem[];
    double fe[3];
    const SpringsBlk B = springs_stage(sp, q, Fext, Gblob, P, smem, fe, sp.k);
    double F[3];
    int64_t i;
    springs_forces(sp, B, fe, F, &i);
    if (i < 0) return;
    Fout[3 * i] = F[0];
    Fout[3 * i + 1] = F[1];
    Fout[3 * i + 2] = F[2];
}

// Transposed Jacobian of the spring forces applied to Fbar (float64).  For
// blob i and each incident pair with other blob o, d = q_o - q_i, the pair
// force on i is k (1 - r0/|d|) d with the symmetric Jacobian
// J(d) = k [(1 - r0/|d|) I + r0 d d^T / |d|^3]; since F_i depends on q_i
// through -J and F_o through +J, qbar_i += sum_o J(d) (Fbar_o - Fbar_i).
// Per blob also kbar += Fbar_i . (1 - r0/|d|) d and r0bar_e += -k Fbar_i .
// d/|d| (both ends of a pair together give the pair's full term); the block
// sums these in LDS and adds them to kbar / r0bar with one float64 atomic
// per entry (their order, hence the last bits, may vary run to run).  With
// part (deterministic sums) the block instead writes its kbar sum and, per
// pair e = (a, b), the sum over its particles of
// -k (Fbar_a - Fbar_b) . d/|d| (d = q_b - q_a), in particle order, to
// part[block][1 + npairs]; k_sum_parts adds the blocks in order.
__global__ void __launch_bounds__(BLK)
k_springs_adjoint(SpringsDev sp, const double* __restrict__ q,
                  const double* __restrict__ Fbar, int64_t P,
                  double* __restrict__ qbar, double* __restrict__ kbar,
                  double* __restrict__ r0bar, double* __restrict__ part) {
    extern __shared__ double smem[];
    __shared__ double red[16];
    double fe[3];
    const SpringsBlk B = springs_stage(sp, q, nullptr, nullptr, P, smem, fe, 1.0);
    // Fbar of the block's blobs and the per-pair sums after the positions
    double* fb = B.qs + 3 * sp.ppb * sp.nb + sp.npairs + 
                 (sp.nb + 1 + 2 * sp.npairs + 1) / 2;
    double* rb = fb + 3 * sp.ppb * sp.nb;
    const int nb = sp.nb;
    for (int i = threadIdx.x; i < 3 * B.nblob; i += BLK) fb[i] = Fbar[3 * B.p0 * nb + i];
    for (int e = threadIdx.x; e < sp.npairs; e += BLK) rb[e] = 0.0;
    __syncthreads();
    double kb = 0.0;
    const int j = threadIdx.x;
    if (j < B.nblob) {
        const int pl = j / nb;
        const int b = j - pl * nb;
        const double* qp = B.qs + 3 * pl * nb;
        const double* fp = fb + 3 * pl * nb;
        const double qx = qp[3 * b], qy = qp[3 * b + 1], qz = qp[3 * b + 2];
        const double fx = fp[3 * b], fy = fp[3 * b + 1], fz = fp[3 * b + 2];
        double gx = 0.0, gy = 0.0, gz = 0.0;
        const int* inc = B.adj + nb + 1;
        const int e1 = B.adj[b + 1];
        for (int x = B.adj[b]; x < e1; ++x) {
            const int code = inc[x];
            const int o = code & 0xff;
            const int e = code >> 8;
            const double dx = qp[3 * o] - qx, dy = qp[3 * o + 1] - qy, dz = qp[3 * o + 2] - qz;
            const double len = sqrt(dx * dx + dy * dy + dz * dz);
            const double r0 = B.r0s[e];
            const double sc = sp.k * (1.0 - r0 / len);
            const double tc = sp.k * r0 / (len * len * len);
            const double lx = fp[3 * o] - fx, ly = fp[3 * o + 1] - fy, lz = fp[3 * o + 2] - fz;
            const double ld = lx * dx + ly * dy + lz * dz;
            gx += sc * lx + tc * dx * ld;
            gy += sc * ly + tc * dy * ld;
            gz += sc * lz + tc * dz * ld;
            const double fd = fx * dx + fy * dy + fz * dz;
            kb += fd * (1.0 - r0 / len);
            if (!part) atomicAdd(&rb[e], -sp.k * fd / len);
        }
        double* qo = qbar + 3 * (B.p0 * nb + j);
        qo[0] += gx;
        qo[1] += gy;
        qo[2] += gz;
    }
    const double kt = block_reduce<false>(kb, red);  // also orders the LDS sums
    if (part) {
        double* pb = part + (size_t)blockIdx.x * (1 + sp.npairs);
        if (threadIdx.x == 0) pb[0] = kt;
        for (int e = threadIdx.x; e < sp.npairs; e += BLK) {
            const int a = sp.pa[e], b = sp.pb[e];
            double acc = 0.0;
            for (int pl = 0; pl < B.npart; ++pl) {
                const double* qa = B.qs + 3 * (pl * nb + a);
                const double* qb = B.qs + 3 * (pl * nb + b);
                const double* fa = fb + 3 * (pl * nb + a);
                const double* fbb = fb + 3 * (pl * nb + b);
                const double dx = qb[0] - qa[0], dy = qb[1] - qa[1], dz = qb[2] - qa[2];
                const double len = sqrt(dx * dx + dy * dy + dz * dz);
                acc += -sp.k * ((fa[0] - fbb[0]) * dx + (fa[1] - fbb[1]) * dy +
                                (fa[2] - fbb[2]) * dz) / len;
            }
            pb[1 + e] = acc;
        }
        return;
    }
    if (threadIdx.x == 0 && kbar) atomicAdd(kbar, kt);
    if (r0bar)
        for (int e = threadIdx.x; e < sp.npairs; e += BLK)
            if (rb[e] != 0.0) atomicAdd(&r0bar[e], rb[e]);
}

// Block partials of k_springs_adjoint summed in block order: entry 0 into
// *kbar, entry 1 + e into r0bar[e] (either may be null).
__global__ void __launch_bounds__(BLK)
k_sum_parts(const double* __restrict__ part, int nblocks, int nent,
            double* __restrict__ kbar, double* __restrict__ r0bar) {
    const int j = blockIdx.x * BLK + threadIdx.x;
    if (j >= nent) return;
    double acc = 0.0;
    for (int b = 0; b < nblocks; ++b) acc += part[(size_t)b * nent + j];
    if (j == 0) {
        if (kbar) *kbar += acc;
    } else if (r0bar) {
        r0bar[j - 1] += acc;
    }
}

// FFT tables of an L-point grid of spacing h: twiddles W_L^k = e^{-2 pi i
// k/L}, the divergence symbol (1 - e^{-2 pi i k/L})/h (its real part as
// 2 sin^2(pi k/L)/h, accurate for small k) and |symbol|^2 = 4 sin^2(pi
// k/L)/h^2, from float64 sin/cos of multiples of pi, cast to T.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_fft_tables(int L, double h, T* __restrict__ tw, T* __restrict__ ds, T* __restrict__ d2) {
    const int k = blockIdx.x * BLK + threadIdx.x;
    if (k >= L) return;
    double s2, c2;
    sincospi(2.0 * (double)k / (double)L, &s2, &c2);
    const double sh = sinpi((double)k / (double)L);
    tw[2 * k] = (T)c2;
    tw[2 * k + 1] = (T)(-s2);
    ds[2 * k] = (T)(2.0 * sh * sh / h);
    ds[2 * k + 1] = (T)(s2 / h);
    d2[k] = (T)(4.0 * sh * sh / (h * h));
}

__global__ void __launch_bounds__(BLK)
k_zero(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Blob arrays: out = (a ? a : 0) + s b, and y += x, over n entries.
__global__ void __launch_bounds__(BLK)
k_axpy(int64_t n, const double* __restrict__ a, double s, const double* __restrict__ b,
       double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i < n) out[i] = (a ? a[i] : 0.0) + s * b[i];
}

__global__ void __launch_bounds__(BLK)
k_add(int64_t n, const double* __restrict__ x, double* __restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i < n) y[i] += x[i];
}

// y = c0 x + c1 L_h x per component (7-point periodic Laplacian without the
// 1/h^2, folded into c1): the explicit half of the Crank-Nicolson step.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_apply_cn(int L, int nbox, T c0, T c1, const T* __restrict__ x, T* __restrict__ y) {
    const int64_t N = (int64_t)L * L * L;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i >= 3 * N * nbox) return;
    const int64_t cb = (i / N) * N;
    const int64_t r = i - cb;
    const int xx = (int)(r % L), yy = (int)((r / L) % L), zz = (int)(r / ((int64_t)L * L));
    const int xm = xx == 0 ? L - 1 : xx - 1, xp = xx == L - 1 ? 0 : xx + 1;
    const int ym = yy == 0 ? L - 1 : yy - 1, yp = yy == L - 1 ? 0 : yy + 1;
    const int zm = zz == 0 ? L - 1 : zz - 1, zp = zz == L - 1 ? 0 : zz + 1;
    const T* X = x + cb;
    const int64_t row = ((int64_t)zz * L + yy) * L;
    const T c = X[row + xx];
    const T lap = (X[row + xm] + X[row + xp]) +
                  (X[((int64_t)zz * L + ym) * L + xx] + X[((int64_t)zz * L + yp) * L + xx]) +
                  (X[((int64_t)zm * L + yy) * L + xx] + X[((int64_t)zp * L + yy) * L + xx]) -
                  T(6) * c;
    y[i] = c0 * c + c1 * lap;
}

// ---------------------------------------------------------------------------
// Tile helpers shared by spreading and interpolation.
struct TileBox {
    int lo[3];
    int full[3];
    int box;   // box of the batch
    int tile;  // tile within the box
    int gt;    // tile over the batch: box * tiles per box + tile
};

// Block -> (box, tile): the blocks of a box are consecutive; within a box
// the XCD-aware remap gives each XCD a contiguous range of tiles.
__device__ __forceinline__ TileBox tile_box(const Tiles& t, int L) {
    const int b = blockIdx.x;
    TileBox tb;
    tb.box = b / t.n;
    int local = b - tb.box * t.n;
    if (t.remap) local = xcd_remap(local, t.n);
    tb.tile = local;
    tb.gt = tb.box * t.n + local;
    int tc[3];
    tile_coords(local, t, tc);
    tb.lo[0] = tc[0] * t.tx;
    tb.lo[1] = tc[1] * t.ty;
    tb.lo[2] = tc[2] * t.tz;
    tb.full[0] = t.tx == L;
    tb.full[1] = t.ty == L;
    tb.full[2] = t.tz == L;
    return tb;
}

// Periodic wrap of an index known to lie in [-L, 2L).
__device__ __forceinline__ int wrapL(int v, int L) {
    if (v < 0) v += L;
    if (v >= L) v -= L;
    return v;
}

// Fixed-point scale of one tile's box.  A box node receives at most one
// contribution per component from each of the tile's n records, each at
// most (2/3)^3 fmax (fmax = the tile's largest |F h^-3|).  Returns the
// largest e with
//   n (8/27) fmax 2^e + n (rounding) <= lim_sum   and
//   (8/27) fmax 2^e <= lim_one (one contribution),
// with margins for the rounding of the weights and of fmax.
__device__ __forceinline__ int fixed_exponent(double fmax, int n, double lim_sum,
                                              double lim_one) {
    if (!(fmax > 0.0) || n <= 0) return 0;
    const double fm = fmax * (1.0 + 0x1p-20) * (8.0 / 27.0);
    const double avail = lim_sum * (1.0 - 0x1p-20) - n - 1.0;
    const int e_sum = ilogb(avail / (n * fm));
    const int e_one = ilogb(lim_one / fm);
    return e_sum < e_one ? e_sum : e_one;
}

// Spreading: one block per box tile (FX x FY x FZ binning tiles, btl), one
// velocity component at a time.  The box tile's own records (those of its
// cells) add all 27 of their contributions to an LDS box of the nodes they
// can reach, [lo-1, lo+T+1] per axis, so no record is read by more than one
// block and no contribution is masked.  The box is written to the box
// tile's slot of the box array E[a][box tile][box node]; a node of the
// field is the sum of the entries of the (at most 8) boxes holding it
// (box_sum), formed by the fold kernel or by the first FFT pass as it reads
// the force.  Box tiles larger than the binning tiles (16^3 against 16x8x8)
// carry less halo: 1.67 against 2.25 box entries per node, each written
// here and read by the x pass.
//
// Accumulation is in fixed point with integer LDS atomics, which are much
// faster on gfx950 than the floating ones (float32 ones by more than an
// order of magnitude) and make each box independent of the order of the
// additions.  The scale 2^e (fixed_exponent) comes from the tile's record
// count n and largest |F h^-3|, so that no sum can overflow:
//  - mixed: 32-bit sums of float32 contributions rounded to int32 when
//    n <= 2048 (a quantum of about 2^-23 fmax at the ~230 records of a
//    16x8x8 tile of a phi = 0.3 suspension), else 64-bit sums of int32
//    contributions;
//  - float64: 64-bit sums of float64 contributions rounded to int64 (a
//    quantum of at most 2^-50 fmax for n < 27000, coarsening slowly above)
//    when n <= 2^20, else float64 LDS atomics.
// Threads of a spreading block covering f binning tiles: up to 1024 for
// float32 fields, 512 for float64 ones (whose ~80 registers per thread
// would otherwise leave room for one block per CU, not two).
template <typename T>
constexpr int spread_threads(int f) {
    const int cap = sizeof(T) == 4 ? 1024 : 512;
    return f * BLK < cap ? f * BLK : cap;
}

template <typename T, int TX, int TY, int TZ, int FX, int FY, int FZ>
__global__ void __launch_bounds__(spread_threads<T>(FX * FY * FZ))
k_spread(const RecG<T>* __restrict__ rec, const T* __restrict__ recf,
         const int* __restrict__ offs, int L, Tiles btl, Tiles tl, int det,
         T* __restrict__ E) {
    constexpr int NT = spread_threads<T>(FX * FY * FZ);
    constexpr int NR = FX * FY * FZ;  // binning tiles of this box tile
    constexpr int EX = TX + 3, EY = TY + 3, EZ = TZ + 3;
    constexpr int EV = EX * EY * EZ;
    constexpr bool F32 = std::is_same<T, float>::value;
    __shared__ unsigned long long acc[EV];
    __shared__ double red[16];
    unsigned int* acc32 = reinterpret_cast<unsigned int*>(acc);
    double* accd = reinterpret_cast<double*>(acc);
    const TileBox tb = tile_box(btl, L);
    const int tile = tb.tile;
    for (int i = threadIdx.x; i < EV; i += NT) acc[i] = 0ull;
    // the records of this box tile: its binning tiles are numbered
    // consecutively (box-tile major), so their records form one range
    int first, total;
    {
        const int tc[3] = {tb.lo[0] / tl.tx, tb.lo[1] / tl.ty, tb.lo[2] / tl.tz};
        const int g = tb.box * tl.n + tile_index(tc, tl);  // its first binning tile
        first = offs[g];
        total = offs[g + NR] - first;
    }
    // The k-th record a thread takes is the sorted record q(k) of the box
    // tile.  For float32 fields q(k) = (k * P) mod total with P = 263 (269
    // where 263 divides total, 1 where 269 does too), a bijection since P is
    // then prime to total, which gives each wave records from all over
    // the box tile instead of 64 neighbours in one binning tile, whose 27
    // nodes mostly coincide and whose same-address LDS atomics serialise
    // (2.3 us of the 24.7 us spread of a phi = 0.3 suspension on a 128^3
    // grid).  Float64 fields keep the sorted order, q(k) = k, which measured
    // no slower.  The fixed-point sums do not depend on the order.
    int q0 = threadIdx.x, step = NT;  // q(threadIdx.x), q(k + NT) - q(k) mod total
    if constexpr (F32) {
        if (total > 0) {
            const int P = total % 263 ? 263 : (total % 269 ? 269 : 1);
            q0 = (int)(((unsigned long long)threadIdx.x * P) % (unsigned)total);
            step = (int)(((unsigned long long)NT * P) % (unsigned)total);
        }
    }
    auto adv = [&](int q) { q += step; return q >= total ? q - total : q; };
    // this thread's first record is kept in registers for all components
    RecG<T> r0{};
    T F0[3] = {T(0), T(0), T(0)};
    if ((int)threadIdx.x < total) {
        const int p = first + q0;
        r0 = rec[p];
#pragma unroll
        for (int b = 0; b < 3; ++b) F0[b] = recf[3 * (size_t)p + b];
    }
    double fm = 0.0;
#pragma unroll
    for (int b = 0; b < 3; ++b) fm = fmax(fm, fabs((double)F0[b]));
    for (int k = threadIdx.x + NT, q = adv(q0); k < total; k += NT, q = adv(q)) {
        const size_t p = (size_t)(first + q);
#pragma unroll
        for (int b = 0; b < 3; ++b) fm = fmax(fm, fabs((double)recf[3 * p + b]));
    }
    const double fmx = block_reduce<true>(fm, red);
    // mode 0: the fast fixed-point form (u32 for float, u64 for double)
    int mode, e;
    if (F32) {
        mode = total <= 2048 ? 0 : 1;
        e = fixed_exponent(fmx, total, mode == 0 ? 0x1p31 : 0x1p63, 0x1p30);
    } else {
        // up to 2^20 records one 64-bit fixed-point sum (mode 0); beyond,
        // float64 LDS atomics (mode 1, whose last bits depend on the order)
        // or, with det, two 64-bit fixed-point sums (mode 2): the
        // contributions rounded to the quantum 2^-e, then their rounding
        // remainders to 2^-(e+38), which cannot overflow up to 2^25 records
        // (each remainder at most 2^37 quanta)
        mode = total <= (1 << 20) ? 0 : ((det && total <= (1 << 25)) ? 2 : 1);
        e = mode != 1 ? fixed_exponent(fmx, total, 0x1p63, 0x1p50) : 0;
    }
    const int npass = mode == 2 ? 2 : 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      for (int pass = 0; pass < npass; ++pass) {
        for (int k = threadIdx.x, q = q0; k < total; k += NT, q = adv(q)) {
            RecG<T> r = r0;
            // (selected, not indexed: the component loop need not unroll, and an
            // indexed register array would live in scratch memory)
            T Fr = a == 0 ? F0[0] : (a == 1 ? F0[1] : F0[2]);
            if (k >= NT) {
                const size_t p = (size_t)(first + q);
                r = rec[p];
                Fr = recf[3 * p + a];
            }
            T w[3][3];
            int e0[3];  // box index of node i0 - 1
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                kernel_weights<T>(rec_t(r, a, b), w[b]);
                const int c = (int)((r.cell >> (9 * b)) & 511u) - tb.lo[b];  // [0, T)
                const int up = (int)((r.cell >> (27 + b)) & 1u);
                e0[b] = a == b ? c : c + up;
            }
            const int base = (e0[2] * EY + e0[1]) * EX + e0[0];
            const T Fa = ldexp(Fr, e);
            // the 27 node offsets from base are compile-time constants
#define MB_SPREAD_27(ADD)                                                    \
    _Pragma("unroll") for (int oz = 0; oz < 3; ++oz) {                       \
        const T wz = w[2][oz] * Fa;                                          \
        _Pragma("unroll") for (int oy = 0; oy < 3; ++oy) {                   \
            const T wyz = w[1][oy] * wz;                                     \
            _Pragma("unroll") for (int ox = 0; ox < 3; ++ox)                 \
                ADD(base + (oz * EY + oy) * EX + ox, w[0][ox] * wyz);        \
        }                                                                    \
    }
            if (F32) {
                if (mode == 0) {
#define MB_ADD(i, v) atomicAdd(&acc32[i], (unsigned int)__float2int_rn((float)(v)))
                    MB_SPREAD_27(MB_ADD)
#undef MB_ADD
                } else {
#define MB_ADD(i, v) \
    atomicAdd(&acc[i], (unsigned long long)(long long)__float2int_rn((float)(v)))
                    MB_SPREAD_27(MB_ADD)
#undef MB_ADD
                }
            } else {
                if (mode == 0 || (mode == 2 && pass == 0)) {
                    // round to the nearest integer (|v| <= 2^50): adding
                    // 1.5 * 2^52 leaves it in the low bits of the sum
#define MB_ADD(i, v)                                                               \
    atomicAdd(&acc[i], (unsigned long long)(__double_as_longlong((double)(v) + 0x1.8p52) - \
                                            __double_as_longlong(0x1.8p52)))
                    MB_SPREAD_27(MB_ADD)
#undef MB_ADD
                } else if (mode == 2) {
                    // the remainder v - rint(v) (exact), in units of 2^-38
#define MB_ADD(i, v)                                                                   \
    do {                                                                               \
        const double v_ = (double)(v);                                                 \
        const double r_ = v_ - ((v_ + 0x1.8p52) - 0x1.8p52);                           \
        atomicAdd(&acc[i], (unsigned long long)(__double_as_longlong(r_ * 0x1p38 + 0x1.8p52) - \
                                                __double_as_longlong(0x1.8p52)));      \
    } while (0)
                    MB_SPREAD_27(MB_ADD)
#undef MB_ADD
                } else {
#define MB_ADD(i, v) atomicAdd(&accd[i], (double)(v))
                    MB_SPREAD_27(MB_ADD)
#undef MB_ADD
                }
            }
#undef MB_SPREAD_27
        }
        __syncthreads();
        // write the box and clear it for the next component
        T* Ea = E + ((size_t)(tb.box * 3 + a) * btl.n + tile) * EV;
        for (int i = threadIdx.x; i < EV; i += NT) {
            T val;
            if (F32 && mode == 0) {
                val = ldexpf((float)(int)acc32[i], -e);
                acc32[i] = 0u;
            } else if (F32 || mode == 0 || (mode == 2 && pass == 0)) {
                val = (T)ldexp((double)(long long)acc[i], -e);
                acc[i] = 0ull;
            } else if (mode == 2) {  // the remainders, added to the first sum
                val = Ea[i] + (T)ldexp((double)(long long)acc[i], -(e + 38));
                acc[i] = 0ull;
            } else {
                val = (T)accd[i];
                acc[i] = 0ull;
            }
            st32(Ea, (unsigned)i, val);
        }
        __syncthreads();
      }
    }
}

// The field from the boxes (the spreading call of the library), plus an
// optional field `add`.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_fold(const T* __restrict__ E, int L, Tiles tl, const T* __restrict__ add,
       T* __restrict__ f) {
    const int64_t N = (int64_t)L * L * L;
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i >= 3 * N * tl.nbox) return;
    const int64_t bc = i / N;  // box * 3 + component
    const int box = (int)(bc / 3);
    const int a = (int)(bc - 3 * box);
    const int64_t rem = i - bc * N;
    const int x = (int)(rem % L);
    const int y = (int)((rem / L) % L);
    const int z = (int)(rem / ((int64_t)L * L));
    const T val = box_sum(E + (size_t)box * 3 * tl.n * box_volume(tl), tl, a, x, y, z);
    f[i] = add ? val + add[i] : val;
}

// Binning of the moved blobs for the next step, done by the interpolation
// that moves them (count: per-tile counts, zero before; null: none).
struct BinNext {
    int* count;
    int* tile_of;
    int* rank;
};

// Interpolation: one block per tile.  The velocity on nodes [lo-1, hi+2]
// is staged in LDS (rows located through a table of wrapped row offsets),
// all three components at once for float32 fields and one at a time for
// float64 ones (LDS size); then every record of the tile's cells gathers its
// 27 nodes per component.  u (and the move of the blob by dt u) is written
// once per blob for each thread's first record (16x8x8-size tiles: first
// two, held in registers), per component for the rest (tiles with more records than
// threads), scaled by uscale.  With part the block also writes its float64
// sum of each component and the max |Dv| over its cells.  With bn.count the
// block also bins the moved blobs as k_tile_count would bin the new
// positions: through LDS counts for the 27 tiles around this one (a blob
// moves less than a tile per step), with one global atomic per tile, and a
// global atomic of its own for any farther move.
// Threads: one per four cells of the tile, at least BLK and at most 512 (the
// 16x16x8 family: one record per thread at these densities).
// Float64: registers capped for four waves per SIMD from 1,024 cells up
// (16x8x8: 115 registers with its second record, 306 against 351 us at
// 256^3 phi = 0.4 and 31.1 against 32.1 us at 128^3 phi = 0.3 with one
// record at five waves; larger tiles fit two blocks per CU either way),
// five below (93, no spills; six spill with the column staging); float32
// is bound by its LDS.
constexpr int interp_threads(int cells) {
    return cells / 4 < BLK ? BLK : (cells / 4 > 512 ? 512 : cells / 4);
}
template <typename T>
constexpr int interp_min_waves(int cells) {
    return sizeof(T) == 8 ? (cells >= 4 * BLK ? 4 : 5) : 1;
}

template <typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(interp_threads(TX * TY * TZ), interp_min_waves<T>(TX * TY * TZ))
k_interp(const RecG<T>* __restrict__ rec, const int* __restrict__ perm,
         const int* __restrict__ offs, int L, Tiles tl, const T* __restrict__ v,
         double* __restrict__ u_out, double uscale, double* __restrict__ q, double dt,
         double inv_h, double* __restrict__ part, BinNext bn) {
    // Staged nodes of component a: [lo-1, lo+T+1] along the axes b != a and
    // [lo-1, lo+T] along its own (half-cell shifted) axis, rows of EX nodes
    // along x; the components' regions follow one another in vt.
    constexpr int EX = TX + 3, EY = TY + 3, EZ = TZ + 3;
    constexpr int TV = TX * TY * TZ;
    constexpr int NT = interp_threads(TV);
    constexpr int RP = NT / EX;              // rows staged per pass
    constexpr int CPT = (TV + NT - 1) / NT;  // own cells per thread
    constexpr int NCS = sizeof(T) == 4 ? 3 : 1;  // components staged together
    constexpr int EYA[3] = {EY, EY - 1, EY};   // rows along y per component
    constexpr int EZA[3] = {EZ, EZ, EZ - 1};   // along z
    constexpr int VOFF[4] = {0, EX * EY * EZ, EX * EY * EZ + EX * (EY - 1) * EZ,
                             EX * EY * EZ + EX * (EY - 1) * EZ + EX * EY * (EZ - 1)};
    // Staging: where EX * EY threads fit in the block (COLS), thread
    // (sx, sy) takes the x slot sx of the row ey = sy at every z of the
    // component (the wrapped z offset is uniform over the block, so each
    // load is one add to the thread's fixed offset; 128^3: float32 23.5 ->
    // 21.2 us, float64 34.2 -> 31.7 us, against ~18 integer instructions
    // per load for a flattened row); otherwise rows r = sr + k RP of the
    // flattened (ey, ez) rows.
    constexpr bool COLS = EX * EY <= NT;
    constexpr int NR = COLS ? EZ : (EY * EZ + RP - 1) / RP;  // loads per component
    __shared__ T vt[NCS == 3 ? VOFF[3] : EX * EY * EZ];
    __shared__ double red[4 * (NT / WAVE)];
    __shared__ int lcount[27];
    __shared__ int lbase[27];
    const TileBox tb = tile_box(tl, L);
    const int tile = tb.gt;
    const int N = L * L * L;  // 3 L^3 < 2^31 for L <= 512
    if (bn.count && threadIdx.x < 27) lcount[threadIdx.x] = 0;
    v += (size_t)tb.box * 3 * N;
    // the tile's own records
    const int first = offs[tile];
    const int total = offs[tile + 1] - first;
    const int sx = threadIdx.x % EX;  // staging: x slot and first row
    const int sr = threadIdx.x / EX;
    const int gx = wrapL(tb.lo[0] - 1 + sx, L);
    const int pos0 = (int)threadIdx.x < total ? first + (int)threadIdx.x : -1;
    // the thread's first record and its blob, loaded once
    RecG<T> r0{};
    int64_t i0 = -1;
    double q0[3] = {0.0, 0.0, 0.0};  // its position, fetched with the staging
    {
        // loads without branches (an index clamped into the records), so
        // that nothing waits for them before their first use
        const int pc = pos0 >= 0 ? pos0 : 0;
        r0 = rec[pc];
        const int ic = perm[pc];
        i0 = pos0 >= 0 ? ic : -1;
    }
    // tiles of four cells per thread and BLK threads (16x8x8: 233 records
    // on average at phi = 0.3, 310 at 0.4): the thread's second record too,
    // so that tiles with more records than threads have no chain of
    // dependent loads for it in the gathers or the binning (float32 has the
    // registers to spare at the occupancy its LDS allows; float64 is capped
    // at four waves for it, above)
    constexpr bool R2 = NT == BLK && TV >= 4 * NT;
    constexpr int KREG = R2 ? 2 * NT : NT;  // records k < KREG are in registers
    const int pos1 = R2 && (int)threadIdx.x + NT < total ? first + (int)threadIdx.x + NT : -1;
    RecG<T> r1{};
    int64_t i1 = -1;
    double q1[3] = {0.0, 0.0, 0.0};
    if constexpr (R2) {
        const int pc = pos1 >= 0 ? pos1 : (pos0 >= 0 ? pos0 : 0);
        r1 = rec[pc];
        const int ic = perm[pc];
        i1 = pos1 >= 0 ? ic : -1;
    }
    double u0[3] = {0.0, 0.0, 0.0};  // velocity of the first record
    double u1[3] = {0.0, 0.0, 0.0};  // of the second
    double sv[3] = {0.0, 0.0, 0.0};
    double dv[CPT];
#pragma unroll
    for (int j = 0; j < CPT; ++j) dv[j] = 0.0;
#pragma unroll
    for (int a0 = 0; a0 < 3; a0 += NCS) {
        if (a0 > 0) __syncthreads();  // the previous component's gathers are done
        // all loads of the thread first, then the LDS stores; row r of
        // component a is (ey, ez) = (r mod EYA[a], r / EYA[a])
        // (threads beyond the staged rows load row 0 and store nothing:
        // no branch around the loads)
        T ld[NCS][NR];
        if constexpr (COLS) {
            // byte offsets of the staged z planes (uniform), then per load
            // one add to the thread's offset within the plane
            unsigned zo[NR];
#pragma unroll
            for (int ez = 0; ez < NR; ++ez)
                zo[ez] = (unsigned)(wrapL(tb.lo[2] - 1 + ez, L) * L * L) * (unsigned)sizeof(T);
#pragma unroll
            for (int c = 0; c < NCS; ++c) {
                const int a = a0 + c;
                const int ey = sr < EYA[a] ? sr : 0;
                const unsigned yx = (unsigned)(wrapL(tb.lo[1] - 1 + ey, L) * L + gx) *
                                    (unsigned)sizeof(T);
                const char* va = reinterpret_cast<const char*>(v + (int64_t)a * N);
#pragma unroll
                for (int ez = 0; ez < NR; ++ez)
                    ld[c][ez] = *reinterpret_cast<const T*>(
                        va + ((ez < EZA[a] ? zo[ez] : zo[0]) + yx));
            }
        } else {
            const int srl = sr < RP ? sr : 0;
#pragma unroll
            for (int c = 0; c < NCS; ++c) {
                const int a = a0 + c;
                const int rows = EYA[a] * EZA[a];
                const T* va = v + (int64_t)a * N;  // uniform base, 32-bit offsets
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    int r = srl + k * RP;
                    r = r < rows ? r : srl;
                    const int ey = r % EYA[a], ez = r / EYA[a];
                    ld[c][k] = ld32(va, (unsigned)((wrapL(tb.lo[2] - 1 + ez, L) * L +
                                                    wrapL(tb.lo[1] - 1 + ey, L)) * L + gx));
                }
            }
        }
        if (a0 == 0 && q) {
            // the first record's position, requested once its blob index is
            // in and the staging loads are on their way (blob i0 belongs to
            // this record only: no other thread updates it; without a record
            // blob 0 is read and not used)
            const int64_t ic = i0 >= 0 ? i0 : 0;
            q0[0] = q[3 * ic];
            q0[1] = q[3 * ic + 1];
            q0[2] = q[3 * ic + 2];
            if constexpr (R2) {
                const int64_t jc = i1 >= 0 ? i1 : ic;
                q1[0] = q[3 * jc];
                q1[1] = q[3 * jc + 1];
                q1[2] = q[3 * jc + 2];
            }
        }
        if constexpr (COLS) {
#pragma unroll
            for (int c = 0; c < NCS; ++c) {
                const int a = a0 + c;
                const int off = NCS == 3 ? VOFF[a] : 0;
                if (sr < EYA[a]) {
#pragma unroll
                    for (int ez = 0; ez < NR; ++ez)
                        if (ez < EZA[a]) vt[off + (ez * EYA[a] + sr) * EX + sx] = ld[c][ez];
                }
            }
        } else if (sr < RP) {
#pragma unroll
            for (int c = 0; c < NCS; ++c) {
                const int a = a0 + c;
                const int rows = EYA[a] * EZA[a];
                const int off = NCS == 3 ? VOFF[a] : 0;
#pragma unroll
                for (int k = 0; k < NR; ++k) {
                    const int r = sr + k * RP;
                    if (r < rows) vt[off + r * EX + sx] = ld[c][k];
                }
            }
        }
        __syncthreads();
        for (int k = threadIdx.x; k < total; k += NT) {
            const int pos = first + k;
            RecG<T> r = k < NT ? r0 : r1;
            if (k >= KREG) r = rec[pos];
            double ua[NCS];
#pragma unroll
            for (int c = 0; c < NCS; ++c) {
                const int a = a0 + c;
                T w[3][3];
                int e0[3];  // extended-tile index of node i0 - 1
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    kernel_weights<T>(rec_t(r, a, b), w[b]);
                    const int cc = (int)((r.cell >> (9 * b)) & 511u) - tb.lo[b];  // [0, T)
                    const int up = (int)((r.cell >> (27 + b)) & 1u);
                    e0[b] = a == b ? cc : cc + up;
                }
                const int eya = EYA[a];
                const T* base = vt + (NCS == 3 ? VOFF[a] : 0) + (e0[2] * eya + e0[1]) * EX + e0[0];
                T acc = T(0);
#pragma unroll
                for (int oz = 0; oz < 3; ++oz) {
#pragma unroll
                    for (int oy = 0; oy < 3; ++oy) {
                        const T* row = base + (oz * eya + oy) * EX;
                        const T sxv = w[0][0] * row[0] + w[0][1] * row[1] + w[0][2] * row[2];
                        acc += (w[2][oz] * w[1][oy]) * sxv;
                    }
                }
                ua[c] = uscale * (double)acc;
            }
            if (k < NT) {
#pragma unroll
                for (int c = 0; c < NCS; ++c) u0[a0 + c] = ua[c];  // written at the end
            } else if (k < KREG) {
#pragma unroll
                for (int c = 0; c < NCS; ++c) u1[a0 + c] = ua[c];  // likewise
            } else {
                const int64_t i = perm[pos];
#pragma unroll
                for (int c = 0; c < NCS; ++c) {
                    if (u_out) u_out[3 * i + a0 + c] = ua[c];
                    if (q) q[3 * i + a0 + c] += dt * ua[c];
                }
            }
        }
        if (part) {
#pragma unroll
            for (int c = 0; c < NCS; ++c) {
                const int a = a0 + c;
                const int eya = EYA[a];
                const int str = a == 0 ? 1 : (a == 1 ? EX : EX * eya);
#pragma unroll
                for (int j = 0; j < CPT; ++j) {
                    const int i = threadIdx.x + j * NT;
                    if (i < TV) {
                        const int x = i % TX + 1;
                        const int y = (i / TX) % TY + 1;
                        const int z = i / (TX * TY) + 1;
                        const int c0 = (NCS == 3 ? VOFF[a] : 0) + (z * eya + y) * EX + x;
                        const T val = vt[c0];
                        sv[a] += (double)val;
                        dv[j] += (double)(val - vt[c0 - str]);
                    }
                }
            }
        }
    }
    double qn[3] = {0.0, 0.0, 0.0};  // the first record's new position
    if (pos0 >= 0) {
        const int64_t i = i0;
        if (u_out) {
            u_out[3 * i] = u0[0];
            u_out[3 * i + 1] = u0[1];
            u_out[3 * i + 2] = u0[2];
        }
        if (q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                qn[c] = q0[c] + dt * u0[c];
                q[3 * i + c] = qn[c];
            }
        }
    }
    double qn1[3] = {0.0, 0.0, 0.0};  // the second record's new position
    if (R2 && pos1 >= 0) {
        if (u_out) {
            u_out[3 * i1] = u1[0];
            u_out[3 * i1 + 1] = u1[1];
            u_out[3 * i1 + 2] = u1[2];
        }
        if (q) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                qn1[c] = q1[c] + dt * u1[c];
                q[3 * i1 + c] = qn1[c];
            }
        }
    }
    if (bn.count) {
        // tile coordinates of this tile
        const int ot[3] = {tb.lo[0] / tl.tx, tb.lo[1] / tl.ty, tb.lo[2] / tl.tz};
        const int nt[3] = {tl.ntx, tl.nty, tl.ntz};
        const int sh[3] = {__ffs(tl.tx) - 1, __ffs(tl.ty) - 1, __ffs(tl.tz) - 1};
        int slot = -1, rk = 0, tnew = 0;
        auto slot_of = [&](const int c[3]) {
            int sl = 0;
#pragma unroll
            for (int b = 2; b >= 0; --b) {
                int d = (c[b] >> sh[b]) - ot[b];
                if (d == nt[b] - 1) d = -1;
                if (d == 1 - nt[b]) d = 1;
                if (sl >= 0 && d >= -1 && d <= 1) sl = sl * 3 + d + 1;
                else sl = -1;
            }
            return sl;
        };
        if (pos0 >= 0) {
            const Geom gn = blob_geom(qn, 0, inv_h, L);
            tnew = tb.box * tl.n + tile_linear(gn.c, tl);
            slot = slot_of(gn.c);
            if (slot >= 0) rk = atomicAdd(&lcount[slot], 1);
            else rk = atomicAdd(&bn.count[tnew], 1);
        }
        // the second record (float32) from its registers
        int slot1 = -1, rk1 = 0, tnew1 = 0;
        if (R2 && pos1 >= 0) {
            const Geom gn = blob_geom(qn1, 0, inv_h, L);
            tnew1 = tb.box * tl.n + tile_linear(gn.c, tl);
            slot1 = slot_of(gn.c);
            if (slot1 >= 0) rk1 = atomicAdd(&lcount[slot1], 1);
            else rk1 = atomicAdd(&bn.count[tnew1], 1);
        }
        // records beyond those (positions re-read: written by this thread
        // above): counted through the same LDS slots, their rank within the
        // slot stored and completed below (a global atomic each only for a
        // move beyond the neighbour tiles)
        for (int k = threadIdx.x + KREG; k < total; k += NT) {
            const int64_t i = perm[first + k];
            const Geom gk = blob_geom(q, i, inv_h, L);
            const int t = tb.box * tl.n + tile_linear(gk.c, tl);
            const int sl = slot_of(gk.c);
            bn.tile_of[i] = t;
            bn.rank[i] = sl >= 0 ? atomicAdd(&lcount[sl], 1) : atomicAdd(&bn.count[t], 1);
        }
        __syncthreads();
        if (threadIdx.x < 27) {
            const int c = lcount[threadIdx.x];
            int base = 0;
            if (c > 0) {
                const int d[3] = {(int)threadIdx.x % 3 - 1, ((int)threadIdx.x / 3) % 3 - 1,
                                  (int)threadIdx.x / 9 - 1};
                int tc[3];
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    tc[b] = ot[b] + d[b];
                    if (tc[b] < 0) tc[b] += nt[b];
                    if (tc[b] >= nt[b]) tc[b] -= nt[b];
                }
                const int t = tb.box * tl.n + tile_index(tc, tl);
                base = atomicAdd(&bn.count[t], c);
            }
            lbase[threadIdx.x] = base;
        }
        __syncthreads();
        if (pos0 >= 0) {
            bn.tile_of[i0] = tnew;
            bn.rank[i0] = slot >= 0 ? lbase[slot] + rk : rk;
        }
        if (R2 && pos1 >= 0) {
            bn.tile_of[i1] = tnew1;
            bn.rank[i1] = slot1 >= 0 ? lbase[slot1] + rk1 : rk1;
        }
        for (int k = threadIdx.x + KREG; k < total; k += NT) {
            const int64_t i = perm[first + k];
            int tc[3];  // the tile written above, back to its slot
            tile_coords(bn.tile_of[i] - tb.box * tl.n, tl, tc);
            int sl = 0;
#pragma unroll
            for (int b = 2; b >= 0; --b) {
                int d = tc[b] - ot[b];
                if (d == nt[b] - 1) d = -1;
                if (d == 1 - nt[b]) d = 1;
                if (sl >= 0 && d >= -1 && d <= 1) sl = sl * 3 + d + 1;
                else sl = -1;
            }
            if (sl >= 0) bn.rank[i] += lbase[sl];
        }
    }
    if (part) {
        // the three sums and the max over the block, combined by thread 0
        double dmax = 0.0;
#pragma unroll
        for (int j = 0; j < CPT; ++j) dmax = fmax(dmax, fabs(dv[j]) * inv_h);
        double w4[4] = {wave_sum(sv[0]), wave_sum(sv[1]), wave_sum(sv[2]), wave_max(dmax)};
        constexpr int NW = NT / WAVE;
        static_assert(4 * NW <= 4 * (NT / WAVE), "reduction scratch");
        const int lane = threadIdx.x % WAVE, wid = threadIdx.x / WAVE;
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < 4; ++c) red[4 * wid + c] = w4[c];
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t4[4] = {red[0], red[1], red[2], red[3]};
            for (int w = 1; w < NW; ++w) {
                t4[0] += red[4 * w];
                t4[1] += red[4 * w + 1];
                t4[2] += red[4 * w + 2];
                t4[3] = fmax(t4[3], red[4 * w + 3]);
            }
#pragma unroll
            for (int c = 0; c < 4; ++c) part[4 * tile + c] = t4[c];
        }
    }
}

// Position derivative of the interpolation, contracted with blob weights:
// g_i += wscale sum_a W_{i,a} grad_{q_i} (J_i v)_a.  One block per tile as in
// k_interp (same staged field, one component at a time); per record and
// component the 27-node gather also forms the three derivative sums, with
// d/dq_b of a weight = (1/h) d/dt of it (kernel_weights_deriv).  W and g are
// indexed by blob; each blob belongs to one record, so g is updated without
// atomics.
template <typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(BLK)
k_interp_grad(const RecG<T>* __restrict__ rec, const int* __restrict__ perm,
              const int* __restrict__ offs, int L, Tiles tl, const T* __restrict__ v,
              const double* __restrict__ W, double wscale, double inv_h,
              double* __restrict__ gout) {
    constexpr int EX = TX + 3, EY = TY + 3, EZ = TZ + 3;
    constexpr int EV = EX * EY * EZ;
    constexpr int RP = BLK / EX;
    constexpr int NR = (EY * EZ + RP - 1) / RP;
    __shared__ T vt[EV];
    __shared__ int rowoff[EY * EZ];
    const TileBox tb = tile_box(tl, L);
    const int tile = tb.gt;
    const int N = L * L * L;
    v += (size_t)tb.box * 3 * N;
    for (int r = threadIdx.x; r < EY * EZ; r += BLK) {
        const int ey = r % EY, ez = r / EY;
        rowoff[r] = (wrapL(tb.lo[2] - 1 + ez, L) * L + wrapL(tb.lo[1] - 1 + ey, L)) * L;
    }
    const int first = offs[tile];
    const int total = offs[tile + 1] - first;
    const int sx = threadIdx.x % EX;
    const int sr = threadIdx.x / EX;
    const int gx = wrapL(tb.lo[0] - 1 + sx, L);
    __syncthreads();
    for (int k0 = 0; k0 < total; k0 += BLK) {
        const int k = k0 + threadIdx.x;
        const bool has = k < total;
        RecG<T> r{};
        int64_t i = 0;
        double wgt[3] = {0.0, 0.0, 0.0};
        if (has) {
            r = rec[first + k];
            i = perm[first + k];
            wgt[0] = W[3 * i];
            wgt[1] = W[3 * i + 1];
            wgt[2] = W[3 * i + 2];
        }
        double gr[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < 3; ++a) {
            __syncthreads();  // the previous component's gathers are done
            if (sr < RP) {
                const T* va = v + (int64_t)a * N + gx;
                T ld[NR];
#pragma unroll
                for (int kk = 0; kk < NR; ++kk) {
                    const int rr = sr + kk * RP;
                    ld[kk] = va[rowoff[rr < EY * EZ ? rr : sr]];
                }
#pragma unroll
                for (int kk = 0; kk < NR; ++kk) {
                    const int rr = sr + kk * RP;
                    if (rr < EY * EZ) vt[rr * EX + sx] = ld[kk];
                }
            }
            __syncthreads();
            if (!has) continue;
            T w[3][3], dw[3][3];
            int e0[3];
#pragma unroll
            for (int b = 0; b < 3; ++b) {
                kernel_weights_deriv<T>(rec_t(r, a, b), w[b], dw[b]);
                const int cc = (int)((r.cell >> (9 * b)) & 511u) - tb.lo[b];
                const int up = (int)((r.cell >> (27 + b)) & 1u);
                e0[b] = a == b ? cc : cc + up;
            }
            const T* base = vt + (e0[2] * EY + e0[1]) * EX + e0[0];
            T dx = T(0), dy = T(0), dz = T(0);
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) {
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                    const T* row = base + (oz * EY + oy) * EX;
                    const T sxv = w[0][0] * row[0] + w[0][1] * row[1] + w[0][2] * row[2];
                    const T dsx = dw[0][0] * row[0] + dw[0][1] * row[1] + dw[0][2] * row[2];
                    dx += (w[2][oz] * w[1][oy]) * dsx;
                    dy += (w[2][oz] * dw[1][oy]) * sxv;
                    dz += (dw[2][oz] * w[1][oy]) * sxv;
                }
            }
            const double c = wscale * inv_h * wgt[a];
            gr[0] += c * (double)dx;
            gr[1] += c * (double)dy;
            gr[2] += c * (double)dz;
        }
        if (has) {
            gout[3 * i] += gr[0];
            gout[3 * i + 1] += gr[1];
            gout[3 * i + 2] += gr[2];
        }
    }
}

__global__ void __launch_bounds__(BLK)
k_u0(const double* __restrict__ u, int64_t P, int nb, double* __restrict__ U0) {
    const int64_t p = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (p >= P) return;
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < 3; ++c) s[c] += u[3 * (p * nb + b) + c];
    for (int c = 0; c < 3; ++c) U0[3 * p + c] = s[c] / (double)nb;
}

// Particle order of a step call.  Each particle is counted into the tile
// (box included) of its last blob with one global atomic; after the scan of
// the counts, internal particle offs[tile] + rank is that particle.  The
// gather and the scatter run one thread per float64 of the positions, so
// both sides of every copy are runs of 3 nb contiguous values.
__global__ void __launch_bounds__(BLK)
k_part_count(const double* __restrict__ q, int64_t P, int nb, int64_t pbox, double inv_h,
             int L, Tiles tl, int* __restrict__ count, int* __restrict__ tile_of,
             int* __restrict__ rank) {
    const int64_t p = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (p >= P) return;
    const Geom g = blob_geom(q, p * nb + nb - 1, inv_h, L);
    const int t = (int)(p / pbox) * tl.n + tile_linear(g.c, tl);
    tile_of[p] = t;
    rank[p] = atomicAdd(&count[t], 1);
}

__global__ void __launch_bounds__(BLK)
k_part_gather(const double* __restrict__ q, const double* __restrict__ Fext, int64_t P,
              int nb, const int* __restrict__ offs, const int* __restrict__ tile_of,
              const int* __restrict__ rank, int* __restrict__ order,
              double* __restrict__ qi, double* __restrict__ Fi) {
    const int64_t j = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const int64_t per = 3 * (int64_t)nb;
    if (j >= per * P) return;
    const int64_t p = j / per;
    const int64_t c = j - p * per;
    const int64_t pos = (int64_t)offs[tile_of[p]] + rank[p];
    qi[pos * per + c] = q[j];
    if (c < 3 && Fext) Fi[3 * pos + c] = Fext[3 * p + c];
    if (c == 0) order[pos] = (int)p;
}

__global__ void __launch_bounds__(BLK)
k_part_scatter(const double* __restrict__ qi, const int* __restrict__ order, int64_t P,
               int nb, double* __restrict__ q, const double* __restrict__ ui,
               double* __restrict__ u, const double* __restrict__ U0i,
               double* __restrict__ U0) {
    const int64_t j = (int64_t)blockIdx.x * BLK + threadIdx.x;
    const int64_t per = 3 * (int64_t)nb;
    if (j >= per * P) return;
    const int64_t pi = j / per;
    const int64_t c = j - pi * per;
    const int64_t p = order[pi];
    q[p * per + c] = qi[j];
    if (u) u[p * per + c] = ui[j];
    if (U0 && c < 3) U0[3 * p + c] = U0i[3 * pi + c];
}

__global__ void __launch_bounds__(BLK)
k_diag(const double* __restrict__ tile_part, int ntiles,
       const double* __restrict__ force_part, int nfb, double mom_scale,
       double* __restrict__ diag) {
    __shared__ double red[16];
    double s[3] = {0.0, 0.0, 0.0}, sf[3] = {0.0, 0.0, 0.0}, mx = 0.0;
    for (int i = threadIdx.x; i < ntiles; i += BLK) {
        for (int c = 0; c < 3; ++c) s[c] += tile_part[4 * i + c];
        mx = fmax(mx, tile_part[4 * i + 3]);
    }
    for (int i = threadIdx.x; i < nfb; i += BLK)
        for (int c = 0; c < 3; ++c) sf[c] += force_part[3 * i + c];
    for (int c = 0; c < 3; ++c) {
        const double a = block_reduce<false>(s[c], red);
        const double b = block_reduce<false>(sf[c], red);
        if (threadIdx.x == 0) {
            diag[c] = mom_scale * a;
            diag[3 + c] = b;
        }
    }
    const double m = block_reduce<true>(mx, red);
    if (threadIdx.x == 0) diag[6] = m;
}

// ---------------------------------------------------------------------------
// Launchers.

static inline unsigned blocks_for(int64_t n) {
    return (unsigned)((n + BLK - 1) / BLK);
}

// The two record arrays in the grid's record scratch: geometry, then forces.
template <typename T>
static RecG<T>* rec_geo(mb_grid* g) {
    return (RecG<T>*)g->d_rec;
}
template <typename T>
static T* rec_force(mb_grid* g) {
    const size_t cap = (size_t)std::max<int64_t>(g->d.max_blobs, 1);
    return (T*)((char*)g->d_rec + cap * sizeof(RecG<T>));
}

// Exclusive scan of the tile counts into offs (the counts reset to zero).
static void scan_tiles(mb_grid* g, hipStream_t s) {
    const int nt = g->tiles.n * g->tiles.nbox;
    if (g->nscan > 1)
        MB_LAUNCH(g, K_SCAN_REDUCE, s, k_scan_reduce, g->nscan, BLK, 0, g->d_count,
                  (int64_t)nt, g->d_bsum);
    MB_LAUNCH(g, K_SCAN_APPLY, s, k_scan_apply, g->nscan, BLK, 0, g->d_count,
              (int64_t)nt, g->d_bsum, g->d_offs);
}

template <typename T>
hipError_t bin_blobs(mb_grid* g, int64_t M, const double* q, hipStream_t s, bool counted,
                     bool scan) {
    if (M > 0 && !counted) {
        // the previous sorted order, when it is a permutation of these blobs
        const int* order = g->perm_m == M ? g->d_perm : nullptr;
        MB_LAUNCH(g, K_BIN_COUNT, s, k_tile_count, blocks_for(M), BLK, 0, q, order, M,
                  M / g->tiles.nbox, 1.0 / g->d.h, g->L, g->tiles, g->d_count, g->d_tile,
                  g->d_rank);
    }
    if (scan) scan_tiles(g, s);
    return hipGetLastError();
}

hipError_t order_particles(mb_grid* g, int64_t P, int nb, const double* q,
                           const double* Fext, hipStream_t s) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_part_count, dim3(blocks_for(P)), dim3(BLK), 0, s, q, P, nb,
                       P / g->tiles.nbox, 1.0 / g->d.h, g->L, g->tiles, g->d_count, g->d_tile,
                       g->d_rank);
    scan_tiles(g, s);
    hipLaunchKernelGGL(k_part_gather, dim3(blocks_for(3 * nb * P)), dim3(BLK), 0, s, q, Fext, P,
                       nb, g->d_offs, g->d_tile, g->d_rank, g->d_order, g->d_qint, g->d_pint);
    return hipGetLastError();
}

hipError_t unorder_particles(mb_grid* g, int64_t P, int nb, double* q, const double* u_int,
                             double* u_out, const double* U0_int, double* U0_out,
                             hipStream_t s) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_part_scatter, dim3(blocks_for(3 * nb * P)), dim3(BLK), 0, s,
                       g->d_qint, g->d_order, P, nb, q, u_int, u_out, U0_int, U0_out);
    return hipGetLastError();
}

template <typename T>
hipError_t scatter_records(mb_grid* g, int64_t M, const double* q,
                           const double* F, hipStream_t s, double fscale) {
    if (M == 0) return hipSuccess;
    const double h = g->d.h;
    const double sc = fscale > 0.0 ? fscale : 1.0 / (h * h * h);
    MB_LAUNCH(g, K_BIN_SCATTER, s, k_bin_scatter<T>, blocks_for(M), BLK, 0, q, F,
              M, 1.0 / h, g->L, sc, g->d_offs, g->d_tile, g->d_rank,
              rec_geo<T>(g), rec_force<T>(g), g->d_perm, finite_flag(g));
    g->perm_m = M;
    return hipGetLastError();
}

template <typename T>
hipError_t scatter_springs(mb_grid* g, const SpringsDev& sp, int64_t P,
                           const double* q, const double* Fext, hipStream_t s,
                           const double* Gblob, bool force_sums, bool scan) {
    const int64_t M = P * sp.nb;
    if (M == 0) {
        if (scan) scan_tiles(g, s);
        return hipGetLastError();
    }
    const double h = g->d.h;
    int scan_n = 0, epoch = 0;
    if (scan) {
        scan_n = g->tiles.n * g->tiles.nbox;
        epoch = (int)(++g->scan_epoch & 0x7fffffff);
        if (epoch == 0) epoch = (int)(++g->scan_epoch & 0x7fffffff);
    }
    MB_LAUNCH(g, K_SPRINGS_SCATTER, s, k_springs_scatter<T>, springs_blocks(sp, P), BLK,
              springs_lds(sp), sp, q, Fext, Gblob, P, 1.0 / h, g->L, 1.0 / (h * h * h), g->d_offs,
              g->d_tile, g->d_rank, rec_geo<T>(g), rec_force<T>(g), g->d_perm,
              force_sums ? g->d_force_part : nullptr, finite_flag(g), g->d_count, scan_n,
              g->d_flag + 1, epoch, g->d_flag);
    g->perm_m = M;
    return hipGetLastError();
}

bool fused_scan_ok(mb_grid* g, hipStream_t s) {
    if (g->nscan != 1) return false;
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return st == hipStreamCaptureStatusNone;
}

hipError_t spring_forces(const SpringsDev& sp, int64_t P, const double* q,
                         const double* Fext, double* F, hipStream_t s,
                         mb_grid* tg, const double* Gblob) {
    const int64_t M = P * sp.nb;
    if (M == 0) return hipSuccess;
    MB_LAUNCH(tg, K_SPRINGS, s, k_springs, springs_blocks(sp, P), BLK, springs_lds(sp),
              sp, q, Fext, Gblob, P, F);
    return hipGetLastError();
}

size_t springs_adjoint_lds(const SpringsDev& sp) {
    return springs_lds(sp) + (size_t)(3 * sp.ppb * sp.nb + sp.npairs) * sizeof(double) +
           sizeof(double);
}

hipError_t springs_adjoint(const SpringsDev& sp, int64_t P, const double* q,
                           const double* Fbar, double* qbar, double* kbar,
                           double* r0bar, hipStream_t s, mb_grid* tg, double* part) {
    const int64_t M = P * sp.nb;
    if (M == 0) return hipSuccess;
    const int nblk = springs_blocks(sp, P);
    MB_LAUNCH(tg, K_SPRINGS_ADJ, s, k_springs_adjoint, nblk, BLK,
              springs_adjoint_lds(sp), sp, q, Fbar, P, qbar, kbar, r0bar, part);
    if (part && (kbar || r0bar)) {
        const int nent = 1 + sp.npairs;
        hipLaunchKernelGGL(k_sum_parts, dim3(blocks_for(nent)), dim3(BLK), 0, s, part, nblk,
                           nent, kbar, r0bar);
    }
    return hipGetLastError();
}

size_t springs_adjoint_part_size(const SpringsDev& sp, int64_t P) {
    return (size_t)springs_blocks(sp, P) * (1 + sp.npairs);
}

hipError_t zero_words(void* p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for((int64_t)n)), dim3(BLK), 0, s, (uint32_t*)p,
                       (int64_t)n);
    return hipGetLastError();
}

hipError_t init_workspace(mb_grid* g, hipStream_t s) {
    const int L = g->L;
    if (g->fsz == 4)
        hipLaunchKernelGGL(k_fft_tables<float>, dim3(blocks_for(L)), dim3(BLK), 0, s, L,
                           g->d.h, (float*)g->d_tw, (float*)g->d_dsym, (float*)g->d_d2);
    else
        hipLaunchKernelGGL(k_fft_tables<double>, dim3(blocks_for(L)), dim3(BLK), 0, s, L,
                           g->d.h, (double*)g->d_tw, (double*)g->d_dsym, (double*)g->d_d2);
    const size_t nt = (size_t)g->ntiles_cap * g->tiles.nbox;
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = zero_words(g->d_count, nt, s);
    if (e == hipSuccess) e = zero_words(g->d_tile_part, nt * 4 * 2, s);
    if (e == hipSuccess) e = zero_words(g->d_force_part, (size_t)g->force_blocks_cap * 3 * 2, s);
    if (e == hipSuccess) e = zero_words(g->d_flag, 2, s);
    return e;
}

hipError_t blob_axpy(int64_t n, const double* a, double sc, const double* b, double* out,
                     hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(BLK), 0, s, n, a, sc, b, out);
    return hipGetLastError();
}

hipError_t blob_add(int64_t n, const double* x, double* y, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add, dim3(blocks_for(n)), dim3(BLK), 0, s, n, x, y);
    return hipGetLastError();
}

template <typename T>
hipError_t apply_cn(mb_grid* g, const T* x, T* y, hipStream_t s) {
    const double h = g->d.h;
    const T c0 = (T)(g->d.rho / g->d.dt);
    const T c1 = (T)(0.5 * g->d.eta / (h * h));
    hipLaunchKernelGGL(k_apply_cn<T>, dim3(blocks_for(3 * g->N * g->tiles.nbox)), dim3(BLK), 0,
                       s, g->L, g->tiles.nbox, c0, c1, x, y);
    return hipGetLastError();
}
template hipError_t apply_cn<float>(mb_grid*, const float*, float*, hipStream_t);
template hipError_t apply_cn<double>(mb_grid*, const double*, double*, hipStream_t);

int springs_blocks(const SpringsDev& sp, int64_t P) {
    return (int)((P + sp.ppb - 1) / sp.ppb);
}

size_t springs_lds(const SpringsDev& sp) {
    return (size_t)sp.ppb * sp.nb * 3 * sizeof(double) + (size_t)sp.npairs * sizeof(double) +
           (size_t)(sp.nb + 1 + 2 * sp.npairs) * sizeof(int);
}

// Tile shapes with instantiated spreading and interpolation kernels (cells
// per axis; each a power of two dividing L).  fn receives the extents as
// integral constants; false when the shape has no kernels.
template <typename Fn>
static bool with_tile_shape(const Tiles& t, Fn&& fn) {
#define MB_SHAPE(X, Y, Z)                                                         \
    if (t.tx == X && t.ty == Y && t.tz == Z) {                                    \
        fn(std::integral_constant<int, X>{}, std::integral_constant<int, Y>{},    \
           std::integral_constant<int, Z>{});                                     \
        return true;                                                              \
    }
    MB_TILE_SHAPES(MB_SHAPE)
#undef MB_SHAPE
    return false;
}

bool tile_shape_supported(int tx, int ty, int tz) {
#define MB_SHAPE(X, Y, Z) if (tx == X && ty == Y && tz == Z) return true;
    MB_TILE_SHAPES(MB_SHAPE)
#undef MB_SHAPE
    return false;
}

// Box tiles with instantiated spreading kernels: (box tile extents, binning
// tiles per box tile along x, y, z).  box_tiles picks them.
#define MB_BOX_SHAPES(X)                                                     \
    X(16, 16, 16, 1, 2, 2) X(16, 16, 16, 2, 2, 2) X(16, 16, 16, 1, 1, 2)     \
    X(16, 16, 16, 1, 2, 1) X(16, 16, 16, 2, 1, 1) X(32, 8, 16, 1, 1, 2)      \
    X(8, 8, 8, 1, 1, 1) X(16, 8, 8, 1, 1, 1) X(32, 8, 8, 1, 1, 1)            \
    X(16, 16, 8, 1, 1, 1) X(16, 8, 16, 1, 1, 1) X(8, 16, 16, 1, 1, 1)

template <typename T>
hipError_t spread_boxes(mb_grid* g, hipStream_t s) {
    const Tiles& t = g->tiles;
    const Tiles& b = g->btiles;
    bool ok = false;
#define MB_BOX(SX, SY, SZ, FX, FY, FZ)                                                   \
    if (!ok && b.tx == SX && b.ty == SY && b.tz == SZ && SX == FX * t.tx &&              \
        SY == FY * t.ty && SZ == FZ * t.tz) {                                            \
        MB_LAUNCH(g, K_SPREAD, s, (k_spread<T, SX, SY, SZ, FX, FY, FZ>), b.n * b.nbox,   \
                  spread_threads<T>(FX * FY * FZ), 0, rec_geo<T>(g), rec_force<T>(g),    \
                  g->d_offs, g->L, b, t, g->d.deterministic, (T*)g->d_box);              \
        ok = true;                                                                       \
    }
    MB_BOX_SHAPES(MB_BOX)
#undef MB_BOX
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

bool box_shape_supported(int sx, int sy, int sz, int tx, int ty, int tz) {
#define MB_BOX(SX, SY, SZ, FX, FY, FZ) \
    if (sx == SX && sy == SY && sz == SZ && SX == FX * tx && SY == FY * ty && SZ == FZ * tz) return true;
    MB_BOX_SHAPES(MB_BOX)
#undef MB_BOX
    return false;
}

template <typename T>
hipError_t fold_boxes(mb_grid* g, T* f, hipStream_t s, const T* add) {
    MB_LAUNCH(g, K_FOLD, s, k_fold<T>, blocks_for(3 * g->N * g->tiles.nbox), BLK, 0,
              (const T*)g->d_box, g->L, g->btiles, add, f);
    return hipGetLastError();
}

template <typename T>
hipError_t interpolate(mb_grid* g, int64_t M, const T* v, double* u_out,
                       double* q_update, int diag, hipStream_t s, double uscale,
                       bool bin_next) {
    (void)M;
    double* part = diag ? g->d_tile_part : nullptr;
    const int kid = q_update ? K_INTERP_STEP : K_INTERP;
    BinNext bn{nullptr, nullptr, nullptr};
    if (bin_next && q_update) bn = BinNext{g->d_count, g->d_tile, g->d_rank};
    const bool ok = with_tile_shape(g->tiles, [&](auto X, auto Y, auto Z) {
        MB_LAUNCH(g, kid, s, (k_interp<T, decltype(X)::value, decltype(Y)::value, decltype(Z)::value>),
                  g->tiles.n * g->tiles.nbox,
                  interp_threads(decltype(X)::value * decltype(Y)::value * decltype(Z)::value),
                  0, rec_geo<T>(g), g->d_perm,
                  g->d_offs, g->L, g->tiles, v, u_out, uscale, q_update, g->d.dt,
                  1.0 / g->d.h, part, bn);
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}

template <typename T>
hipError_t interpolate_grad(mb_grid* g, const T* v, const double* W, double wscale,
                            double* gout, hipStream_t s) {
    const bool ok = with_tile_shape(g->tiles, [&](auto X, auto Y, auto Z) {
        MB_LAUNCH(g, K_INTERP_GRAD, s, (k_interp_grad<T, decltype(X)::value, decltype(Y)::value, decltype(Z)::value>),
                  g->tiles.n * g->tiles.nbox, BLK, 0, rec_geo<T>(g), g->d_perm,
                  g->d_offs, g->L, g->tiles, v, W, wscale, 1.0 / g->d.h, gout);
    });
    return ok ? hipGetLastError() : hipErrorInvalidValue;
}


hipError_t particle_means(mb_grid* g, int64_t P, int nb, const double* u,
                          double* U0, hipStream_t s) {
    if (P == 0) return hipSuccess;
    MB_LAUNCH(g, K_U0, s, k_u0, blocks_for(P), BLK, 0, u, P, nb, U0);
    return hipGetLastError();
}

hipError_t diagnostics(mb_grid* g, int force_blocks, double* diag,
                       hipStream_t s) {
    const double h = g->d.h;
    const double scale = g->d.rho * h * h * h;
    MB_LAUNCH(g, K_DIAG, s, k_diag, 1, BLK, 0, g->d_tile_part, g->tiles.n * g->tiles.nbox,
              g->d_force_part, force_blocks, scale, diag);
    return hipGetLastError();
}

// Explicit instantiations.
template hipError_t bin_blobs<float>(mb_grid*, int64_t, const double*, hipStream_t, bool, bool);
template hipError_t bin_blobs<double>(mb_grid*, int64_t, const double*, hipStream_t, bool, bool);
template hipError_t scatter_records<float>(mb_grid*, int64_t, const double*, const double*, hipStream_t, double);
template hipError_t scatter_records<double>(mb_grid*, int64_t, const double*, const double*, hipStream_t, double);
template hipError_t scatter_springs<float>(mb_grid*, const SpringsDev&, int64_t, const double*, const double*, hipStream_t, const double*, bool, bool);
template hipError_t scatter_springs<double>(mb_grid*, const SpringsDev&, int64_t, const double*, const double*, hipStream_t, const double*, bool, bool);
template hipError_t spread_boxes<float>(mb_grid*, hipStream_t);
template hipError_t spread_boxes<double>(mb_grid*, hipStream_t);
template hipError_t fold_boxes<float>(mb_grid*, float*, hipStream_t, const float*);
template hipError_t fold_boxes<double>(mb_grid*, double*, hipStream_t, const double*);
template hipError_t interpolate<float>(mb_grid*, int64_t, const float*, double*, double*, int, hipStream_t, double, bool);
template hipError_t interpolate<double>(mb_grid*, int64_t, const double*, double*, double*, int, hipStream_t, double, bool);
template hipError_t interpolate_grad<float>(mb_grid*, const float*, const double*, double, double*, hipStream_t);
template hipError_t interpolate_grad<double>(mb_grid*, const double*, const double*, double, double*, hipStream_t);

size_t box_elems(const Tiles& t) {
    return (size_t)3 * t.nbox * t.n * (t.tx + 3) * (t.ty + 3) * (t.tz + 3);
}

size_t record_size(int precision) {
    return precision == MB_MIXED ? sizeof(RecG<float>) + 3 * sizeof(float)
                                 : sizeof(RecG<double>) + 3 * sizeof(double);
}

}  // namespace mb
