// HIP kernels of the multiblob step for gfx950 and their launchers.
//
// Per step: blobs are counting-sorted by cell (count, scan, scatter with the
// spring forces), spread tile by tile with LDS accumulation, the fluid is
// solved by a hand-written 3-D FFT (x pass with the Crank-Nicolson
// right-hand side fused in, y pass, z pass fused with the projection and
// the viscous divide, inverse y, inverse x), and the new velocity is
// interpolated tile by tile from an LDS copy of the field, moving the blobs.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "mb_device.h"
#include "mb_internal.h"

namespace mb {

// Sorted-blob record: kernel offsets for the cell-centred (tu) and the
// component's own, half-cell shifted (ts) node sets, the force scaled by
// h^-3, and the packed cell: bits 0-8 x, 9-17 y, 18-26 z, 27-29 the
// "rounds up" bit per axis (node i0 = c + bit for the cell-centred set).
template <typename T>
struct __align__(16) Rec {
    T tu[3];
    T ts[3];
    T F[3];
    uint32_t cell;
    uint32_t pad;
};

constexpr int BLK = 256;

struct Geom {
    int c[3];
    int up[3];
    double tu[3];
    double ts[3];
};

// Cell, rounding bits and kernel offsets of a position (float64).  For the
// node set of velocity component a along axis b the node coordinate is
// x = q_b/h - (1/2) delta_ab; the nearest node is i0 = floor(x + 1/2) and
// t = x - i0 in [-1/2, 1/2).
__device__ __forceinline__ Geom blob_geom(const double* __restrict__ q,
                                          int64_t i, double h, int L) {
    Geom g;
    const double Ld = (double)L;
    const double invL = 1.0 / Ld;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const double x = q[3 * i + b] / h;
        const double fl = floor(x);
        const double s = x - fl;  // [0, 1)
        // fl mod L without integer division: exact for |fl| < 2^53, the
        // rounded quotient is off by at most one and corrected
        double c = fl - floor(fl * invL) * Ld;
        if (c < 0.0) c += Ld;
        if (c >= Ld) c -= Ld;
        g.c[b] = (int)c;
        g.up[b] = s >= 0.5 ? 1 : 0;
        g.tu[b] = s - (double)g.up[b];
        g.ts[b] = s - 0.5;
    }
    return g;
}

// Bin of a blob: blobs are sorted by 2x2x2 groups of cells ("bins"),
// (L/2)^3 of them, x fastest.
__device__ __forceinline__ int bin_linear(const Geom& g, int L) {
    const int Lb = L >> 1;
    return ((g.c[2] >> 1) * Lb + (g.c[1] >> 1)) * Lb + (g.c[0] >> 1);
}

__device__ __forceinline__ uint32_t cell_pack(const Geom& g) {
    return (uint32_t)g.c[0] | ((uint32_t)g.c[1] << 9) | ((uint32_t)g.c[2] << 18) |
           ((uint32_t)g.up[0] << 27) | ((uint32_t)g.up[1] << 28) |
           ((uint32_t)g.up[2] << 29);
}

// ---------------------------------------------------------------------------
// Binning: counting sort of blobs by cell.
__global__ void __launch_bounds__(BLK)
k_bin_count(const double* __restrict__ q, int64_t M, double h, int L,
            int* __restrict__ count, int* __restrict__ rank,
            unsigned int* __restrict__ fmax) {
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    if (i == 0) *fmax = 0u;  // max |F h^-3| of this step, set by the scatter
    if (i >= M) return;
    const Geom g = blob_geom(q, i, h, L);
    rank[i] = atomicAdd(&count[bin_linear(g, L)], 1);
}

constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = BLK * SCAN_ITEMS;  // 4096

__device__ __forceinline__ int scan_pad(int i) { return i + (i >> 5); }

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

// offs[i] = exclusive prefix of count; offs[n] = total; count reset to 0.
// Each block adds the sums of the blocks before it (a few hundred at most).
__global__ void __launch_bounds__(BLK)
k_scan_apply(int* __restrict__ count, int64_t n, const int* __restrict__ bsum,
             int* __restrict__ offs) {
    __shared__ int s[SCAN_TILE + SCAN_TILE / 32];
    __shared__ int scratch[16];
    __shared__ double red[16];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    int before = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += BLK) before += bsum[b];
    const int off = (int)block_reduce<false>((double)before, red);
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int i = k * BLK + threadIdx.x;
        s[scan_pad(i)] = (base + i < n) ? count[base + i] : 0;
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

// Writes the record and returns the largest |F h^-3| it stores (as float).
template <typename T>
__device__ __forceinline__ float write_record(Rec<T>* __restrict__ rec,
                                              int* __restrict__ perm,
                                              int64_t pos, int64_t i,
                                              const Geom& g, const double F[3],
                                              double inv_vol) {
    Rec<T> r;
    float m = 0.f;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        r.tu[b] = (T)g.tu[b];
        r.ts[b] = (T)g.ts[b];
        r.F[b] = (T)(F[b] * inv_vol);
        m = fmaxf(m, fabsf((float)r.F[b]));
    }
    r.cell = cell_pack(g);
    r.pad = 0;
    rec[pos] = r;
    perm[pos] = (int)i;
    return m;
}

// Block maximum of non-negative floats folded into *fmax (bit patterns of
// non-negative floats order like the values).
__device__ __forceinline__ void fold_fmax(float m, double* red,
                                          unsigned int* __restrict__ fmax) {
    const double bm = block_reduce<true>((double)m, red);
    if (threadIdx.x == 0) atomicMax(fmax, __float_as_uint((float)bm));
}

// Records in cell order for given forces (F may be null: interpolation).
template <typename T>
__global__ void __launch_bounds__(BLK)
k_bin_scatter(const double* __restrict__ q, const double* __restrict__ F,
              int64_t M, double h, int L, double inv_vol,
              const int* __restrict__ offs, const int* __restrict__ rank,
              Rec<T>* __restrict__ rec, int* __restrict__ perm,
              unsigned int* __restrict__ fmax) {
    __shared__ double red[16];
    const int64_t i = (int64_t)blockIdx.x * BLK + threadIdx.x;
    float m = 0.f;
    if (i < M) {
        const Geom g = blob_geom(q, i, h, L);
        double f[3] = {0.0, 0.0, 0.0};
        if (F) {
            f[0] = F[3 * i];
            f[1] = F[3 * i + 1];
            f[2] = F[3 * i + 2];
        }
        const int64_t pos = (int64_t)offs[bin_linear(g, L)] + rank[i];
        m = write_record<T>(rec, perm, pos, i, g, f, inv_vol);
    }
    fold_fmax(m, red, fmax);
}

// Spring forces of the sp.ppb particles of this block (float64).  Their
// blob positions are loaded into LDS once; each pair force of every
// particle, s d with d = q_b - q_a and s = k (|d| - r0) / |d|, is computed
// once; then thread j (< nblob) sums the incident pair forces of its blob
// (+s d on pair_a, -s d on pair_b) plus Fext_p / nb.  Returns the number of
// blobs of the block; F holds thread j's blob force.
__device__ __forceinline__ int springs_block(const SpringsDev& sp,
                                             const double* __restrict__ q,
                                             const double* __restrict__ Fext,
                                             int64_t P, double* smem,
                                             double F[3], int64_t* blob) {
    const int nb = sp.nb, np = sp.npairs;
    const int64_t p0 = (int64_t)blockIdx.x * sp.ppb;
    const int npart = (int)(P - p0 < sp.ppb ? P - p0 : sp.ppb);
    const int nblob = npart * nb;
    double* qs = smem;                     // [ppb * nb][3]
    double* fp = smem + 3 * sp.ppb * nb;   // [ppb * np][3]
    double* r0s = fp + 3 * sp.ppb * np;    // [np]
    int* pab = (int*)(r0s + np);           // [np] packed pair_a | pair_b << 16
    const double* qg = q + 3 * p0 * nb;    // contiguous blobs of the block
    for (int i = threadIdx.x; i < 3 * nblob; i += BLK) qs[i] = qg[i];
    for (int e = threadIdx.x; e < np; e += BLK) {
        r0s[e] = sp.r0[e];
        pab[e] = sp.pa[e] | (sp.pb[e] << 16);
    }
    __syncthreads();
    for (int w = threadIdx.x; w < npart * np; w += BLK) {
        const int pl = w / np;
        const int e = w - pl * np;
        const int ab = pab[e];
        const double* qa = qs + 3 * (pl * nb + (ab & 0xffff));
        const double* qb = qs + 3 * (pl * nb + (ab >> 16));
        const double dx = qb[0] - qa[0], dy = qb[1] - qa[1], dz = qb[2] - qa[2];
        const double len = sqrt(dx * dx + dy * dy + dz * dz);
        const double s = sp.k * (len - r0s[e]) / len;
        fp[3 * w] = s * dx;
        fp[3 * w + 1] = s * dy;
        fp[3 * w + 2] = s * dz;
    }
    __syncthreads();
    F[0] = F[1] = F[2] = 0.0;
    *blob = -1;
    const int j = threadIdx.x;
    if (j < nblob) {
        const int pl = j / nb;
        const int b = j - pl * nb;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        if (Fext) {
            const double inv_nb = 1.0 / (double)nb;
            const double* fe = Fext + 3 * (p0 + pl);
            fx = fe[0] * inv_nb;
            fy = fe[1] * inv_nb;
            fz = fe[2] * inv_nb;
        }
        const int e1 = sp.adj_start[b + 1];
        for (int x = sp.adj_start[b]; x < e1; ++x) {
            const int code = sp.adj_pair[x];
            const int e = (code > 0 ? code : -code) - 1;
            const double* f = fp + 3 * (pl * np + e);
            if (code > 0) {
                fx += f[0];
                fy += f[1];
                fz += f[2];
            } else {
                fx -= f[0];
                fy -= f[1];
                fz -= f[2];
            }
        }
        F[0] = fx;
        F[1] = fy;
        F[2] = fz;
        *blob = p0 * nb + j;
    }
    return nblob;
}

// Spring forces fused with the scatter of the records; also the per-block
// float64 sums of the blob forces (momentum diagnostics) and max |F h^-3|.
template <typename T>
__global__ void __launch_bounds__(BLK)
k_springs_scatter(SpringsDev sp, const double* __restrict__ q,
                  const double* __restrict__ Fext, int64_t P, double h, int L,
                  double inv_vol, const int* __restrict__ offs,
                  const int* __restrict__ rank, Rec<T>* __restrict__ rec,
                  int* __restrict__ perm, double* __restrict__ fpart,
                  unsigned int* __restrict__ fmax) {
    extern __shared__ double smem[];
    __shared__ double red[16];
    double F[3];
    int64_t i;
    springs_block(sp, q, Fext, P, smem, F, &i);
    float m = 0.f;
    if (i >= 0) {
        const Geom g = blob_geom(q, i, h, L);
        const int64_t pos = (int64_t)offs[bin_linear(g, L)] + rank[i];
        m = write_record<T>(rec, perm, pos, i, g, F, inv_vol);
    }
    fold_fmax(m, red, fmax);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double s = block_reduce<false>(F[c], red);
        if (threadIdx.x == 0) fpart[3 * blockIdx.x + c] = s;
    }
}

__global__ void __launch_bounds__(BLK)
k_springs(SpringsDev sp, const double* __restrict__ q,
          const double* __restrict__ Fext, int64_t P, double* __restrict__ Fout) {
    extern __shared__ double smem[];
    double F[3];
    int64_t i;
    springs_block(sp, q, Fext, P, smem, F, &i);
    if (i < 0) return;
    Fout[3 * i] = F[0];
    Fout[3 * i + 1] = F[1];
    Fout[3 * i + 2] = F[2];
}

// ---------------------------------------------------------------------------
// Tile helpers shared by spreading and interpolation.
struct TileBox {
    int lo[3];
    int full[3];
};

__device__ __forceinline__ TileBox tile_box(const Tiles& t, int L) {
    int b = blockIdx.x;
    if (t.remap) b = xcd_remap(b, t.n);
    TileBox tb;
    const int ix = b % t.ntx;
    const int iy = (b / t.ntx) % t.nty;
    const int iz = b / (t.ntx * t.nty);
    tb.lo[0] = ix * t.tx;
    tb.lo[1] = iy * t.ty;
    tb.lo[2] = iz * t.tz;
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

// Contiguous ranges of sorted records for the cells of a box of rows.
// Rows y in [ylo, ylo + ny), z in [zlo, zlo + nz) (wrapped), x cells
// [xlo, xlo + nx) (wrapped, split in at most two runs).  Fills seg_start /
// seg_pre (exclusive prefix of lengths) and returns the record count.
__device__ int gather_segments(const int* __restrict__ offs, int L, int xlo,
                               int nx, int ylo, int ny, int zlo, int nz,
                               int* seg_start, int* seg_pre, int* scratch,
                               int* nseg_out) {
    // x runs
    int xs0 = wrapL(xlo, L), xe0, xs1 = 0, xe1 = -1, nxs = 1;
    if (nx >= L) {
        xs0 = 0;
        xe0 = L - 1;
    } else if (xs0 + nx - 1 < L) {
        xe0 = xs0 + nx - 1;
    } else {
        xe0 = L - 1;
        xs1 = 0;
        xe1 = xs0 + nx - 1 - L;
        nxs = 2;
    }
    const int nseg = ny * nz * nxs;
    // one segment per thread per pass; nseg <= blockDim.x * passes
    int carry = 0;
    for (int base = 0; base < nseg; base += blockDim.x) {
        const int s = base + threadIdx.x;
        int len = 0;
        if (s < nseg) {
            const int xi = s % nxs;
            const int r = s / nxs;
            const int y = wrapL(ylo + r % ny, L);
            const int z = wrapL(zlo + r / ny, L);
            const int row = (z * L + y) * L;
            const int a = row + (xi ? xs1 : xs0);
            const int e = row + (xi ? xe1 : xe0);
            const int st = offs[a];
            len = offs[e + 1] - st;
            seg_start[s] = st;
        }
        int total;
        const int ex = block_exclusive_scan(len, scratch, &total);
        if (s < nseg) seg_pre[s] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) seg_pre[nseg] = carry;
    __syncthreads();
    *nseg_out = nseg;
    return carry;
}

__device__ __forceinline__ int find_segment(const int* seg_pre, int nseg, int k) {
    int lo = 0, hi = nseg - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_pre[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Adds one record's contributions to the in-tile nodes of all three
// components.  ACC = double: float64 LDS atomics on the float64 path.
// ACC = unsigned long long (mixed path): each float32 contribution, already
// scaled by 2^e, is rounded to int32 and added to a 64-bit integer sum.
template <typename T, typename ACC, int TX, int TY, int TZ>
__device__ __forceinline__ void spread_record(const Rec<T>& r, const TileBox& tb,
                                              const int* tdim, int L, int e,
                                              ACC* acc) {
    constexpr int TV = TX * TY * TZ;
    T w[3][2][3];     // per axis, node set (0 cell-centred, 1 shifted), node
    int rel[3][2][3]; // tile-relative node index, -1 outside the tile
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        kernel_weights<T>(r.tu[b], w[b][0]);
        kernel_weights<T>(r.ts[b], w[b][1]);
        const int cb = (int)((r.cell >> (9 * b)) & 511u);
        const int up = (int)((r.cell >> (27 + b)) & 1u);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            int r0 = cb + (v == 0 ? up : 0) - 1 - tb.lo[b];
            if (r0 < 0) r0 += L;
            if (r0 >= L) r0 -= L;
#pragma unroll
            for (int o = 0; o < 3; ++o) {
                int rr = r0 + o;
                if (rr >= L) rr -= L;
                rel[b][v][o] = rr < tdim[b] ? rr : -1;
            }
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int vx = a == 0, vy = a == 1, vz = a == 2;
        T Fa = r.F[a];
        if constexpr (!std::is_same<ACC, double>::value) Fa = ldexp(Fa, e);
        ACC* A = acc + a * TV;
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
            const int rz = rel[2][vz][oz];
            if (rz < 0) continue;
            const T wz = w[2][vz][oz] * Fa;
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                const int ry = rel[1][vy][oy];
                if (ry < 0) continue;
                const T wyz = w[1][vy][oy] * wz;
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    const int rx = rel[0][vx][ox];
                    if (rx < 0) continue;
                    const T val = w[0][vx][ox] * wyz;
                    ACC* dst = &A[(rz * TY + ry) * TX + rx];
                    if constexpr (std::is_same<ACC, double>::value)
                        atomicAdd(dst, (double)val);
                    else
                        atomicAdd(dst, (unsigned long long)(long long)__float2int_rn((float)val));
                }
            }
        }
    }
}

// Spreading: one block per tile; every record whose 3x3x3 support may reach
// the tile (cells [lo-2, hi+1]) is expanded and its in-tile nodes are added
// to an LDS copy of the tile, which is then written out once.
//
// Accumulation: float64 LDS atomics on the float64 path.  On the mixed path
// the float LDS atomic add of gfx950 is an order of magnitude slower than
// the integer one, so the float32 contributions are accumulated as fixed
// point: with fmax the largest |F h^-3| of the step and 2^e the power of two
// with fmax 2^e < 2^30, each contribution w F 2^e is rounded to int32 (a
// quantum of at most 2^-29 fmax) and summed in 64-bit integers, which can
// not overflow and do not depend on the order of the additions.
template <typename T, typename ACC, int TX, int TY, int TZ>
__global__ void __launch_bounds__(BLK)
k_spread(const Rec<T>* __restrict__ rec, const int* __restrict__ offs, int L,
         Tiles tl, const float* __restrict__ fmax, T* __restrict__ f) {
    constexpr int TV = TX * TY * TZ;
    constexpr bool FIXED = !std::is_same<ACC, double>::value;
    __shared__ ACC acc[3 * TV];
    __shared__ int seg_start[2 * (TY / 2 + 2) * (TZ / 2 + 2)];
    __shared__ int seg_pre[2 * (TY / 2 + 2) * (TZ / 2 + 2) + 1];
    __shared__ int scratch[16];
    const TileBox tb = tile_box(tl, L);
    const int tdim[3] = {tl.tx, tl.ty, tl.tz};
    for (int i = threadIdx.x; i < 3 * TV; i += BLK) acc[i] = ACC(0);
    int e = 0;
    if (FIXED) {
        const float fm = *fmax;
        if (fm > 0.f) {
            int ex;
            (void)frexpf(fm, &ex);  // fm < 2^ex
            e = 30 - ex;
        }
    }
    // bins (2x2x2 cells) covering the cells [lo-2, hi+1] that can reach the
    // tile: bins [lo/2 - 1, (lo+T)/2] per axis (one spare cell layer above)
    int nseg;
    const int Lb = L >> 1;
    const int ext[3] = {tb.full[0] ? Lb : tl.tx / 2 + 2, tb.full[1] ? Lb : tl.ty / 2 + 2,
                        tb.full[2] ? Lb : tl.tz / 2 + 2};
    const int elo[3] = {tb.full[0] ? 0 : tb.lo[0] / 2 - 1, tb.full[1] ? 0 : tb.lo[1] / 2 - 1,
                        tb.full[2] ? 0 : tb.lo[2] / 2 - 1};
    const int total = gather_segments(offs, Lb, elo[0], ext[0], elo[1], ext[1],
                                      elo[2], ext[2], seg_start, seg_pre,
                                      scratch, &nseg);
    // Records are bin-sorted, so consecutive records hit the same nodes.
    // Lane l of a wave takes record l * span + j instead of 64 j + l: a
    // wave's atomics then land far apart in the tile (fewer same-address and
    // same-bank collisions).
    const int span = (total + WAVE - 1) / WAVE;
    for (int it = threadIdx.x; it < span * WAVE; it += BLK) {
        const int k = (it % WAVE) * span + it / WAVE;
        if (k >= total) continue;
        const int s = find_segment(seg_pre, nseg, k);
        const Rec<T> r = rec[seg_start[s] + (k - seg_pre[s])];
        spread_record<T, ACC, TX, TY, TZ>(r, tb, tdim, L, e, acc);
    }
    __syncthreads();
    const int64_t N = (int64_t)L * L * L;
    for (int i = threadIdx.x; i < 3 * TV; i += BLK) {
        const int a = i / TV;
        const int rem = i - a * TV;
        const int x = rem % TX;
        const int y = (rem / TX) % TY;
        const int z = rem / (TX * TY);
        T val;
        if constexpr (FIXED)
            val = (T)ldexp((double)(long long)acc[i], -e);
        else
            val = (T)acc[i];
        f[a * N + ((int64_t)(tb.lo[2] + z) * L + tb.lo[1] + y) * L + tb.lo[0] + x] = val;
    }
}

// Interpolation: one block per tile; the field on nodes [lo-1, hi+2] of all
// three components is staged in LDS, then every record of the tile's cells
// gathers its 27 nodes per component.  With q_update the blob is moved by
// dt*u; with diag the block also writes its float64 sum of each component
// and the max |Dv| over its cells.
template <typename T, int TX, int TY, int TZ>
__global__ void __launch_bounds__(BLK)
k_interp(const Rec<T>* __restrict__ rec, const int* __restrict__ perm,
         const int* __restrict__ offs, int L, Tiles tl, const T* __restrict__ v,
         double* __restrict__ u_out, double* __restrict__ q, double dt,
         double inv_h, double* __restrict__ part) {
    constexpr int EX = TX + 3, EY = TY + 3, EZ = TZ + 3;
    constexpr int EV = EX * EY * EZ;
    __shared__ T vt[3 * EV];
    __shared__ int seg_start[(TY / 2) * (TZ / 2)];
    __shared__ int seg_pre[(TY / 2) * (TZ / 2) + 1];
    __shared__ int scratch[16];
    __shared__ double red[16];
    const TileBox tb = tile_box(tl, L);
    const int N = L * L * L;  // 3 L^3 < 2^31 for L <= 512
    // the tile's own cells are exactly the bins [lo/2, (lo+T)/2)
    int nseg;
    const int total = gather_segments(offs, L >> 1, tb.lo[0] >> 1, tl.tx >> 1,
                                      tb.lo[1] >> 1, tl.ty >> 1, tb.lo[2] >> 1,
                                      tl.tz >> 1, seg_start, seg_pre, scratch, &nseg);
    for (int i = threadIdx.x; i < 3 * EV; i += BLK) {
        const int a = i / EV;
        const int rem = i - a * EV;
        const int ex = rem % EX;
        const int ey = (rem / EX) % EY;
        const int ez = rem / (EX * EY);
        const int x = wrapL(tb.lo[0] - 1 + ex, L);
        const int y = wrapL(tb.lo[1] - 1 + ey, L);
        const int z = wrapL(tb.lo[2] - 1 + ez, L);
        vt[i] = v[a * N + (z * L + y) * L + x];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < total; k += BLK) {
        const int s = find_segment(seg_pre, nseg, k);
        const int pos = seg_start[s] + (k - seg_pre[s]);
        const Rec<T> r = rec[pos];
        const int c[3] = {(int)(r.cell & 511u), (int)((r.cell >> 9) & 511u),
                          (int)((r.cell >> 18) & 511u)};
        T w[3][2][3];
        int e0[3][2];  // extended-tile index of node i0 - 1
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            kernel_weights<T>(r.tu[b], w[b][0]);
            kernel_weights<T>(r.ts[b], w[b][1]);
            const int up = (r.cell >> (27 + b)) & 1u;
            const int rc = c[b] - tb.lo[b];  // in [0, T)
            e0[b][0] = rc + up;              // (i0 - 1) - (lo - 1)
            e0[b][1] = rc;
        }
        double u[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int vx = a == 0, vy = a == 1, vz = a == 2;
            const T* V = vt + a * EV;
            T acc = T(0);
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) {
                const int z = e0[2][vz] + oz;
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                    const int y = e0[1][vy] + oy;
                    const T wyz = w[2][vz][oz] * w[1][vy][oy];
                    const T* row = V + (z * EY + y) * EX + e0[0][vx];
                    T sx = w[0][vx][0] * row[0] + w[0][vx][1] * row[1] + w[0][vx][2] * row[2];
                    acc += wyz * sx;
                }
            }
            u[a] = (double)acc;
        }
        const int64_t i = perm[pos];
        if (u_out) {
            u_out[3 * i] = u[0];
            u_out[3 * i + 1] = u[1];
            u_out[3 * i + 2] = u[2];
        }
        if (q) {
            q[3 * i] += dt * u[0];
            q[3 * i + 1] += dt * u[1];
            q[3 * i + 2] += dt * u[2];
        }
    }
    if (part) {
        double sv[3] = {0.0, 0.0, 0.0};
        double dmax = 0.0;
        const int TV = TX * TY * TZ;
        for (int i = threadIdx.x; i < TV; i += BLK) {
            const int x = i % TX + 1;
            const int y = (i / TX) % TY + 1;
            const int z = i / (TX * TY) + 1;
            const int c0 = (z * EY + y) * EX + x;
            const T vxc = vt[c0], vyc = vt[EV + c0], vzc = vt[2 * EV + c0];
            sv[0] += (double)vxc;
            sv[1] += (double)vyc;
            sv[2] += (double)vzc;
            const double dv = ((double)(vxc - vt[c0 - 1]) +
                               (double)(vyc - vt[EV + c0 - EX]) +
                               (double)(vzc - vt[2 * EV + c0 - EX * EY])) * inv_h;
            dmax = fmax(dmax, fabs(dv));
        }
        const int tile = tl.remap ? xcd_remap(blockIdx.x, tl.n) : blockIdx.x;
        for (int a = 0; a < 3; ++a) {
            const double s = block_reduce<false>(sv[a], red);
            if (threadIdx.x == 0) part[4 * tile + a] = s;
        }
        const double m = block_reduce<true>(dmax, red);
        if (threadIdx.x == 0) part[4 * tile + 3] = m;
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

template <typename T>
hipError_t bin_blobs(mb_grid* g, int64_t M, const double* q, hipStream_t s) {
    if (M > 0)
        MB_LAUNCH(g, K_BIN_COUNT, s, k_bin_count, blocks_for(M), BLK, 0, q, M,
                  g->d.h, g->L, g->d_count, g->d_rank, (unsigned int*)g->d_fmax);
    MB_LAUNCH(g, K_SCAN_REDUCE, s, k_scan_reduce, g->nscan, BLK, 0, g->d_count,
              g->nbins, g->d_bsum);
    MB_LAUNCH(g, K_SCAN_APPLY, s, k_scan_apply, g->nscan, BLK, 0, g->d_count,
              g->nbins, g->d_bsum, g->d_offs);
    return hipGetLastError();
}

template <typename T>
hipError_t scatter_records(mb_grid* g, int64_t M, const double* q,
                           const double* F, hipStream_t s) {
    if (M == 0) return hipSuccess;
    const double h = g->d.h;
    MB_LAUNCH(g, K_BIN_SCATTER, s, k_bin_scatter<T>, blocks_for(M), BLK, 0, q, F,
              M, h, g->L, 1.0 / (h * h * h), g->d_offs, g->d_rank,
              (Rec<T>*)g->d_rec, g->d_perm, (unsigned int*)g->d_fmax);
    return hipGetLastError();
}

template <typename T>
hipError_t scatter_springs(mb_grid* g, const SpringsDev& sp, int64_t P,
                           const double* q, const double* Fext, hipStream_t s) {
    const int64_t M = P * sp.nb;
    if (M == 0) return hipSuccess;
    const double h = g->d.h;
    MB_LAUNCH(g, K_SPRINGS_SCATTER, s, k_springs_scatter<T>, springs_blocks(sp, P), BLK,
              springs_lds(sp), sp, q, Fext, P, h, g->L, 1.0 / (h * h * h), g->d_offs,
              g->d_rank, (Rec<T>*)g->d_rec, g->d_perm, g->d_force_part,
              (unsigned int*)g->d_fmax);
    return hipGetLastError();
}

hipError_t spring_forces(const SpringsDev& sp, int64_t P, const double* q,
                         const double* Fext, double* F, hipStream_t s,
                         mb_grid* tg) {
    const int64_t M = P * sp.nb;
    if (M == 0) return hipSuccess;
    MB_LAUNCH(tg, K_SPRINGS, s, k_springs, springs_blocks(sp, P), BLK, springs_lds(sp),
              sp, q, Fext, P, F);
    return hipGetLastError();
}

int springs_blocks(const SpringsDev& sp, int64_t P) {
    return (int)((P + sp.ppb - 1) / sp.ppb);
}

size_t springs_lds(const SpringsDev& sp) {
    return (size_t)sp.ppb * (sp.nb + sp.npairs) * 3 * sizeof(double) +
           (size_t)sp.npairs * (sizeof(double) + sizeof(int));
}

template <typename T, int TX>
static void launch_spread(mb_grid* g, T* f, hipStream_t s) {
    using ACC = typename std::conditional<std::is_same<T, float>::value,
                                          unsigned long long, double>::type;
    MB_LAUNCH(g, K_SPREAD, s, (k_spread<T, ACC, TX, 8, 8>), g->tiles.n, BLK, 0,
              (const Rec<T>*)g->d_rec, g->d_offs, g->L, g->tiles,
              (const float*)g->d_fmax, f);
}

template <typename T>
hipError_t spread(mb_grid* g, T* f, hipStream_t s) {
    switch (g->tiles.tx) {
        case 32: launch_spread<T, 32>(g, f, s); break;
        case 16: launch_spread<T, 16>(g, f, s); break;
        default: launch_spread<T, 8>(g, f, s); break;
    }
    return hipGetLastError();
}

template <typename T, int TX>
static void launch_interp(mb_grid* g, const T* v, double* u_out, double* q,
                          double* part, int kid, hipStream_t s) {
    MB_LAUNCH(g, kid, s, (k_interp<T, TX, 8, 8>), g->tiles.n, BLK, 0,
              (const Rec<T>*)g->d_rec, g->d_perm, g->d_offs, g->L, g->tiles, v,
              u_out, q, g->d.dt, 1.0 / g->d.h, part);
}

template <typename T>
hipError_t interpolate(mb_grid* g, int64_t M, const T* v, double* u_out,
                       double* q_update, int diag, hipStream_t s) {
    (void)M;
    double* part = diag ? g->d_tile_part : nullptr;
    const int kid = q_update ? K_INTERP_STEP : K_INTERP;
    switch (g->tiles.tx) {
        case 32: launch_interp<T, 32>(g, v, u_out, q_update, part, kid, s); break;
        case 16: launch_interp<T, 16>(g, v, u_out, q_update, part, kid, s); break;
        default: launch_interp<T, 8>(g, v, u_out, q_update, part, kid, s); break;
    }
    return hipGetLastError();
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
    MB_LAUNCH(g, K_DIAG, s, k_diag, 1, BLK, 0, g->d_tile_part, g->tiles.n,
              g->d_force_part, force_blocks, scale, diag);
    return hipGetLastError();
}

// Explicit instantiations.
template hipError_t bin_blobs<float>(mb_grid*, int64_t, const double*, hipStream_t);
template hipError_t bin_blobs<double>(mb_grid*, int64_t, const double*, hipStream_t);
template hipError_t scatter_records<float>(mb_grid*, int64_t, const double*, const double*, hipStream_t);
template hipError_t scatter_records<double>(mb_grid*, int64_t, const double*, const double*, hipStream_t);
template hipError_t scatter_springs<float>(mb_grid*, const SpringsDev&, int64_t, const double*, const double*, hipStream_t);
template hipError_t scatter_springs<double>(mb_grid*, const SpringsDev&, int64_t, const double*, const double*, hipStream_t);
template hipError_t spread<float>(mb_grid*, float*, hipStream_t);
template hipError_t spread<double>(mb_grid*, double*, hipStream_t);
template hipError_t interpolate<float>(mb_grid*, int64_t, const float*, double*, double*, int, hipStream_t);
template hipError_t interpolate<double>(mb_grid*, int64_t, const double*, double*, double*, int, hipStream_t);

size_t record_size(int precision) {
    return precision == MB_MIXED ? sizeof(Rec<float>) : sizeof(Rec<double>);
}

}  // namespace mb
