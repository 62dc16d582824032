// Spread boxes: the per-tile partial force fields written by the spreading
// kernel, and the sum over the boxes that hold a node.
#pragma once

#include <hip/hip_runtime.h>

#include "mb_device.h"
#include "mb_internal.h"

namespace mb {

// Box entries holding node v of one axis, for tiles of extent T (nt of them):
// the node's own tile at box index l + 1 (l = v mod T), the previous tile at
// l + T + 1 when l <= 1 and the next tile at 0 when l = T - 1 (periodic in
// the tile index; T a power of two >= 4).  Each entry is stored as an
// element offset: tile * tstride + box index * bstride.
struct AxisSrc {
    int n;
    int off[2];
};

__device__ __forceinline__ AxisSrc axis_sources(int v, int T, int nt, int tstride,
                                                int bstride) {
    const int t = v >> (__ffs(T) - 1);
    const int l = v & (T - 1);
    AxisSrc s;
    s.n = 1;
    s.off[0] = t * tstride + (l + 1) * bstride;
    s.off[1] = 0;
    if (l <= 1) {
        s.n = 2;
        s.off[1] = (t == 0 ? nt - 1 : t - 1) * tstride + (l + T + 1) * bstride;
    } else if (l == T - 1) {
        s.n = 2;
        s.off[1] = (t == nt - 1 ? 0 : t + 1) * tstride;
    }
    return s;
}

// Elements of one tile's box.
__device__ __forceinline__ int box_volume(const Tiles& tl) {
    return (tl.tx + 3) * (tl.ty + 3) * (tl.tz + 3);
}

// Sources of a node along x, y and z of the box array.
__device__ __forceinline__ AxisSrc box_src_x(const Tiles& tl, int x) {
    return axis_sources(x, tl.tx, tl.ntx, box_volume(tl), 1);
}
__device__ __forceinline__ AxisSrc box_src_y(const Tiles& tl, int y) {
    return axis_sources(y, tl.ty, tl.nty, tl.ntx * box_volume(tl), tl.tx + 3);
}
__device__ __forceinline__ AxisSrc box_src_z(const Tiles& tl, int z) {
    return axis_sources(z, tl.tz, tl.ntz, tl.nty * tl.ntx * box_volume(tl),
                        (tl.tx + 3) * (tl.ty + 3));
}

// Sum of the entries of component array Ea (E + a * tiles * box volume)
// holding the node with the given sources, formed so that the loads of a
// node are issued together: an absent x, y or z source reads the node's own
// entry again and is multiplied by zero.
template <typename T>
__device__ __forceinline__ T box_sum(const T* __restrict__ Ea, const AxisSrc& sx,
                                     const AxisSrc& sy, const AxisSrc& sz) {
    const int x0 = sx.off[0];
    const int x1 = sx.n > 1 ? sx.off[1] : x0;
    const T mx = sx.n > 1 ? T(1) : T(0);
    const int y1 = sy.n > 1 ? sy.off[1] : sy.off[0];
    const int z1 = sz.n > 1 ? sz.off[1] : sz.off[0];
    const T my = sy.n > 1 ? T(1) : T(0);
    const T mz = sz.n > 1 ? T(1) : T(0);
#define MB_ROW(o) (Ea[(o) + x0] + mx * Ea[(o) + x1])
    const T r0 = MB_ROW(sz.off[0] + sy.off[0]);
    const T r1 = MB_ROW(sz.off[0] + y1);
    const T r2 = MB_ROW(z1 + sy.off[0]);
    const T r3 = MB_ROW(z1 + y1);
#undef MB_ROW
    return (r0 + my * r1) + mz * (r2 + my * r3);
}

// The entries of component array Ea holding a node, loaded without
// arithmetic: e[s][0] (first x source) and e[s][1] (second x source, lane
// masked) for the (z, y) source pairs s = 0 (z0, y0), 1 (z0, y1), 2 (z1, y0),
// 3 (z1, y1); pairs absent from the node are not loaded and stay zero.  The
// y and z counts are uniform over the wave when the lanes share y and z, so
// the branches do not diverge, and since nothing is added inside them the
// loads of several nodes stay in flight together; box_entries_sum then adds
// them in the order of box_sum.
template <typename T>
__device__ __forceinline__ void box_entries(const T* __restrict__ Ea, const AxisSrc& sx,
                                            const AxisSrc& sy, const AxisSrc& sz,
                                            T e[4][2]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) e[k][0] = e[k][1] = T(0);
    const unsigned x0 = (unsigned)sx.off[0], x1 = (unsigned)sx.off[1];
    const unsigned o0 = (unsigned)(sz.off[0] + sy.off[0]);
    e[0][0] = ld32(Ea, o0 + x0);
    if (sx.n > 1) e[0][1] = ld32(Ea, o0 + x1);
    if (sy.n > 1) {
        const unsigned o1 = (unsigned)(sz.off[0] + sy.off[1]);
        e[1][0] = ld32(Ea, o1 + x0);
        if (sx.n > 1) e[1][1] = ld32(Ea, o1 + x1);
    }
    if (sz.n > 1) {
        const unsigned o2 = (unsigned)(sz.off[1] + sy.off[0]);
        e[2][0] = ld32(Ea, o2 + x0);
        if (sx.n > 1) e[2][1] = ld32(Ea, o2 + x1);
        if (sy.n > 1) {
            const unsigned o3 = (unsigned)(sz.off[1] + sy.off[1]);
            e[3][0] = ld32(Ea, o3 + x0);
            if (sx.n > 1) e[3][1] = ld32(Ea, o3 + x1);
        }
    }
}
template <typename T>
__device__ __forceinline__ T box_entries_sum(const T e[4][2]) {
    return ((e[0][0] + e[0][1]) + (e[1][0] + e[1][1])) +
           ((e[2][0] + e[2][1]) + (e[3][0] + e[3][1]));
}

// Node (x, y, z) of component a.
template <typename T>
__device__ __forceinline__ T box_sum(const T* __restrict__ E, const Tiles& tl,
                                     int a, int x, int y, int z) {
    const T* Ea = E + (size_t)a * tl.n * box_volume(tl);
    return box_sum(Ea, box_src_x(tl, x), box_src_y(tl, y), box_src_z(tl, z));
}


}  // namespace mb
