// Spread boxes: the per-tile partial force fields written by the spreading
// kernel, and the sum over the boxes that hold a node.
#pragma once

#include <hip/hip_runtime.h>

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
// holding the node with the given sources, in a fixed order.
template <typename T>
__device__ __forceinline__ T box_sum(const T* __restrict__ Ea, const AxisSrc& sx,
                                     const AxisSrc& sy, const AxisSrc& sz) {
    // All loads are issued unconditionally (an absent source reads the
    // node's own entry and is dropped), so that they overlap.
    const int x1 = sx.n > 1 ? sx.off[1] : sx.off[0];
    const int y1 = sy.n > 1 ? sy.off[1] : sy.off[0];
    const int z1 = sz.n > 1 ? sz.off[1] : sz.off[0];
    const T v000 = Ea[sz.off[0] + sy.off[0] + sx.off[0]];
    const T v001 = Ea[sz.off[0] + sy.off[0] + x1];
    const T v010 = Ea[sz.off[0] + y1 + sx.off[0]];
    const T v011 = Ea[sz.off[0] + y1 + x1];
    const T v100 = Ea[z1 + sy.off[0] + sx.off[0]];
    const T v101 = Ea[z1 + sy.off[0] + x1];
    const T v110 = Ea[z1 + y1 + sx.off[0]];
    const T v111 = Ea[z1 + y1 + x1];
    const T zero = T(0);
    const bool hx = sx.n > 1, hy = sy.n > 1, hz = sz.n > 1;
    T s = v000;
    s += hx ? v001 : zero;
    s += hy ? v010 : zero;
    s += (hx && hy) ? v011 : zero;
    s += hz ? v100 : zero;
    s += (hz && hx) ? v101 : zero;
    s += (hz && hy) ? v110 : zero;
    s += (hz && hx && hy) ? v111 : zero;
    return s;
}

// Node (x, y, z) of component a.
template <typename T>
__device__ __forceinline__ T box_sum(const T* __restrict__ E, const Tiles& tl,
                                     int a, int x, int y, int z) {
    const T* Ea = E + (size_t)a * tl.n * box_volume(tl);
    return box_sum(Ea, box_src_x(tl, x), box_src_y(tl, y), box_src_z(tl, z));
}


}  // namespace mb
