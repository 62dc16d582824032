// C ABI of the multiblob library: argument checking, grid set-up (FFT plan,
// twiddle and symbol tables, tiles, scratch), the call sequences of
// mb_spread / mb_interpolate / mb_fluid_solve / mb_spring_forces / mb_step,
// and the per-kernel timing hooks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/multiblob.h"
#include "mb_internal.h"

namespace mb {
size_t record_size(int precision);
}

using namespace mb;

namespace {

const char* const kKernelNames[K_NUM] = {
    "bin_count",   "scan_reduce", "scan_apply",
    "springs_scatter", "bin_scatter", "springs",      "spread",
    "fft_x_fwd",   "fft_y_fwd",   "fft_z_spectral",   "fft_y_inv",
    "fft_x_inv",   "interp",      "interp_step",      "u0",
    "diag",        "fold",        "interp_grad",      "springs_adjoint",
    "fft_xy_inv"};

// Grid sizes: 2^a 3^b in [8, 512]; kernels exist for the multiples of 8.
mb_status size_status(int L) {
    if (L < 8 || L > 512) return MB_ERR_INVALID;
    int n = L;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    if (n != 1) return MB_ERR_INVALID;
    return L % 8 == 0 ? MB_OK : MB_ERR_UNSUPPORTED;
}

bool device_ok(int* dev) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return false;
    }
    if (hipGetDevice(dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return true;
}

mb_status from_hip(hipError_t e) {
    if (e == hipSuccess) return MB_OK;
    if (e == hipErrorOutOfMemory) return MB_ERR_NOMEM;
    return MB_ERR_DEVICE;
}

// Tile geometry of a box of edge L cut into tiles of tx x ty x tz cells.
Tiles make_tiles(int L, int nbox, int tx, int ty, int tz) {
    Tiles t{};
    t.tx = tx;
    t.ty = ty;
    t.tz = tz;
    t.ntx = L / tx;
    t.nty = L / ty;
    t.ntz = L / tz;
    t.n = t.ntx * t.nty * t.ntz;
    t.remap = (t.n % 8 == 0 && t.n >= 64) ? 1 : 0;
    t.nbox = nbox;
    t.lfx = t.lfy = t.lfz = 0;
    t.nbx = t.ntx;
    t.nby = t.nty;
    return t;
}

// Groups tiles t by the box tiles b built from them (their extents
// multiples of t's): the numbering of t becomes box-tile major.
void link_box_tiles(Tiles& t, const Tiles& b) {
    auto lg = [](int r) { int l = 0; while ((1 << l) < r) ++l; return l; };
    t.lfx = lg(b.tx / t.tx);
    t.lfy = lg(b.ty / t.ty);
    t.lfz = lg(b.tz / t.tz);
    t.nbx = b.ntx;
    t.nby = b.nty;
}

// Box tiles of the spreading for binning tiles t: each extent below 16 is
// doubled once (z, then y, then x) when the doubled extent divides L and the
// box of (sx+3)(sy+3)(sz+3) nodes stays within 7,400 (58 KB of 64-bit LDS
// accumulators, two blocks per CU); the binning tiles are kept when no
// spreading kernel exists for the result.  Larger box tiles carry less halo
// per node.
Tiles make_box_tiles(int L, const Tiles& t) {
    int sx = t.tx, sy = t.ty, sz = t.tz;
    int* ext[3] = {&sz, &sy, &sx};
    for (int* e : ext) {
        const int old = *e;
        if (old >= 16 || L % (2 * old) != 0) continue;
        *e = 2 * old;
        if ((sx + 3) * (sy + 3) * (sz + 3) > 7400) *e = old;
    }
    if (!box_shape_supported(sx, sy, sz, t.tx, t.ty, t.tz)) {
        sx = t.tx;
        sy = t.ty;
        sz = t.tz;
    }
    return make_tiles(L, t.nbox, sx, sy, sz);
}

// Validity of a grid description (the checks of mb_grid_create).
mb_status desc_status(const mb_grid_desc& d, int nbox) {
    if (nbox < 1 || nbox > 65536) return MB_ERR_INVALID;
    const mb_status ss = size_status(d.L);
    if (ss != MB_OK) return ss;
    if (d.precision != MB_FP64 && d.precision != MB_MIXED) return MB_ERR_INVALID;
    if (d.mode != MB_UNSTEADY_CN && d.mode != MB_STEADY_STOKES) return MB_ERR_INVALID;
    if (d.zero_mean != 0 && d.zero_mean != 1) return MB_ERR_INVALID;
    if ((d.deterministic != 0 && d.deterministic != 1) ||
        (d.check_finite != 0 && d.check_finite != 1) ||
        (d.external_workspace != 0 && d.external_workspace != 1) || d.reserved != 0)
        return MB_ERR_INVALID;
    if (!(d.h > 0.0) || !std::isfinite(d.h)) return MB_ERR_INVALID;
    if (!(d.dt > 0.0) || !std::isfinite(d.dt)) return MB_ERR_INVALID;
    if (!(d.eta >= 0.0) || !std::isfinite(d.eta)) return MB_ERR_INVALID;
    if (d.mode == MB_UNSTEADY_CN && (!(d.rho > 0.0) || !std::isfinite(d.rho)))
        return MB_ERR_INVALID;
    if (d.mode == MB_STEADY_STOKES && !(d.eta > 0.0)) return MB_ERR_INVALID;
    if (d.max_blobs < 0 || d.max_blobs > (int64_t)1 << 30) return MB_ERR_INVALID;
    const int64_t N = (int64_t)d.L * d.L * d.L;
    if ((N / 512) * nbox + 1 > ((int64_t)1 << 30) || 3 * N * nbox > ((int64_t)1 << 40))
        return MB_ERR_INVALID;
    return MB_OK;
}

// The default tiles of a box of edge L: 16 x 8 x 8 cells, 8 x 8 x 8 when 16
// does not divide L (mb_grid_set_tiles and mb_grid_autotune choose others).
Tiles default_tiles(int L, int nbox) {
    return make_tiles(L, nbox, (L % 16 == 0) ? 16 : 8, 8, 8);
}

size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// The grid's scratch as regions of one workspace, each 256-byte aligned, in
// this order: FFT tables (twiddles, divergence symbol, |symbol|^2), the
// spectrum, the x-pass partial sums, the per-tile arrays (counts, offsets,
// scan block sums, diagnostics partials) and the spread boxes, both sized
// for the tile shape of L with the most tiles / box entries, the per-blob
// arrays (tile, rank, sorted blob, records, velocities), the springs
// blocks' force sums, the non-finite flag, and the particle reordering of
// the step calls (positions and a per-particle array in the calls' own
// particle order, and that order).
struct WsLayout {
    enum { TW, DSYM, D2, SPEC, PSUM, COUNT, OFFS, BSUM, TPART, BOX, TILE, RANK, PERM,
           REC, U, FPART, FLAG, QINT, PINT, ORDER, NREG };
    size_t off[NREG];
    size_t total;
    int ntiles_cap;  // tiles per box
    int nscan;       // scan blocks over ntiles_cap * nbox tiles
};

WsLayout ws_layout(const mb_grid_desc& d, int nbox) {
    WsLayout w{};
    const int L = d.L;
    const size_t fsz = d.precision == MB_MIXED ? 4 : 8;
    const size_t NC = (size_t)L / 2 + 1;
    const int64_t cap = std::max<int64_t>(d.max_blobs, 1);
    int ntiles = 0;
    size_t boxe = 0;
#define MB_SHAPE(X, Y, Z)                                                        \
    if (L % X == 0 && L % Y == 0 && L % Z == 0) {                                \
        const Tiles t = make_tiles(L, nbox, X, Y, Z);                            \
        ntiles = std::max(ntiles, t.n);                                          \
        boxe = std::max(boxe, box_elems(make_box_tiles(L, t)));                  \
    }
    MB_TILE_SHAPES(MB_SHAPE)
#undef MB_SHAPE
    const int64_t nt = (int64_t)ntiles * nbox;
    w.ntiles_cap = ntiles;
    w.nscan = (int)((nt + 4095) / 4096);
    size_t sz[WsLayout::NREG];
    sz[WsLayout::TW] = (size_t)L * 2 * fsz;
    sz[WsLayout::DSYM] = (size_t)L * 2 * fsz;
    sz[WsLayout::D2] = (size_t)L * fsz;
    sz[WsLayout::SPEC] = (size_t)nbox * 3 * L * L * NC * 2 * fsz;
    sz[WsLayout::PSUM] = (size_t)nbox * fft_x_blocks(L, d.precision) * 2 * sizeof(double);
    sz[WsLayout::COUNT] = (size_t)nt * sizeof(int);
    sz[WsLayout::OFFS] = (size_t)(nt + 1) * sizeof(int);
    sz[WsLayout::BSUM] = (size_t)w.nscan * sizeof(int);
    sz[WsLayout::TPART] = (size_t)nt * 4 * sizeof(double);
    sz[WsLayout::BOX] = boxe * fsz;
    sz[WsLayout::TILE] = (size_t)cap * sizeof(int);
    sz[WsLayout::RANK] = (size_t)cap * sizeof(int);
    sz[WsLayout::PERM] = (size_t)cap * sizeof(int);
    sz[WsLayout::REC] = (size_t)cap * record_size(d.precision);
    sz[WsLayout::U] = (size_t)cap * 3 * sizeof(double);
    sz[WsLayout::FPART] = (size_t)cap * 3 * sizeof(double);  // one springs block per blob at most
    sz[WsLayout::FLAG] = 2 * sizeof(int);
    sz[WsLayout::QINT] = (size_t)cap * 3 * sizeof(double);
    sz[WsLayout::PINT] = (size_t)cap * 3 * sizeof(double);  // particles <= blobs
    sz[WsLayout::ORDER] = (size_t)cap * sizeof(int);
    size_t o = 0;
    for (int r = 0; r < WsLayout::NREG; ++r) {
        w.off[r] = o;
        o += up256(sz[r]);
    }
    w.total = o;
    return w;
}

// Points the grid's scratch pointers into workspace `base` (layout of the
// grid's description and box count).
void ws_bind(mb_grid* g, void* base) {
    const WsLayout w = ws_layout(g->d, g->tiles.nbox);
    char* b = (char*)base;
    g->ws = base;
    g->ws_bytes = w.total;
    g->ntiles_cap = w.ntiles_cap;
    g->nscan = w.nscan;
    g->d_tw = b + w.off[WsLayout::TW];
    g->d_dsym = b + w.off[WsLayout::DSYM];
    g->d_d2 = b + w.off[WsLayout::D2];
    g->d_spec = b + w.off[WsLayout::SPEC];
    g->d_psum = (double*)(b + w.off[WsLayout::PSUM]);
    g->d_count = (int*)(b + w.off[WsLayout::COUNT]);
    g->d_offs = (int*)(b + w.off[WsLayout::OFFS]);
    g->d_bsum = (int*)(b + w.off[WsLayout::BSUM]);
    g->d_tile_part = (double*)(b + w.off[WsLayout::TPART]);
    g->d_box = b + w.off[WsLayout::BOX];
    g->d_tile = (int*)(b + w.off[WsLayout::TILE]);
    g->d_rank = (int*)(b + w.off[WsLayout::RANK]);
    g->d_perm = (int*)(b + w.off[WsLayout::PERM]);
    g->d_rec = b + w.off[WsLayout::REC];
    g->d_u = (double*)(b + w.off[WsLayout::U]);
    g->d_force_part = (double*)(b + w.off[WsLayout::FPART]);
    g->d_flag = (int*)(b + w.off[WsLayout::FLAG]);
    g->d_qint = (double*)(b + w.off[WsLayout::QINT]);
    g->d_pint = (double*)(b + w.off[WsLayout::PINT]);
    g->d_order = (int*)(b + w.off[WsLayout::ORDER]);
    g->perm_m = -1;
}

// Scan blocks for the current tiles (at most the workspace's).
void set_scan_blocks(mb_grid* g) {
    const int64_t nt = (int64_t)g->tiles.n * g->tiles.nbox;
    g->nscan = (int)((nt + 4095) / 4096);
}

void free_grid(mb_grid* g) {
    if (!g) return;
    if (g->ws_owned && g->ws) (void)hipFree(g->ws);
    void* ptrs[] = {g->d_adj, g->d_adj_part, g->d_ffield, g->d_mid};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (auto& tp : g->pending) {
        (void)hipEventDestroy(tp.a);
        (void)hipEventDestroy(tp.b);
    }
    for (auto e : g->free_events) (void)hipEventDestroy(e);
    delete g;
}

// Device buffers passed to the library are 256-byte aligned (null passes).
bool aligned(const void* p) { return ((uintptr_t)p & 255u) == 0; }

// Makes the grid's device current; the grid must have its workspace.
mb_status enter(mb_grid* g) {
    if (!g->ws) return MB_ERR_INVALID;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
    if (cur != g->device && hipSetDevice(g->device) != hipSuccess)
        return MB_ERR_DEVICE;
    return MB_OK;
}

// Result of a call whose launches gave e: with check_finite, waits for the
// stream and reports (then clears) the flag its kernels set: bit 1 a
// non-finite input, bit 2 a springs block that gave up waiting for the
// tile offsets (a device failure).
mb_status finish(mb_grid* g, hipError_t e, hipStream_t s) {
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? MB_ERR_NOMEM : MB_ERR_DEVICE;
    if (!g->d.check_finite) return MB_OK;
    int flag = 0;
    e = hipMemcpyAsync(&flag, g->d_flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && flag) e = zero_words(g->d_flag, 1, s);
    if (e != hipSuccess || (flag & 2)) return MB_ERR_DEVICE;
    return flag ? MB_ERR_NONFINITE : MB_OK;
}

SpringsDev springs_dev(const mb_springs* sp) {
    SpringsDev d;
    d.pa = sp->d_pa;
    d.pb = sp->d_pb;
    d.r0 = sp->d_r0;
    d.adj_start = sp->d_adj_start;
    d.adj_pair = sp->d_adj_pair;
    d.k = sp->k;
    d.nb = sp->nb;
    d.npairs = sp->npairs;
    d.ppb = sp->ppb;
    return d;
}

}  // namespace

namespace mb {

bool timer_pair(mb_grid* g, int id, hipEvent_t* start, hipEvent_t* stop) {
    if (!g || !((g->timing >> id) & 1u)) return false;
    hipEvent_t ev[2];
    for (int k = 0; k < 2; ++k) {
        if (!g->free_events.empty()) {
            ev[k] = g->free_events.back();
            g->free_events.pop_back();
        } else if (hipEventCreate(&ev[k]) != hipSuccess) {
            if (k == 1) g->free_events.push_back(ev[0]);
            return false;
        }
    }
    g->pending.push_back(TimerPair{ev[0], ev[1], id});
    *start = ev[0];
    *stop = ev[1];
    return true;
}

}  // namespace mb

extern "C" {

const char* mb_status_string(mb_status st) {
    switch (st) {
        case MB_OK: return "success";
        case MB_ERR_INVALID: return "invalid argument";
        case MB_ERR_UNSUPPORTED: return "unsupported configuration";
        case MB_ERR_NOMEM: return "out of device memory";
        case MB_ERR_DEVICE: return "no usable GPU or device error";
        case MB_ERR_NONFINITE: return "non-finite blob position or force";
    }
    return "unknown status";
}

const char* mb_kernel_name(int32_t id) {
    if (id < 0 || id >= K_NUM) return nullptr;
    return kKernelNames[id];
}

mb_status mb_grid_create(const mb_grid_desc* desc, mb_grid** out) {
    return mb_grid_create_batch(desc, 1, out);
}

mb_status mb_grid_create_batch(const mb_grid_desc* desc, int32_t nbox, mb_grid** out) {
    if (!out) return MB_ERR_INVALID;
    *out = nullptr;
    if (!desc) return MB_ERR_INVALID;
    const mb_grid_desc d = *desc;
    const mb_status ds = desc_status(d, nbox);
    if (ds != MB_OK) return ds;
    int dev = 0;
    if (!device_ok(&dev)) return MB_ERR_DEVICE;

    mb_grid* g = new (std::nothrow) mb_grid();
    if (!g) return MB_ERR_NOMEM;
    g->d = d;
    g->device = dev;
    g->L = d.L;
    g->NC = d.L / 2 + 1;
    g->N = (int64_t)d.L * d.L * d.L;
    g->fsz = d.precision == MB_MIXED ? 4 : 8;
    g->nblk_x = fft_x_blocks(d.L, d.precision);
    g->tiles = default_tiles(d.L, nbox);
    g->btiles = make_box_tiles(d.L, g->tiles);
    link_box_tiles(g->tiles, g->btiles);
    g->rec_size = record_size(d.precision);
    // springs blocks hold at least one particle of at least one blob
    g->force_blocks_cap = (int)std::max<int64_t>(d.max_blobs, 1);
    g->perm_m = -1;
    if (d.external_workspace) {
        *out = g;  // no scratch until mb_grid_set_workspace
        return MB_OK;
    }
    const size_t bytes = ws_layout(d, nbox).total;
    void* ws = nullptr;
    hipError_t e = hipMalloc(&ws, bytes);
    if (e == hipSuccess) {
        g->ws_owned = true;
        ws_bind(g, ws);
        set_scan_blocks(g);
        e = init_workspace(g, nullptr);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_grid(g);
        return from_hip(e);
    }
    *out = g;
    return MB_OK;
}

size_t mb_workspace_size(const mb_grid_desc* desc, int32_t nbox) {
    if (!desc || desc_status(*desc, nbox) != MB_OK) return 0;
    return ws_layout(*desc, nbox).total;
}

mb_status mb_grid_set_workspace(mb_grid* g, void* ptr, size_t bytes) {
    if (!g || !ptr || !aligned(ptr)) return MB_ERR_INVALID;
    const size_t need = ws_layout(g->d, g->tiles.nbox).total;
    if (bytes < need) return MB_ERR_INVALID;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
    if (cur != g->device && hipSetDevice(g->device) != hipSuccess) return MB_ERR_DEVICE;
    hipPointerAttribute_t attr{};
    if (hipPointerGetAttributes(&attr, ptr) != hipSuccess || attr.device != g->device ||
        attr.type == hipMemoryTypeHost) {
        (void)hipGetLastError();
        if (cur >= 0 && cur != g->device) (void)hipSetDevice(cur);
        return MB_ERR_INVALID;
    }
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) {
        if (g->ws_owned && g->ws) (void)hipFree(g->ws);
        g->ws_owned = false;
        ws_bind(g, ptr);
        set_scan_blocks(g);
        e = init_workspace(g, nullptr);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (cur >= 0 && cur != g->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        g->ws = nullptr;  // unusable until a workspace is set again
        return from_hip(e);
    }
    return MB_OK;
}

mb_status mb_grid_destroy(mb_grid* g) {
    if (!g) return MB_OK;
    const int dev = g->device;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    free_grid(g);
    if (cur >= 0 && cur != dev) (void)hipSetDevice(cur);
    return MB_OK;
}

mb_status mb_springs_create(int32_t nb, int32_t npairs, const int32_t* pa,
                            const int32_t* pb, const double* r0, double k,
                            mb_springs** out) {
    if (!out) return MB_ERR_INVALID;
    *out = nullptr;
    if (nb < 1 || nb > 64 || npairs < 0 || npairs > nb * (nb - 1) / 2)
        return MB_ERR_INVALID;
    if (npairs > 0 && (!pa || !pb || !r0)) return MB_ERR_INVALID;
    if (!(k >= 0.0) || !std::isfinite(k)) return MB_ERR_INVALID;
    std::vector<int> deg(nb, 0);
    for (int e = 0; e < npairs; ++e) {
        if (pa[e] < 0 || pa[e] >= nb || pb[e] < 0 || pb[e] >= nb || pa[e] == pb[e])
            return MB_ERR_INVALID;
        if (!(r0[e] > 0.0) || !std::isfinite(r0[e])) return MB_ERR_INVALID;
        deg[pa[e]]++;
        deg[pb[e]]++;
    }
    for (int b = 0; b < nb; ++b)
        if (deg[b] > 63) return MB_ERR_INVALID;
    int dev = 0;
    if (!device_ok(&dev)) return MB_ERR_DEVICE;
    // per-blob incident pairs: e << 8 | (the pair's other blob)
    std::vector<int> start(nb + 1, 0);
    for (int b = 0; b < nb; ++b) start[b + 1] = start[b] + deg[b];
    std::vector<int> inc(std::max(1, 2 * npairs), 0), fill(start.begin(), start.end() - 1);
    for (int e = 0; e < npairs; ++e) {
        inc[fill[pa[e]]++] = (e << 8) | pb[e];
        inc[fill[pb[e]]++] = (e << 8) | pa[e];
    }
    std::vector<int> hpa(std::max(1, npairs), 0), hpb(std::max(1, npairs), 0);
    std::vector<double> hr0(std::max(1, npairs), 1.0);
    for (int e = 0; e < npairs; ++e) {
        hpa[e] = pa[e];
        hpb[e] = pb[e];
        hr0[e] = r0[e];
    }
    // particles per block: at most 256 blobs; their positions plus the rest
    // lengths and incidence lists in at most 48 KB of LDS (at most 34 KB
    // for a single particle of 64 blobs and all 2016 pairs)
    const int per_particle = nb * 3 * (int)sizeof(double);
    const int tables = npairs * (int)sizeof(double) + (nb + 1 + 2 * npairs) * (int)sizeof(int);
    mb_springs* sp = new (std::nothrow) mb_springs();
    if (!sp) return MB_ERR_NOMEM;
    sp->nb = nb;
    sp->npairs = npairs;
    sp->k = k;
    sp->device = dev;
    {
        const int by_blobs = std::max(1, 256 / nb);
        const int by_lds = std::max(1, (48 * 1024 - tables) / per_particle);
        sp->ppb = std::min(by_blobs, by_lds);
    }
    hipError_t e = hipSuccess;
    auto up = [&](void** dst, const void* src, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(dst, bytes);
        if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    up((void**)&sp->d_pa, hpa.data(), hpa.size() * sizeof(int));
    up((void**)&sp->d_pb, hpb.data(), hpb.size() * sizeof(int));
    up((void**)&sp->d_r0, hr0.data(), hr0.size() * sizeof(double));
    up((void**)&sp->d_adj_start, start.data(), start.size() * sizeof(int));
    up((void**)&sp->d_adj_pair, inc.data(), inc.size() * sizeof(int));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        mb_springs_destroy(sp);
        return from_hip(e);
    }
    *out = sp;
    return MB_OK;
}

mb_status mb_springs_destroy(mb_springs* sp) {
    if (!sp) return MB_OK;
    (void)hipDeviceSynchronize();
    void* ptrs[] = {sp->d_pa, sp->d_pb, sp->d_r0, sp->d_adj_start, sp->d_adj_pair};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete sp;
    return MB_OK;
}

mb_status mb_springs_set_params(mb_springs* sp, const double* r0, double k, void* stream) {
    if (!sp || (sp->npairs > 0 && !r0)) return MB_ERR_INVALID;
    if (!(k >= 0.0) || !std::isfinite(k)) return MB_ERR_INVALID;
    for (int e = 0; e < sp->npairs; ++e)
        if (!(r0[e] > 0.0) || !std::isfinite(r0[e])) return MB_ERR_INVALID;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
    if (cur != sp->device && hipSetDevice(sp->device) != hipSuccess) return MB_ERR_DEVICE;
    hipError_t e = hipSuccess;
    if (sp->npairs > 0)
        e = hipMemcpyAsync(sp->d_r0, r0, (size_t)sp->npairs * sizeof(double),
                           hipMemcpyHostToDevice, (hipStream_t)stream);
    if (cur >= 0 && cur != sp->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return from_hip(e);
    sp->k = k;
    return MB_OK;
}

mb_status mb_spread(mb_grid* g, int64_t M, const double* q, const double* F,
                    void* f_out, void* stream) {
    if (!g || !f_out || M < 0 || M > g->d.max_blobs) return MB_ERR_INVALID;
    if (M % g->tiles.nbox) return MB_ERR_INVALID;  // the same number of blobs per box
    if (M > 0 && (!q || !F || !aligned(q) || !aligned(F))) return MB_ERR_INVALID;
    if (!aligned(f_out)) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (g->fsz == 4) {
        e = bin_blobs<float>(g, M, q, s);
        if (e == hipSuccess) e = scatter_records<float>(g, M, q, F, s);
        if (e == hipSuccess) e = spread_boxes<float>(g, s);
        if (e == hipSuccess) e = fold_boxes<float>(g, (float*)f_out, s);
    } else {
        e = bin_blobs<double>(g, M, q, s);
        if (e == hipSuccess) e = scatter_records<double>(g, M, q, F, s);
        if (e == hipSuccess) e = spread_boxes<double>(g, s);
        if (e == hipSuccess) e = fold_boxes<double>(g, (double*)f_out, s);
    }
    return finish(g, e, s);
}

mb_status mb_interpolate(mb_grid* g, int64_t M, const double* q, const void* v,
                         double* u_out, void* stream) {
    if (!g || !v || M < 0 || M > g->d.max_blobs) return MB_ERR_INVALID;
    if (M % g->tiles.nbox) return MB_ERR_INVALID;
    if (M > 0 && (!q || !u_out || !aligned(q) || !aligned(u_out))) return MB_ERR_INVALID;
    if (!aligned(v)) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    if (M == 0) return MB_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (g->fsz == 4) {
        e = bin_blobs<float>(g, M, q, s);
        if (e == hipSuccess) e = scatter_records<float>(g, M, q, nullptr, s);
        if (e == hipSuccess) e = interpolate<float>(g, M, (const float*)v, u_out, nullptr, 0, s);
    } else {
        e = bin_blobs<double>(g, M, q, s);
        if (e == hipSuccess) e = scatter_records<double>(g, M, q, nullptr, s);
        if (e == hipSuccess) e = interpolate<double>(g, M, (const double*)v, u_out, nullptr, 0, s);
    }
    return finish(g, e, s);
}

mb_status mb_fluid_solve(mb_grid* g, const void* v_in, const void* f,
                         void* v_out, void* stream) {
    if (!g || !f || !v_out) return MB_ERR_INVALID;
    const bool steady = g->d.mode == MB_STEADY_STOKES;
    if (!steady && !v_in) return MB_ERR_INVALID;
    if (!aligned(v_in) || !aligned(f) || !aligned(v_out)) return MB_ERR_INVALID;
    if (!v_in) v_in = v_out;  // unread in steady mode
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (g->fsz == 4)
        e = fluid_solve<float>(g, (const float*)v_in, (const float*)f, (float*)v_out, s);
    else
        e = fluid_solve<double>(g, (const double*)v_in, (const double*)f, (double*)v_out, s);
    return from_hip(e);
}

mb_status mb_spring_forces(const mb_springs* sp, int64_t P, const double* q,
                           const double* Fext, double* F_out, void* stream) {
    if (!sp || P < 0) return MB_ERR_INVALID;
    if (P > 0 && (!q || !F_out || !aligned(q) || !aligned(F_out))) return MB_ERR_INVALID;
    if (!aligned(Fext)) return MB_ERR_INVALID;
    if ((int64_t)P * sp->nb > ((int64_t)1 << 31) - 1) return MB_ERR_INVALID;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
    if (cur != sp->device && hipSetDevice(sp->device) != hipSuccess) return MB_ERR_DEVICE;
    return from_hip(spring_forces(springs_dev(sp), P, q, Fext, F_out,
                                  (hipStream_t)stream, nullptr));
}

// One step of the grid's scheme on fields of type T (u_dst: blob velocities
// of the step, or null).
extern "C++" {
template <typename T>
static hipError_t step_once(mb_grid* g, const SpringsDev& sd, int64_t P, int64_t M,
                            double* q, T* v, const double* Fext, const double* Gblob,
                            const T* ffluid, double* u_dst, hipStream_t s,
                            bool binned = false, bool bin_next = false, bool diag = true) {
    T* ff = (T*)g->d_ffield;
    // forces at positions x, spread into the boxes (and folded with the
    // fluid force when there is one); binned: the counts of q are in place;
    // sums: the force sums of the diagnostics.  The diagnostics' partial
    // sums (forces, momentum, max |Dv|) are formed only when diag is set
    // (the step whose diagnostics are returned).
    auto forces = [&](const double* x, bool counted, bool sums) {
        const bool fuse = fused_scan_ok(g, s);  // the scan in the springs kernel
        hipError_t e = bin_blobs<T>(g, M, x, s, counted, !fuse);
        if (e == hipSuccess) e = scatter_springs<T>(g, sd, P, x, Fext, s, Gblob, sums, fuse);
        if (e == hipSuccess) e = spread_boxes<T>(g, s);
        if (e == hipSuccess && ffluid) e = fold_boxes<T>(g, ff, s, ffluid);
        return e;
    };
    auto solve = [&]() { return fluid_solve<T>(g, v, ff, v, s, !ffluid); };
    hipError_t e;
    const int dg = diag ? 1 : 0;
    if (g->scheme == MB_SCHEME_EULER) {
        e = forces(q, binned, diag);
        if (e == hipSuccess) e = solve();
        if (e == hipSuccess) e = interpolate<T>(g, M, v, u_dst, q, dg, s, 1.0, bin_next);
        return e;
    }
    // midpoint predictor-corrector: q* in d_mid, the second half of the
    // interpolated velocity in d_mid + 3 max_blobs
    double* qs = g->d_mid;
    double* u2 = g->d_mid + 3 * std::max<int64_t>(g->d.max_blobs, 1);
    e = blob_axpy(3 * M, nullptr, 1.0, q, qs, s);  // q* = q^n
    if (g->d.mode == MB_STEADY_STOKES) {
        // q* += (dt/2) J(q^n) v(q^n);  q += dt J(q*) v(q*)
        if (e == hipSuccess) e = forces(q, false, false);
        if (e == hipSuccess) e = solve();
        if (e == hipSuccess) e = interpolate<T>(g, M, v, nullptr, qs, 0, s, 0.5);
        if (e == hipSuccess) e = forces(qs, false, diag);
        if (e == hipSuccess) e = solve();
        if (e == hipSuccess) e = interpolate<T>(g, M, v, u_dst, q, dg, s);
        return e;
    }
    // q* += (dt/2) J(q^n) v^n on the records of q^n
    if (e == hipSuccess) e = bin_blobs<T>(g, M, q, s);
    if (e == hipSuccess) e = scatter_records<T>(g, M, q, nullptr, s);
    if (e == hipSuccess) e = interpolate<T>(g, M, v, nullptr, qs, 0, s, 0.5);
    // forces at q*; q += (dt/2) J(q*) v^n; solve; q += (dt/2) J(q*) v^{n+1}
    if (e == hipSuccess) e = forces(qs, false, diag);
    if (e == hipSuccess) e = interpolate<T>(g, M, v, u_dst, q, 0, s, 0.5);
    if (e == hipSuccess) e = solve();
    if (e == hipSuccess) e = interpolate<T>(g, M, v, u_dst ? u2 : nullptr, q, dg, s, 0.5);
    if (e == hipSuccess && u_dst) e = blob_add(3 * M, u2, u_dst, s);
    return e;
}
}  // extern "C++"

static hipError_t alloc_lazy(void** p, size_t bytes) {
    if (*p) return hipSuccess;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) *p = nullptr;
    return e;
}

// Calls of at least this many steps reorder the particles for locality.
constexpr int kReorderMinSteps = 8;

// Steps of one grid; check: report the non-finite flag at the end (false
// inside a graph capture, where the caller checks after the replays).
static mb_status step_impl(mb_grid* g, const mb_springs* sp, int64_t P, double* q,
                           void* v, const double* Fext, const double* Gblob,
                           double* u_out, double* U0_out, double* diag_out,
                           int32_t nsteps, void* stream, const void* ffluid = nullptr,
                           bool check = true) {
    if (!g || !sp || !v || P < 0 || nsteps < 0) return MB_ERR_INVALID;
    const int64_t M = P * sp->nb;
    if (M > g->d.max_blobs) return MB_ERR_INVALID;
    if (P % g->tiles.nbox) return MB_ERR_INVALID;  // the same particles per box
    if (M > 0 && !q) return MB_ERR_INVALID;
    if (!aligned(q) || !aligned(v) || !aligned(Fext) || !aligned(Gblob) || !aligned(u_out) ||
        !aligned(U0_out) || !aligned(diag_out) || !aligned(ffluid))
        return MB_ERR_INVALID;
    if (sp->device != g->device) return MB_ERR_INVALID;
    if (g->scheme == MB_SCHEME_MIDPOINT && !g->d_mid) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    if (nsteps == 0) return MB_OK;
    hipStream_t s = (hipStream_t)stream;
    const SpringsDev sd = springs_dev(sp);
    const int fb = springs_blocks(sd, P);
    hipError_t e = hipSuccess;
    if (ffluid) e = alloc_lazy(&g->d_ffield, (size_t)3 * g->N * g->tiles.nbox * g->fsz);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? MB_ERR_NOMEM : MB_ERR_DEVICE;
    if (M == 0 && diag_out) {
        // no blobs: the force partials of the diagnostics are zero
        e = zero_words(g->d_force_part, 3 * 2, s);
        if (e != hipSuccess) return from_hip(e);
    }
    // A call of many steps runs them on its own copy of the positions (and
    // particle forces) with the particles ordered by tile, so that the blobs
    // of a tile are near one another in memory (their position updates and
    // records then share cache lines); results do not depend on the order.
    const bool reorder = M > 0 && nsteps >= kReorderMinSteps && !Gblob && !ffluid;
    double* qs = q;
    const double* Fs = Fext;
    if (reorder) {
        e = order_particles(g, P, sp->nb, q, Fext, s);
        qs = g->d_qint;
        Fs = Fext ? g->d_pint : nullptr;
        // the call's blob numbering is new: the first binning takes the blobs
        // in index order, which is by tile now, so that each block counts
        // into a few tiles (and ranks follow blob order within a tile)
        g->perm_m = -1;
    }
    // first-order steps after the first of the call take their binning from
    // the interpolation of the step before (the positions it wrote); the
    // last step leaves the counts at zero
    const bool carry = g->scheme == MB_SCHEME_EULER && M > 0;
    double* U0_dst = reorder ? g->d_pint : U0_out;  // particle forces are done by then
    for (int n = 0; n < nsteps && e == hipSuccess; ++n) {
        const bool last = n == nsteps - 1;
        const bool binned = carry && n > 0, bin_next = carry && !last;
        double* u_dst = nullptr;
        if (last && (u_out || U0_out)) u_dst = (u_out && !reorder) ? u_out : g->d_u;
        const bool diag = last && diag_out;  // partial sums only where they are read
        if (g->fsz == 4)
            e = step_once<float>(g, sd, P, M, qs, (float*)v, Fs, Gblob, (const float*)ffluid,
                                 u_dst, s, binned, bin_next, diag);
        else
            e = step_once<double>(g, sd, P, M, qs, (double*)v, Fs, Gblob,
                                  (const double*)ffluid, u_dst, s, binned, bin_next, diag);
        if (!last && e != hipSuccess && bin_next)
            (void)zero_words(g->d_count, (size_t)g->tiles.n * g->tiles.nbox, s);
        if (last && e == hipSuccess && U0_out)
            e = particle_means(g, P, sp->nb, u_dst, U0_dst, s);
        if (last && e == hipSuccess && diag_out)
            e = diagnostics(g, M > 0 ? fb : 1, diag_out, s);
    }
    if (reorder && e == hipSuccess)
        e = unorder_particles(g, P, sp->nb, q, u_out ? g->d_u : nullptr, u_out,
                              U0_out ? g->d_pint : nullptr, U0_out, s);
    if (!check) return from_hip(e);
    return finish(g, e, s);
}

mb_status mb_step(mb_grid* g, const mb_springs* sp, int64_t P, double* q,
                  void* v, const double* Fext, double* u_out, double* U0_out,
                  double* diag_out, int32_t nsteps, void* stream) {
    return step_impl(g, sp, P, q, v, Fext, nullptr, u_out, U0_out, diag_out, nsteps,
                     stream);
}

mb_status mb_step_ext(mb_grid* g, const mb_springs* sp, int64_t P, double* q,
                      void* v, const double* Fext, const double* F_blob,
                      double* u_out, double* U0_out, double* diag_out,
                      int32_t nsteps, void* stream) {
    return step_impl(g, sp, P, q, v, Fext, F_blob, u_out, U0_out, diag_out, nsteps,
                     stream);
}

mb_status mb_step_forced(mb_grid* g, const mb_springs* sp, int64_t P, double* q,
                         void* v, const double* Fext, const double* F_blob,
                         const void* f_fluid, double* u_out, double* U0_out,
                         double* diag_out, int32_t nsteps, void* stream) {
    if (!f_fluid) return MB_ERR_INVALID;
    return step_impl(g, sp, P, q, v, Fext, F_blob, u_out, U0_out, diag_out, nsteps,
                     stream, f_fluid);
}

mb_status mb_step_graph(int32_t ngrids, mb_grid* const* grids,
                        const mb_springs* const* springs, const int64_t* nparticles,
                        double* const* q, void* const* v, const double* const* Fext,
                        const double* const* F_blob, int32_t nsteps, void* stream) {
    if (ngrids < 1 || !grids || !springs || !nparticles || !q || !v || nsteps < 0)
        return MB_ERR_INVALID;
    for (int i = 0; i < ngrids; ++i) {
        mb_grid* g = grids[i];
        const mb_springs* sp = springs[i];
        if (!g || !sp || !v[i] || nparticles[i] < 0) return MB_ERR_INVALID;
        const int64_t M = nparticles[i] * sp->nb;
        if (M > g->d.max_blobs || nparticles[i] % g->tiles.nbox) return MB_ERR_INVALID;
        if (M > 0 && !q[i]) return MB_ERR_INVALID;
        if (!aligned(q[i]) || !aligned(v[i]) || (F_blob && !aligned(F_blob[i])) ||
            (Fext && !aligned(Fext[i])))
            return MB_ERR_INVALID;
        if (sp->device != g->device || g->device != grids[0]->device) return MB_ERR_INVALID;
        if (!g->ws) return MB_ERR_INVALID;
        if (g->scheme == MB_SCHEME_MIDPOINT && !g->d_mid) return MB_ERR_INVALID;
    }
    mb_status st = enter(grids[0]);
    if (st != MB_OK) return st;
    if (nsteps == 0) return MB_OK;
    // the non-finite checks of the grids that ask for them are read once,
    // after the last step
    auto one_step = [&](hipStream_t s) -> mb_status {
        for (int i = 0; i < ngrids; ++i) {
            mb_status r = step_impl(grids[i], springs[i], nparticles[i], q[i], v[i],
                                    Fext ? Fext[i] : nullptr, F_blob ? F_blob[i] : nullptr,
                                    nullptr, nullptr, nullptr, 1, (void*)s, nullptr, false);
            if (r != MB_OK) return r;
        }
        return MB_OK;
    };
    auto check_all = [&](hipError_t e) -> mb_status {
        mb_status r = MB_OK;
        for (int i = 0; i < ngrids; ++i) {
            const mb_status ri = finish(grids[i], e, (hipStream_t)stream);
            if (r == MB_OK) r = ri;
        }
        return r;
    };
    hipStream_t caller = (hipStream_t)stream;
    int done = 0;
    // an eager first step when a grid has no sorted order from an earlier
    // binning of these blobs, so that the captured binning uses it
    bool warm = true;
    for (int i = 0; i < ngrids; ++i)
        if (grids[i]->perm_m != nparticles[i] * springs[i]->nb) warm = false;
    if (!warm) {
        st = one_step(caller);
        if (st != MB_OK) return st;
        done = 1;
    }
    if (done == nsteps) return check_all(hipSuccess);
    hipStream_t cs = nullptr;
    hipEvent_t ev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<uint32_t> timing(ngrids);
    for (int i = 0; i < ngrids; ++i) {
        timing[i] = grids[i]->timing;
        grids[i]->timing = 0;
    }
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, caller);
    if (e == hipSuccess) e = hipStreamWaitEvent(cs, ev, 0);
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        st = one_step(cs);
        hipError_t ec = hipStreamEndCapture(cs, &graph);
        if (st == MB_OK) e = ec;
    }
    if (e == hipSuccess && st == MB_OK) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int n = done; n < nsteps && e == hipSuccess && st == MB_OK; ++n)
        e = hipGraphLaunch(exec, cs);
    if (e == hipSuccess && st == MB_OK) e = hipStreamSynchronize(cs);
    for (int i = 0; i < ngrids; ++i) grids[i]->timing = timing[i];
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (ev) (void)hipEventDestroy(ev);
    if (cs) (void)hipStreamDestroy(cs);
    if (st != MB_OK) return st;
    return check_all(e);
}

mb_status mb_spring_forces_ext(const mb_springs* sp, int64_t P, const double* q,
                               const double* Fext, const double* F_blob, double* F_out,
                               void* stream) {
    if (!sp || P < 0) return MB_ERR_INVALID;
    if (P > 0 && (!q || !F_out)) return MB_ERR_INVALID;
    if (!aligned(q) || !aligned(F_out) || !aligned(Fext) || !aligned(F_blob))
        return MB_ERR_INVALID;
    if ((int64_t)P * sp->nb > ((int64_t)1 << 31) - 1) return MB_ERR_INVALID;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
    if (cur != sp->device && hipSetDevice(sp->device) != hipSuccess) return MB_ERR_DEVICE;
    return from_hip(spring_forces(springs_dev(sp), P, q, Fext, F_out, (hipStream_t)stream,
                                  nullptr, F_blob));
}

mb_status mb_interpolate_grad(mb_grid* g, int64_t M, const double* q, const void* v,
                              const double* W, double* g_inout, void* stream) {
    if (!g || !v || M < 0 || M > g->d.max_blobs) return MB_ERR_INVALID;
    if (M % g->tiles.nbox) return MB_ERR_INVALID;
    if (M > 0 && (!q || !W || !g_inout)) return MB_ERR_INVALID;
    if (!aligned(q) || !aligned(W) || !aligned(g_inout) || !aligned(v)) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    if (M == 0) return MB_OK;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (g->fsz == 4) {
        e = bin_blobs<float>(g, M, q, s);
        if (e == hipSuccess) e = scatter_records<float>(g, M, q, nullptr, s);
        if (e == hipSuccess) e = interpolate_grad<float>(g, (const float*)v, W, 1.0, g_inout, s);
    } else {
        e = bin_blobs<double>(g, M, q, s);
        if (e == hipSuccess) e = scatter_records<double>(g, M, q, nullptr, s);
        if (e == hipSuccess)
            e = interpolate_grad<double>(g, (const double*)v, W, 1.0, g_inout, s);
    }
    return finish(g, e, s);
}

mb_status mb_spring_adjoint(const mb_springs* sp, int64_t P, const double* q,
                            const double* Fbar, double* qbar, double* kbar, double* r0bar,
                            void* stream) {
    if (!sp || P < 0) return MB_ERR_INVALID;
    if (P > 0 && (!q || !Fbar || !qbar)) return MB_ERR_INVALID;
    if (!aligned(q) || !aligned(Fbar) || !aligned(qbar) || !aligned(kbar) || !aligned(r0bar))
        return MB_ERR_INVALID;
    if ((int64_t)P * sp->nb > ((int64_t)1 << 31) - 1) return MB_ERR_INVALID;
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
    if (cur != sp->device && hipSetDevice(sp->device) != hipSuccess) return MB_ERR_DEVICE;
    return from_hip(springs_adjoint(springs_dev(sp), P, q, Fbar, qbar, kbar, r0bar,
                                    (hipStream_t)stream, nullptr));
}

mb_status mb_step_adjoint(mb_grid* g, const mb_springs* sp, int64_t P, const double* q_n,
                          const void* v_np1, const double* Fext, const double* F_blob,
                          const double* ubar_loss, double* qbar, void* vbar,
                          double* Fblob_bar, double* kbar, double* r0bar, void* stream) {
    if (!g || !sp || !v_np1 || !vbar || P < 0) return MB_ERR_INVALID;
    if (g->fsz != 8 || g->scheme != MB_SCHEME_EULER) return MB_ERR_UNSUPPORTED;
    const int64_t M = P * sp->nb;
    if (M > g->d.max_blobs) return MB_ERR_INVALID;
    if (P % g->tiles.nbox) return MB_ERR_INVALID;
    if (M > 0 && (!q_n || !qbar)) return MB_ERR_INVALID;
    if (!aligned(q_n) || !aligned(qbar) || !aligned(Fext) || !aligned(F_blob) ||
        !aligned(ubar_loss) || !aligned(Fblob_bar) || !aligned(kbar) || !aligned(r0bar) ||
        !aligned(v_np1) || !aligned(vbar))
        return MB_ERR_INVALID;
    if (sp->device != g->device) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    const size_t nf = (size_t)3 * g->N * g->tiles.nbox;
    const size_t nbl = (size_t)3 * std::max<int64_t>(g->d.max_blobs, 1);
    if (!g->d_adj) {
        // scratch of the reverse step: fields wbar, fbar, zero; blob arrays
        // ubar, F, Fbar
        e = hipMalloc(&g->d_adj, (3 * nf + 3 * nbl) * sizeof(double));
        if (e == hipSuccess) e = hipMemset(g->d_adj, 0, (3 * nf + 3 * nbl) * sizeof(double));
        if (e != hipSuccess) {
            if (g->d_adj) (void)hipFree(g->d_adj);
            g->d_adj = nullptr;
            return e == hipErrorOutOfMemory ? MB_ERR_NOMEM : MB_ERR_DEVICE;
        }
    }
    // deterministic: per-block partial sums of kbar and r0bar, added in
    // block order, instead of float64 atomics
    double* part = nullptr;
    if (g->d.deterministic && (kbar || r0bar) && M > 0) {
        const size_t need = springs_adjoint_part_size(springs_dev(sp), P);
        if (g->adj_part_cap < need) {
            if (g->d_adj_part) (void)hipFree(g->d_adj_part);
            g->d_adj_part = nullptr;
            g->adj_part_cap = 0;
            e = hipMalloc((void**)&g->d_adj_part, need * sizeof(double));
            if (e != hipSuccess) {
                g->d_adj_part = nullptr;
                return e == hipErrorOutOfMemory ? MB_ERR_NOMEM : MB_ERR_DEVICE;
            }
            g->adj_part_cap = need;
        }
        part = g->d_adj_part;
    }
    double* wbar = g->d_adj;
    double* fbar = wbar + nf;
    const double* zero = fbar + nf;  // never written after the allocation
    double* ubar = wbar + 3 * nf;
    double* F = ubar + nbl;
    double* Fbar = F + nbl;
    const double h = g->d.h;
    const double h3 = h * h * h;
    const SpringsDev sd = springs_dev(sp);
    const double* vn1 = (const double*)v_np1;
    double* vb = (double*)vbar;
    // q^{n+1} = q^n + dt u^n:  ubar = ubar_loss + dt qbar
    e = blob_axpy(3 * M, ubar_loss, g->d.dt, qbar, ubar, s);
    // records of q^n carrying ubar (scale 1: h^3 S ubar = J^T ubar)
    if (e == hipSuccess) e = bin_blobs<double>(g, M, q_n, s);
    if (e == hipSuccess) e = scatter_records<double>(g, M, q_n, ubar, s, 1.0);
    // u^n = J(q^n) v^{n+1}: position part
    if (e == hipSuccess && M > 0) e = interpolate_grad<double>(g, vn1, ubar, 1.0, qbar, s);
    // wbar = vbar + J^T ubar
    if (e == hipSuccess) e = spread_boxes<double>(g, s);
    if (e == hipSuccess) e = fold_boxes<double>(g, wbar, s, vb);
    // v^{n+1} = Q (C v^n + f^n): fbar = Q wbar, vbar = C Q wbar (Q and C
    // commute; steady: vbar = 0)
    if (e == hipSuccess) e = fluid_solve<double>(g, zero, wbar, fbar, s);
    if (e == hipSuccess) {
        if (g->d.mode == MB_STEADY_STOKES) e = zero_words(vb, nf * 2, s);
        else e = apply_cn<double>(g, fbar, vb, s);
    }
    // F^n = springs(q^n) + Fext/nb + G
    if (e == hipSuccess) e = spring_forces(sd, P, q_n, Fext, F, s, g, F_blob);
    // f^n = S(q^n) F^n: Fbar = h^-3 J fbar, and the position part
    if (e == hipSuccess && M > 0)
        e = interpolate<double>(g, M, fbar, Fbar, nullptr, 0, s, 1.0 / h3);
    if (e == hipSuccess && M > 0) e = interpolate_grad<double>(g, fbar, F, 1.0 / h3, qbar, s);
    // springs: qbar, kbar, r0bar; the blob forces: Fblob_bar += Fbar
    if (e == hipSuccess) e = springs_adjoint(sd, P, q_n, Fbar, qbar, kbar, r0bar, s, g, part);
    if (e == hipSuccess && Fblob_bar) e = blob_add(3 * M, Fbar, Fblob_bar, s);
    return finish(g, e, s);
}

mb_status mb_grid_set_scheme(mb_grid* g, int32_t scheme) {
    if (!g || (scheme != MB_SCHEME_EULER && scheme != MB_SCHEME_MIDPOINT))
        return MB_ERR_INVALID;
    if (scheme == MB_SCHEME_MIDPOINT && !g->d_mid) {
        // q* and the second half-velocity of every blob, allocated here so
        // that no step (nor a graph capture of one) allocates
        int cur = -1;
        if (hipGetDevice(&cur) != hipSuccess) return MB_ERR_DEVICE;
        if (cur != g->device && hipSetDevice(g->device) != hipSuccess) return MB_ERR_DEVICE;
        const hipError_t e = hipMalloc(
            (void**)&g->d_mid, (size_t)6 * std::max<int64_t>(g->d.max_blobs, 1) * sizeof(double));
        if (cur >= 0 && cur != g->device) (void)hipSetDevice(cur);
        if (e != hipSuccess) {
            g->d_mid = nullptr;
            (void)hipGetLastError();
            return e == hipErrorOutOfMemory ? MB_ERR_NOMEM : MB_ERR_DEVICE;
        }
    }
    g->scheme = scheme;
    return MB_OK;
}

static bool tiles_fit(int L, int tx, int ty, int tz) {
    return tile_shape_supported(tx, ty, tz) && L % tx == 0 && L % ty == 0 && L % tz == 0;
}

// Switch g to tiles of tx x ty x tz cells (waits for the device first).
static mb_status set_tiles(mb_grid* g, int tx, int ty, int tz) {
    if (g->tiles.tx == tx && g->tiles.ty == ty && g->tiles.tz == tz) return MB_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return from_hip(e);
    // the workspace holds the tile arrays and boxes of every shape of L;
    // the counts start from zero under the new numbering
    g->tiles = make_tiles(g->L, g->tiles.nbox, tx, ty, tz);
    g->btiles = make_box_tiles(g->L, g->tiles);
    link_box_tiles(g->tiles, g->btiles);
    set_scan_blocks(g);
    e = zero_words(g->d_count, (size_t)g->ntiles_cap * g->tiles.nbox, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    return from_hip(e);
}

mb_status mb_grid_set_tiles(mb_grid* g, int32_t tx, int32_t ty, int32_t tz) {
    if (!g || !tiles_fit(g->L, tx, ty, tz)) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    return set_tiles(g, tx, ty, tz);
}

mb_status mb_grid_get_tiles(const mb_grid* g, int32_t* shape_out) {
    if (!g || !shape_out) return MB_ERR_INVALID;
    shape_out[0] = g->tiles.tx;
    shape_out[1] = g->tiles.ty;
    shape_out[2] = g->tiles.tz;
    return MB_OK;
}

mb_status mb_grid_autotune(mb_grid* g, const mb_springs* sp, int64_t P, const double* q,
                           const void* v, const double* Fext, int32_t nsteps, void* stream,
                           int32_t* shape_out) {
    if (!g || !sp || !v || P < 0 || nsteps < 1) return MB_ERR_INVALID;
    const int64_t M = P * sp->nb;
    if (M > g->d.max_blobs || P % g->tiles.nbox || sp->device != g->device)
        return MB_ERR_INVALID;
    if (M > 0 && !q) return MB_ERR_INVALID;
    if (!aligned(q) || !aligned(v) || !aligned(Fext)) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const size_t qbytes = (size_t)std::max<int64_t>(M, 1) * 3 * sizeof(double);
    const size_t vbytes = (size_t)3 * g->N * g->tiles.nbox * g->fsz;
    double* qc = nullptr;
    void* vc = nullptr;
    hipEvent_t ea = nullptr, eb = nullptr;
    hipError_t e = hipMalloc((void**)&qc, qbytes);
    if (e == hipSuccess) e = hipMalloc(&vc, vbytes);
    if (e == hipSuccess) e = hipEventCreate(&ea);
    if (e == hipSuccess) e = hipEventCreate(&eb);
    const uint32_t timing = g->timing;
    g->timing = 0;
    const Tiles start = g->tiles;
    int best[3] = {start.tx, start.ty, start.tz};
    float best_ms = 0.0f;
    bool have = false;
    // every candidate steps copies of the same state: one untimed step
    // (binning from the previous order), then nsteps timed ones
    auto trial = [&](int tx, int ty, int tz) {
        if (e != hipSuccess || st != MB_OK) return;
        st = set_tiles(g, tx, ty, tz);
        if (st != MB_OK) return;
        if (M > 0) e = hipMemcpyAsync(qc, q, (size_t)M * 3 * sizeof(double),
                                      hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(vc, v, vbytes, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return;
        st = step_impl(g, sp, P, qc, vc, Fext, nullptr, nullptr, nullptr, nullptr, 1, s);
        if (st != MB_OK) return;
        e = hipEventRecord(ea, s);
        if (e == hipSuccess)
            st = step_impl(g, sp, P, qc, vc, Fext, nullptr, nullptr, nullptr, nullptr, nsteps, s);
        if (st != MB_OK) return;
        e = hipEventRecord(eb, s);
        if (e == hipSuccess) e = hipEventSynchronize(eb);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ea, eb);
        if (e == hipSuccess && (!have || ms < best_ms)) {
            have = true;
            best_ms = ms;
            best[0] = tx;
            best[1] = ty;
            best[2] = tz;
        }
    };
#define MB_SHAPE(X, Y, Z) \
    if (tiles_fit(g->L, X, Y, Z)) trial(X, Y, Z);
    MB_TILE_SHAPES(MB_SHAPE)
#undef MB_SHAPE
    g->timing = timing;
    if (e == hipSuccess && st == MB_OK) st = set_tiles(g, best[0], best[1], best[2]);
    else (void)set_tiles(g, start.tx, start.ty, start.tz);
    if (ea) (void)hipEventDestroy(ea);
    if (eb) (void)hipEventDestroy(eb);
    if (qc) (void)hipFree(qc);
    if (vc) (void)hipFree(vc);
    if (st != MB_OK) return st;
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? MB_ERR_NOMEM : from_hip(e);
    if (shape_out) {
        shape_out[0] = best[0];
        shape_out[1] = best[1];
        shape_out[2] = best[2];
    }
    return MB_OK;
}

mb_status mb_grid_set_timing(mb_grid* g, uint32_t kernel_mask) {
    if (!g) return MB_ERR_INVALID;
    g->timing = kernel_mask;
    for (int i = 0; i < K_NUM; ++i) {
        g->acc_ms[i] = 0.0;
        g->acc_n[i] = 0;
    }
    return MB_OK;
}

mb_status mb_grid_kernel_times(mb_grid* g, void* stream, double* ms_out,
                               int64_t* launches_out, int32_t cap,
                               int32_t* n_out) {
    if (!g || cap < 0 || (cap > 0 && (!ms_out || !launches_out))) return MB_ERR_INVALID;
    mb_status st = enter(g);
    if (st != MB_OK) return st;
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return from_hip(e);
    for (auto& tp : g->pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, tp.a, tp.b) == hipSuccess) {
            g->acc_ms[tp.id] += ms;
            g->acc_n[tp.id] += 1;
        }
        g->free_events.push_back(tp.a);
        g->free_events.push_back(tp.b);
    }
    g->pending.clear();
    for (int i = 0; i < cap && i < K_NUM; ++i) {
        ms_out[i] = g->acc_ms[i];
        launches_out[i] = g->acc_n[i];
    }
    if (n_out) *n_out = K_NUM;
    return MB_OK;
}

// ---- Allocation-free step: the grid's workspace in a static device array.
}  // extern "C"

// The scratch of mb_step_noalloc: one array per device (each GPU the library
// runs on holds it until the process ends).  Host code never uses its name
// as an address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[MB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), looked up once.
mb_status scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return MB_ERR_DEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return MB_ERR_DEVICE;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MB_OK;
}
}  // namespace

extern "C" {

mb_status mb_step_noalloc(const mb_grid_desc* desc, const mb_springs* sp, int64_t P,
                          double* q, void* v, const double* Fext, double* u_out,
                          double* U0_out, double* diag_out, int32_t nsteps, void* stream) {
    if (!desc || !sp) return MB_ERR_INVALID;
    const mb_grid_desc d = *desc;
    const mb_status ds = desc_status(d, 1);
    if (ds != MB_OK) return ds;
    if (P < 0 || P * sp->nb > d.max_blobs) return MB_ERR_INVALID;
    const WsLayout w = ws_layout(d, 1);
    if (w.total > MB_NOALLOC_SCRATCH_BYTES) return MB_ERR_UNSUPPORTED;
    int dev = 0;
    if (!device_ok(&dev)) return MB_ERR_DEVICE;
    void* base = nullptr;
    mb_status st = scratch_address(dev, &base);
    if (st != MB_OK) return st;
    // a grid handle on the stack over the static scratch (no allocation:
    // its timing vectors stay empty)
    mb_grid g{};
    g.d = d;
    g.device = dev;
    g.L = d.L;
    g.NC = d.L / 2 + 1;
    g.N = (int64_t)d.L * d.L * d.L;
    g.fsz = d.precision == MB_MIXED ? 4 : 8;
    g.nblk_x = fft_x_blocks(d.L, d.precision);
    g.tiles = default_tiles(d.L, 1);
    g.btiles = make_box_tiles(d.L, g.tiles);
    link_box_tiles(g.tiles, g.btiles);
    g.rec_size = record_size(d.precision);
    g.force_blocks_cap = (int)std::max<int64_t>(d.max_blobs, 1);
    g.ws_owned = false;
    ws_bind(&g, base);
    set_scan_blocks(&g);
    // tables, zero counts, partial sums and flag, on the caller's stream by
    // kernels (the array keeps the last call's contents)
    hipError_t e = init_workspace(&g, (hipStream_t)stream);
    if (e != hipSuccess) return from_hip(e);
    return step_impl(&g, sp, P, q, v, Fext, nullptr, u_out, U0_out, diag_out, nsteps, stream);
}

}  // extern "C"
