// Fluid solve on the MAC grid by a hand-written 3-D FFT for gfx950.
//
// Kernels are compiled per grid size L (all L = 2^a 3^b, 8 <= L <= 512,
// L a multiple of 8) and per precision, so every radix, stride, twiddle step
// and index division is a compile-time constant.  Spectrum layout
// A[c][z][kx][ky] (kx < L/2 + 1, ky fastest): the x passes transpose through
// LDS, the y pass reads and writes contiguous [kx][ky] blocks, and the z
// pass reads aligned ky segments.
//
//   x forward : right-hand side r = a v + b (7-point Laplacian of v) + f
//               (Crank-Nicolson explicit half; r = f in steady mode), two
//               real rows packed as one complex line, transform along x,
//               unpack the half spectra, transposed store; float64 partial
//               sums of v and f for the mean mode.
//   y         : transform along y (forward or inverse), in place.
//   z+solve   : transform along z, projection and viscous divide per
//               wavevector, mean mode, inverse transform along z.
//   x inverse : rebuild complex lines from row pairs of half spectra
//               (Hermitian extension), inverse transform, store real rows.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mb_box.h"
#include "mb_device.h"
#include "mb_internal.h"

namespace mb {
namespace fft {

constexpr int EPT = 8;  // elements per thread in a line transform

// LDS position of element e within a line: one spare slot after every 16
// elements, so that the radix-16 stage's stores (stride 16) and the
// following stage's loads spread over the banks.
__device__ __forceinline__ constexpr int lpad(int e) { return e + (e >> 4); }
// line stride: room for the padded line, odd
constexpr int line_stride(int L) { return (L + (L - 1) / 16 + 1) | 1; }

// Radix plan: 16s, then 8, 4, 2, then 3s.
constexpr int nstages(int n) {
    int s = 0;
    while (n % 16 == 0) { n /= 16; ++s; }
    while (n % 8 == 0) { n /= 8; ++s; }
    while (n % 4 == 0) { n /= 4; ++s; }
    while (n % 2 == 0) { n /= 2; ++s; }
    while (n % 3 == 0) { n /= 3; ++s; }
    return s;
}
constexpr int radix_at(int n, int k) {
    int s = 0;
    while (n % 16 == 0) { if (s == k) return 16; n /= 16; ++s; }
    while (n % 8 == 0) { if (s == k) return 8; n /= 8; ++s; }
    while (n % 4 == 0) { if (s == k) return 4; n /= 4; ++s; }
    while (n % 2 == 0) { if (s == k) return 2; n /= 2; ++s; }
    while (n % 3 == 0) { if (s == k) return 3; n /= 3; ++s; }
    return 1;
}
constexpr int ns_at(int n, int k) {
    int p = 1;
    for (int i = 0; i < k; ++i) p *= radix_at(n, i);
    return p;
}

// One Stockham stage of radix R on NLINES lines of length N.  Butterfly j
// of a line reads elements j + r N/R through load(line, element),
// multiplies input r by W_N^{r (j mod NS) N/(NS R)}, applies the R-point
// DFT and writes output r to element (j - j mod NS) R + (j mod NS) + r NS
// through store(line, element, value).  With MIDSYNC (loads and stores on
// the same LDS lines) a barrier separates all loads from all stores, so the
// stage runs in place.  Butterflies are spread over the threads with the
// butterfly index fastest, or the line index fastest with LFAST (lanes then
// walk across lines: contiguous when lines are adjacent in memory).
template <typename T, int N, int R, int NS, bool INV, int NLINES, int NTHR, bool LFAST,
          bool MIDSYNC, typename LD, typename ST>
__device__ __forceinline__ void stage_io(const cplx<T>* tw, int tid, const LD& load,
                                         const ST& store) {
    constexpr int NB = N / R;
    constexpr int TOTAL = NB * NLINES;
    constexpr int MAXB = (TOTAL + NTHR - 1) / NTHR;
    constexpr int TSTEP = N / (NS * R);
    cplx<T> v[MAXB][R];
#pragma unroll
    for (int it = 0; it < MAXB; ++it) {
        const int w = tid + it * NTHR;
        if (TOTAL % NTHR == 0 || w < TOTAL) {
            const int line = LFAST ? w % NLINES : w / NB;
            const int j = LFAST ? w / NLINES : w - line * NB;
            const int k = j % NS;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                cplx<T> a = load(line, j + r * NB);
                if (NS > 1 && r > 0) {
                    cplx<T> t = tw[r * k * TSTEP];
                    if (INV) t.y = -t.y;
                    a = cmul(a, t);
                }
                v[it][r] = a;
            }
        }
    }
    if (MIDSYNC) __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXB; ++it) {
        const int w = tid + it * NTHR;
        if (TOTAL % NTHR == 0 || w < TOTAL) {
            const int line = LFAST ? w % NLINES : w / NB;
            const int j = LFAST ? w / NLINES : w - line * NB;
            const int k = j % NS;
            dftR<T, R, INV>(v[it]);
            const int dst = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) store(line, dst + r * NS, v[it][r]);
        }
    }
}

template <typename T, int N, bool INV, int NLINES, int LS, int NTHR, bool LFAST, int S>
__device__ __forceinline__ void middle_stages(cplx<T>* buf, const cplx<T>* tw, int tid) {
    if constexpr (S < nstages(N) - 1) {
        auto ld = [buf](int line, int e) { return buf[line * LS + lpad(e)]; };
        auto st = [buf](int line, int e, cplx<T> x) { buf[line * LS + lpad(e)] = x; };
        stage_io<T, N, radix_at(N, S), ns_at(N, S), INV, NLINES, NTHR, LFAST, true>(tw, tid, ld,
                                                                                     st);
        __syncthreads();
        middle_stages<T, N, INV, NLINES, LS, NTHR, LFAST, S + 1>(buf, tw, tid);
    }
}

// Transform of NLINES lines of length N: the first stage reads through
// `load`, the last writes through `store`, the stages in between work in
// place on the LDS lines buf (element e of line l at buf[l * LS + lpad(e)]).
// FIRST_LDS / LAST_LDS: load / store use buf itself (the stage then needs
// its internal barrier).  A barrier follows every stage but the last; the
// caller orders what comes before the first and after the last.
template <typename T, int N, bool INV, int NLINES, int LS, int NTHR, bool LFAST,
          bool FIRST_LDS, bool LAST_LDS, typename LD, typename ST>
__device__ __forceinline__ void line_fft_io(cplx<T>* buf, const cplx<T>* tw, int tid,
                                            const LD& load, const ST& store) {
    constexpr int S = nstages(N);
    if constexpr (S == 1) {
        stage_io<T, N, N, 1, INV, NLINES, NTHR, LFAST, FIRST_LDS && LAST_LDS>(tw, tid, load,
                                                                           store);
    } else {
        auto ld = [buf](int line, int e) { return buf[line * LS + lpad(e)]; };
        auto st = [buf](int line, int e, cplx<T> x) { buf[line * LS + lpad(e)] = x; };
        stage_io<T, N, radix_at(N, 0), 1, INV, NLINES, NTHR, LFAST, FIRST_LDS>(tw, tid, load,
                                                                            st);
        __syncthreads();
        middle_stages<T, N, INV, NLINES, LS, NTHR, LFAST, 1>(buf, tw, tid);
        stage_io<T, N, radix_at(N, S - 1), ns_at(N, S - 1), INV, NLINES, NTHR, LFAST,
                 LAST_LDS>(tw, tid, ld, store);
    }
}

// In-place transform of LDS lines, ending with a barrier.
template <typename T, int N, bool INV, int NLINES, int LS, int NTHR>
__device__ __forceinline__ void line_fft(cplx<T>* buf, const cplx<T>* tw, int tid) {
    auto ld = [buf](int line, int e) { return buf[line * LS + lpad(e)]; };
    auto st = [buf](int line, int e, cplx<T> x) { buf[line * LS + lpad(e)] = x; };
    line_fft_io<T, N, INV, NLINES, LS, NTHR, false, true, true>(buf, tw, tid, ld, st);
    __syncthreads();
}

// In-place transform of NLINES lines of length N held in LDS at
// buf[idx(line, e)] (any layout), every stage in LDS; ends with a barrier.
template <typename T, int N, bool INV, int NLINES, int NTHR, bool LFAST, int S = 0,
          typename IX>
__device__ __forceinline__ void lds_fft(cplx<T>* buf, const cplx<T>* tw, int tid,
                                        const IX& idx) {
    if constexpr (S < nstages(N)) {
        auto ld = [buf, &idx](int line, int e) { return buf[idx(line, e)]; };
        auto st = [buf, &idx](int line, int e, cplx<T> x) { buf[idx(line, e)] = x; };
        stage_io<T, N, radix_at(N, S), ns_at(N, S), INV, NLINES, NTHR, LFAST, true>(tw, tid,
                                                                                   ld, st);
        __syncthreads();
        lds_fft<T, N, INV, NLINES, NTHR, LFAST, S + 1>(buf, tw, tid, idx);
    }
}

// ---------------------------------------------------------------------------
// Launch geometry per size.
constexpr int largest_even_divisor(int L, int cap) {
    int best = 2;
    for (int d = 2; d <= L && d <= cap; d += 2)
        if (L % d == 0) best = d;
    return best;
}
// rows per block of the x passes (about 256 threads per block)
constexpr int rows_x(int L) { return largest_even_divisor(L, 4096 / L > 2 ? 4096 / L : 2); }
// kx columns per block of the y pass (at least 128 B contiguous per row)
template <typename T>
constexpr int cols_y(int L) {
    int w = 2048 / L;
    if (w < 1) w = 1;
    const int nc = L / 2 + 1;
    return w < nc ? w : nc;
}
// ky columns per block of the z pass (a divisor of L; LDS <= 64 KB for
// float32, 100 KB for float64).  At 128^3 float32, eight columns give 1,040
// blocks of 384 threads, which fill the CUs in one round (sixteen gave 520
// blocks of 768 threads: two per CU, and a nearly empty second round;
// sixteen with 384 threads of sixteen elements, three blocks per CU in one
// round, 18.6 against 15.1 us; four were slower).  Float64 takes four up to
// L = 128 (2,080 blocks of 192 threads at 128^3: 26.5 us against 38.5 us
// with eight) and eight above, where whole 128-byte lines per z row pay
// for one block per CU (256^3: 288 us against 424 us with four).
template <typename T>
constexpr int cols_z(int L) {
    int w = sizeof(T) == 8 ? (L <= 128 ? 4 : 8) : 8;
    const int cap = sizeof(T) == 8 ? 102400 : 65536;
    while (w > 1 && (L % w != 0 || 3 * L * w * 2 * (int)sizeof(T) > cap ||
                     3 * w * L / EPT > 1024))
        w /= 2;
    return w;
}

template <typename T, int L>
struct Geo {
    static constexpr int NC = L / 2 + 1;
    static constexpr int R = rows_x(L);
    static constexpr int NL = R / 2;
    static constexpr int TX = NL * L / EPT;  // threads of an x pass
    static constexpr int LS = line_stride(L); // LDS line stride (complex)
    static constexpr int WY = cols_y<T>(L);
    static constexpr int NCHY = (NC + WY - 1) / WY;
    static constexpr int TY = WY * L / EPT;
    static constexpr int WZ = cols_z<T>(L);
    static constexpr int TZ = 3 * WZ * L / EPT;
    static constexpr int NBX = 3 * L * (L / R);  // blocks of an x pass
    static_assert(NBX % 8 == 0, "x-pass blocks are remapped over the 8 XCDs");
    // inverse plane pass (y and x together, one (component, z) plane per
    // block): the plane as H = L/2 complex columns, row stride PS (room for
    // the padded column H of the staged half spectrum, odd)
    static constexpr int H = L / 2;
    static constexpr int PS = (lpad(H) + 1) | 1;
    static constexpr int PLANE_BYTES = L * PS * 2 * (int)sizeof(T);
    // used when two planes fit in a CU's 160 KB of LDS (float32 L <= 128,
    // float64 L <= 72), or one plane with L <= 144 (float32 L = 144, float64
    // L = 96, 128: faster than the two passes it replaces; float32 L = 192,
    // one block per CU in 1.1 rounds, was slower)
    static constexpr int XY_LDS = PLANE_BYTES + (L + H) * 2 * (int)sizeof(T);
    static constexpr bool XY =
        PLANE_BYTES <= 72 * 1024 || (XY_LDS <= 160 * 1024 && L <= 144);
    // threads: 8 elements each, at most 1,024 (more waves hide more of the
    // latency; at 128^3 float32 18.0 against 18.9 us with 512, float64 32.9
    // against 34.5)
    static constexpr int TXY_RAW = ((L * H / 8 + WAVE - 1) / WAVE) * WAVE;
    static constexpr int TXY = TXY_RAW > 1024 ? 1024 : TXY_RAW;
    static constexpr int NBXY = 3 * L;                         // blocks per box
};

// ---------------------------------------------------------------------------
template <typename T, int L, bool BOX, bool STEADY>
__global__ void __launch_bounds__((Geo<T, L>::TX))
k_x_fwd(const T* __restrict__ v, const T* __restrict__ f, Tiles tl,
        const cplx<T>* __restrict__ tw, T a, T b,
        cplx<T>* __restrict__ A, double* __restrict__ psum) {
    using G = Geo<T, L>;
    constexpr int NC = G::NC, R = G::R, NL = G::NL, NTHR = G::TX, LS = G::LS;
    __shared__ cplx<T> buf[NL * LS];
    __shared__ cplx<T> tws[L];
    __shared__ double red[16];
    const int tid = threadIdx.x;
    // blocks of a box are consecutive (G::NBX per box, a multiple of 8);
    // within a box each XCD takes a contiguous range of (c, z, y) rows, so
    // the rows of the Laplacian's z and y neighbours, read by adjacent
    // blocks, are found in that XCD's L2
    const int box = blockIdx.x / G::NBX;
    const int lb = xcd_remap(blockIdx.x - box * G::NBX, G::NBX);
    const int yb = lb % (L / R);
    const int cz = lb / (L / R);  // c * L + z
    const int z = cz % L;
    const int cbase = (cz - z) * L * L;   // component offset (elements)
    const int y0 = yb * R;
    v += (size_t)box * 3 * L * L * L;
    A += (size_t)box * 3 * L * NC * L;
    for (int i = tid; i < L; i += NTHR) tws[i] = tw[i];
    double sv = 0.0, sf = 0.0;
    const int zm = (z == 0 ? L - 1 : z - 1), zp = (z == L - 1 ? 0 : z + 1);
    // boxed force: the box entries of this z plane and component
    const T* Ec = nullptr;
    AxisSrc bz{};
    if (BOX) {
        Ec = f + ((size_t)box * 3 + cz / L) * tl.n * box_volume(tl);
        bz = box_src_z(tl, z);
    } else {
        f += (size_t)box * 3 * L * L * L;
    }
    // KG iterations (2 KG nodes) per round: all loads of a round, the box
    // entries included (box_entries: loads only, in uniform branches), are
    // issued before its arithmetic.  One iteration: two took 96 registers in
    // float32 (five waves per SIMD, 1.2 rounds of blocks at 128^3); one fits
    // six waves and one round (25.4 against 26.7 us).
    constexpr int KG = 1;
    static_assert(EPT % KG == 0, "rounds of the x pass");
    // a wave's lanes share y when L is a multiple of the wave
    constexpr bool UNI = L % WAVE == 0 && NTHR % L == 0;
    // with UNI, a thread's x (and its neighbours and x box sources) is the
    // same in every round and its line differs by a constant per round, the
    // wave's rows are uniform: each load is a uniform row base plus the
    // thread's fixed x offset
    [[maybe_unused]] const int xu = tid % L;
    [[maybe_unused]] const int line0 = UNI ? __builtin_amdgcn_readfirstlane(tid / L) : 0;
    [[maybe_unused]] const unsigned ox = (unsigned)xu * (unsigned)sizeof(T);
    [[maybe_unused]] const unsigned oxm = (unsigned)(xu == 0 ? L - 1 : xu - 1) * (unsigned)sizeof(T);
    [[maybe_unused]] const unsigned oxp = (unsigned)(xu == L - 1 ? 0 : xu + 1) * (unsigned)sizeof(T);
    [[maybe_unused]] AxisSrc bxu{};
    if constexpr (UNI && BOX) bxu = box_src_x(tl, xu);
#pragma unroll
    for (int k0 = 0; k0 < EPT; k0 += KG) {
        T vc[KG][2], vn[KG][2][6], fv[KG][2];
        T eb[KG][2][4][2];
        if constexpr (UNI && KG == 1) {
            const int line = line0 + k0 * (NTHR / L);
            const char* vb = reinterpret_cast<const char*>(v);
            const char* fb = reinterpret_cast<const char*>(f);
            auto at = [](const char* base, int row, unsigned o) {
                return *reinterpret_cast<const T*>(base + (size_t)row * sizeof(T) + o);
            };
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int y = y0 + 2 * line + hh;
                const int row = cbase + (z * L + y) * L;
                if (!BOX) fv[0][hh] = at(fb, row, ox);
                if (!STEADY) {
                    const int ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
                    vc[0][hh] = at(vb, row, ox);
                    vn[0][hh][0] = at(vb, row, oxm);
                    vn[0][hh][1] = at(vb, row, oxp);
                    vn[0][hh][2] = at(vb, cbase + (z * L + ym) * L, ox);
                    vn[0][hh][3] = at(vb, cbase + (z * L + yp) * L, ox);
                    vn[0][hh][4] = at(vb, cbase + (zm * L + y) * L, ox);
                    vn[0][hh][5] = at(vb, cbase + (zp * L + y) * L, ox);
                }
            }
            if constexpr (BOX) {
#pragma unroll
                for (int hh = 0; hh < 2; ++hh)
                    box_entries(Ec, bxu, box_src_y(tl, y0 + 2 * line + hh), bz, eb[0][hh]);
            }
        } else {
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const int e = tid + (k0 + g) * NTHR;
            const int line = e / L;
            const int x = e - line * L;
            const int xm = x == 0 ? L - 1 : x - 1, xp = x == L - 1 ? 0 : x + 1;
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                const int y = y0 + 2 * line + hh;
                const unsigned row = (unsigned)(cbase + (z * L + y) * L);
                if (!BOX) fv[g][hh] = ld32(f, row + x);
                if (!STEADY) {
                    const int ym = y == 0 ? L - 1 : y - 1, yp = y == L - 1 ? 0 : y + 1;
                    vc[g][hh] = ld32(v, row + x);
                    vn[g][hh][0] = ld32(v, row + xm);
                    vn[g][hh][1] = ld32(v, row + xp);
                    vn[g][hh][2] = ld32(v, (unsigned)(cbase + (z * L + ym) * L + x));
                    vn[g][hh][3] = ld32(v, (unsigned)(cbase + (z * L + yp) * L + x));
                    vn[g][hh][4] = ld32(v, (unsigned)(cbase + (zm * L + y) * L + x));
                    vn[g][hh][5] = ld32(v, (unsigned)(cbase + (zp * L + y) * L + x));
                }
            }
            if constexpr (BOX) {
                const AxisSrc bx = box_src_x(tl, x);
#pragma unroll
                for (int hh = 0; hh < 2; ++hh) {
                    const int y = y0 + 2 * line + hh;
                    const int yu = UNI ? __builtin_amdgcn_readfirstlane(y) : y;
                    box_entries(Ec, bx, box_src_y(tl, yu), bz, eb[g][hh]);
                }
            }
        }
        }
#pragma unroll
        for (int g = 0; g < KG; ++g) {
            const int e = tid + (k0 + g) * NTHR;
            const int line = e / L;
            const int x = e - line * L;
            T val[2];
#pragma unroll
            for (int hh = 0; hh < 2; ++hh) {
                if (BOX) fv[g][hh] = box_entries_sum(eb[g][hh]);
                sf += (double)fv[g][hh];
                if (STEADY) {
                    val[hh] = fv[g][hh];
                } else {
                    sv += (double)vc[g][hh];
                    const T lap = (vn[g][hh][0] + vn[g][hh][1]) + (vn[g][hh][2] + vn[g][hh][3]) +
                                  (vn[g][hh][4] + vn[g][hh][5]) - T(6) * vc[g][hh];
                    val[hh] = a * vc[g][hh] + b * lap + fv[g][hh];
                }
            }
            buf[line * LS + lpad(x)] = cplx<T>{val[0], val[1]};
        }
    }
    __syncthreads();
    line_fft<T, L, false, NL, LS, NTHR>(buf, tws, tid);
    // unpack the two half spectra of each line; store A[c][z][kx][y]
    cplx<T>* out = A + (size_t)cz * NC * L + y0;
    for (int e = tid; e < NC * R; e += NTHR) {
        const int kx = e / R;
        const int rl = e - kx * R;
        const int line = rl >> 1;
        const cplx<T> Z = buf[line * LS + lpad(kx)];
        const cplx<T> Zc = cconj(buf[line * LS + lpad(kx == 0 ? 0 : L - kx)]);
        cplx<T> o;
        if (rl & 1) {  // (Z - Zc) / 2i
            o = cplx<T>{T(0.5) * (Z.y - Zc.y), T(-0.5) * (Z.x - Zc.x)};
        } else {       // (Z + Zc) / 2
            o = cplx<T>{T(0.5) * (Z.x + Zc.x), T(0.5) * (Z.y + Zc.y)};
        }
        st32(out, (unsigned)(kx * L + rl), o);
    }
    // the block's sums of v and f (one barrier; red holds 16 doubles, at
    // most 8 waves of two partials each)
    static_assert(2 * ((NTHR + WAVE - 1) / WAVE) <= 16, "reduction scratch");
    const double wsv = wave_sum(sv), wsf = wave_sum(sf);
    if (tid % WAVE == 0) {
        red[2 * (tid / WAVE)] = wsv;
        red[2 * (tid / WAVE) + 1] = wsf;
    }
    __syncthreads();
    if (tid == 0) {
        double ts = 0.0, tf = 0.0;
        for (int w = 0; w < (NTHR + WAVE - 1) / WAVE; ++w) {
            ts += red[2 * w];
            tf += red[2 * w + 1];
        }
        const size_t pb = (size_t)box * G::NBX + lb;  // component-major order
        psum[2 * pb] = ts;
        psum[2 * pb + 1] = tf;
    }
}

// y pass: block = (component, z plane, WY consecutive kx); the kx rows of
// length L (along ky) are contiguous in A.
template <typename T, int L, bool INV>
__global__ void __launch_bounds__((Geo<T, L>::TY))
k_y(cplx<T>* __restrict__ A, const cplx<T>* __restrict__ tw) {
    using G = Geo<T, L>;
    constexpr int NC = G::NC, W = G::WY, NTHR = G::TY, LS = G::LS;
    __shared__ cplx<T> buf[W * LS];
    __shared__ cplx<T> tws[L];
    const int tid = threadIdx.x;
    const int ch = blockIdx.x % G::NCHY;
    const int cz = blockIdx.x / G::NCHY;  // (box * 3 + c) * L + z
    const int kx0 = ch * W;
    const int wc = NC - kx0 < W ? NC - kx0 : W;
    cplx<T>* base = A + ((size_t)cz * NC + kx0) * L;
    for (int i = tid; i < L; i += NTHR) tws[i] = tw[i];
    // first stage straight from A, last stage straight back (a short last
    // chunk re-reads its first row and stores only its own rows)
    auto gload = [base, wc](int line, int e) {
        return ld32(base, (unsigned)((line < wc ? line : 0) * L + e));
    };
    auto gstore = [base, wc](int line, int e, cplx<T> x) {
        if (line < wc) st32(base, (unsigned)(line * L + e), x);
    };
    __syncthreads();  // twiddles
    line_fft_io<T, L, INV, W, LS, NTHR, false, false, false>(buf, tws, tid, gload, gstore);
}

// z pass fused with the solve: block = (kx, WZ consecutive ky), all three
// components.  Per wavevector m != 0, with D the divergence symbol
// (D_b = (1 - e^{-2 pi i m_b / L}) / h, |D|^2 = sum_b 4 sin^2(pi m_b/L)/h^2):
//   v^ = (r^ - conj(D) (D . r^) / |D|^2) / ((c0 + c1 |D|^2))
// which is the solenoidal projection of eq. vf on the MAC grid followed by
// the Crank-Nicolson (c0 = N rho/dt, c1 = N eta/2) or steady (c0 = 0,
// c1 = N eta) divide, N = L^3 folding in the inverse normalisation.  The
// mean mode is set from float64 sums: mean(v) + (dt/rho) mean(f), or zero.
template <typename T, int L>
__global__ void __launch_bounds__((Geo<T, L>::TZ))
k_z_solve(cplx<T>* __restrict__ A, const cplx<T>* __restrict__ tw,
          const cplx<T>* __restrict__ dsym, const T* __restrict__ d2, T c0, T c1,
          int zero_mean_mode, const double* __restrict__ psum, int per_c, double mv,
          double mf) {
    using G = Geo<T, L>;
    constexpr int NC = G::NC, W = G::WZ, NTHR = G::TZ, LS = G::LS;
    constexpr int NLN = 3 * W;
    __shared__ cplx<T> buf[NLN * LS];
    __shared__ cplx<T> tws[L];
    __shared__ double red[16];
    __shared__ double mean_new[3];
    const int tid = threadIdx.x;
    // blocks of a box are consecutive (NC L / W per box); when their count
    // is a multiple of 8 each XCD takes a contiguous range, so the blocks
    // sharing the cache lines of a ky segment meet in one L2
    constexpr int NZB = NC * (L / W);
    const int box = blockIdx.x / NZB;
    const int lblk = NZB % 8 == 0 ? xcd_remap(blockIdx.x - box * NZB, NZB)
                                  : blockIdx.x - box * NZB;
    const int ch = lblk % (L / W);
    const int kx = lblk / (L / W);
    const int ky0 = ch * W;
    A += (size_t)box * 3 * L * NC * L;
    psum += (size_t)box * 3 * per_c * 2;  // per_c partials per component
    for (int i = tid; i < L; i += NTHR) tws[i] = tw[i];
    if (kx == 0 && ch == 0) {
        for (int c = 0; c < 3; ++c) {
            double s = 0.0;
            for (int i = tid; i < per_c; i += NTHR) {
                const double* p = psum + 2 * (c * per_c + i);
                s += mv * p[0] + mf * p[1];
            }
            s = block_reduce<false>(s, red);
            if (tid == 0) mean_new[c] = zero_mean_mode ? 0.0 : s;
        }
    }
    __syncthreads();  // twiddles, mean mode
    // line (c, w), w fastest: lanes read contiguous ky segments of A; the
    // forward transform reads A and leaves the spectrum in LDS, the inverse
    // reads LDS and writes A
    // unsigned 32-bit offsets from the block's column base (the spectrum of
    // one box is below 4 GiB)
    cplx<T>* Ak = A + (size_t)kx * L + ky0;
    auto gload = [Ak](int line, int z) {
        const int c = line / W, w = line - (line / W) * W;
        return ld32(Ak, (unsigned)((c * L + z) * NC * L + w));
    };
    auto gstore = [Ak](int line, int z, cplx<T> x) {
        const int c = line / W, w = line - (line / W) * W;
        st32(Ak, (unsigned)((c * L + z) * NC * L + w), x);
    };
    cplx<T>* lb = buf;
    auto lload = [lb](int line, int e) { return lb[line * LS + lpad(e)]; };
    auto lstore = [lb](int line, int e, cplx<T> x) { lb[line * LS + lpad(e)] = x; };
    line_fft_io<T, L, false, NLN, LS, NTHR, true, false, true>(buf, tws, tid, gload, lstore);
    __syncthreads();
    const cplx<T> Dx = dsym[kx];
    const T d2x = d2[kx];
    for (int e = tid; e < L * W; e += NTHR) {
        const int w = e % W;
        const int kz = e / W;
        const int ky = ky0 + w;
        cplx<T>* X = buf + w * LS + lpad(kz);
        if (kx == 0 && ky == 0 && kz == 0) {
            X[0] = cplx<T>{(T)mean_new[0], T(0)};
            X[W * LS] = cplx<T>{(T)mean_new[1], T(0)};
            X[2 * W * LS] = cplx<T>{(T)mean_new[2], T(0)};
            continue;
        }
        const cplx<T> Dy = dsym[ky], Dz = dsym[kz];
        const T D2 = d2x + d2[ky] + d2[kz];
        const cplx<T> rx = X[0], ry = X[W * LS], rz = X[2 * W * LS];
        const cplx<T> div = cadd(cadd(cmul(Dx, rx), cmul(Dy, ry)), cmul(Dz, rz));
        const T inv_d2 = field_rcp(D2);
        const T scale = field_rcp(c0 + c1 * D2);
        const cplx<T> g = {div.x * inv_d2, div.y * inv_d2};
        const cplx<T> px = csub(rx, cmul(cconj(Dx), g));
        const cplx<T> py = csub(ry, cmul(cconj(Dy), g));
        const cplx<T> pz = csub(rz, cmul(cconj(Dz), g));
        X[0] = cplx<T>{px.x * scale, px.y * scale};
        X[W * LS] = cplx<T>{py.x * scale, py.y * scale};
        X[2 * W * LS] = cplx<T>{pz.x * scale, pz.y * scale};
    }
    __syncthreads();
    line_fft_io<T, L, true, NLN, LS, NTHR, true, true, false>(buf, tws, tid, lload, gstore);
}

// Inverse x pass: the half spectra of a row pair are staged, combined into
// one complex line Z = X_even + i X_odd (Hermitian extension for kx > L/2,
// imaginary parts of kx = 0 and L/2 dropped), transformed, and the real and
// imaginary parts stored as the two velocity rows.
template <typename T, int L>
__global__ void __launch_bounds__((Geo<T, L>::TX))
k_x_inv(const cplx<T>* __restrict__ A, const cplx<T>* __restrict__ tw,
        T* __restrict__ vout) {
    using G = Geo<T, L>;
    constexpr int NC = G::NC, R = G::R, NL = G::NL, NTHR = G::TX, LS = G::LS;
    constexpr int SS = NC + 1;  // staging row stride
    __shared__ cplx<T> stg[R * SS];
    __shared__ cplx<T> buf[NL * LS];
    __shared__ cplx<T> tws[L];
    const int tid = threadIdx.x;
    const int yb = blockIdx.x % (L / R);
    const int cz = blockIdx.x / (L / R);  // (box * 3 + c) * L + z
    const int y0 = yb * R;
    for (int i = tid; i < L; i += NTHR) tws[i] = tw[i];
    const cplx<T>* in = A + (size_t)cz * NC * L + y0;
    {
        // all loads first (out-of-range slots re-read the first element)
        constexpr int K = (NC * R + NTHR - 1) / NTHR;
        cplx<T> ld[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = tid + k * NTHR;
            const int kx = e / R;
            const int rl = e - kx * R;
            ld[k] = ld32(in, (unsigned)(e < NC * R ? kx * L + rl : 0));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = tid + k * NTHR;
            if (e < NC * R) {
                const int kx = e / R;
                const int rl = e - kx * R;
                cplx<T> X = ld[k];
                if (kx == 0 || kx == L / 2) X.y = T(0);
                stg[rl * SS + kx] = X;
            }
        }
    }
    __syncthreads();
    // first stage: the combined line Z = X_even + i X_odd read from the
    // staged half spectra; last stage: real and imaginary parts stored as
    // the two velocity rows
    const cplx<T>* sg = stg;
    auto ld = [sg](int line, int k) {
        cplx<T> X1, X2;
        if (k <= L / 2) {
            X1 = sg[(2 * line) * SS + k];
            X2 = sg[(2 * line + 1) * SS + k];
        } else {
            X1 = cconj(sg[(2 * line) * SS + (L - k)]);
            X2 = cconj(sg[(2 * line + 1) * SS + (L - k)]);
        }
        return cplx<T>{X1.x - X2.y, X1.y + X2.x};
    };
    T* out = vout + ((size_t)cz * L + y0) * L;
    auto st = [out](int line, int x, cplx<T> zz) {
        st32(out, (unsigned)((2 * line) * L + x), zz.x);
        st32(out, (unsigned)((2 * line + 1) * L + x), zz.y);
    };
    line_fft_io<T, L, true, NL, LS, NTHR, false, false, false>(buf, tws, tid, ld, st);
}

// Inverse plane pass: y and x together for one (component, z) plane per
// block, the plane held in LDS.  The real plane v[y][x] is produced as H =
// L/2 complex columns Z[y][j] = v[y][2j] + i v[y][2j+1]: from the half
// spectrum F[kx][ky] (kx = 0..H, layout A[c][z][kx][ky] of the z pass),
//   Z'[ky][k] = E' + i O',  E' = F[ky][k] + conj F[-ky][H-k],
//   O' = (F[ky][k] - conj F[-ky][H-k]) W^-k   (W = e^{-2 pi i / L}),
// the spectra of the even and odd samples (F[ky][k + H] = conj F[-ky][H-k]
// for a real plane), then inverse transforms along y (L points) and j
// (H points); Z[y][j] is the row pair (v[y][2j], v[y][2j+1]), unnormalised
// like the rest of the solve.  Element (row, column) of the plane sits at
// row * PS + lpad(column).
template <typename T, int L>
__global__ void __launch_bounds__((Geo<T, L>::TXY))
k_xy_inv(const cplx<T>* __restrict__ A, const cplx<T>* __restrict__ tw,
         T* __restrict__ vout) {
    using G = Geo<T, L>;
    constexpr int H = G::H, PS = G::PS, NC = G::NC, NTHR = G::TXY;
    __shared__ cplx<T> buf[L * PS];
    __shared__ cplx<T> tws[L];
    __shared__ cplx<T> twh[H];
    const int tid = threadIdx.x;
    const int cz = blockIdx.x;  // (box * 3 + c) * L + z
    for (int i = tid; i < L; i += NTHR) tws[i] = tw[i];
    for (int i = tid; i < H; i += NTHR) twh[i] = tw[2 * i];
    // stage the half spectrum: F[kx][ky] at row ky, column kx (0..H)
    const cplx<T>* in = A + (size_t)cz * NC * L;
    {
        // every load of the thread issued before the LDS stores (at most 17
        // complex values per thread: K <= (L/2 + 1) L / NTHR)
        constexpr int K = (NC * L + NTHR - 1) / NTHR;
        cplx<T> ld[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = tid + k * NTHR;
            ld[k] = ld32(in, (unsigned)(e < NC * L ? e : 0));
        }
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = tid + k * NTHR;
            if (e < NC * L) {
                const int kx = e / L;
                const int ky = e - kx * L;
                buf[ky * PS + lpad(kx)] = ld[k];
            }
        }
    }
    __syncthreads();
    // Z'[ky][k] in place.  Slot (ky, k) and its partner (-ky, H - k) are
    // formed from each other, so each work item owns both (k = 1 .. H/2;
    // at k = H/2 only ky <= L/2); column 0 pairs with column H:
    // Z'[ky][0] = F[ky][0] + conj F[-ky][H] + i (F[ky][0] - conj F[-ky][H]).
    {
        constexpr int NPAIR = L * (H / 2);  // items (ky, k), k = 1 .. H/2 (k = H/2: ky <= L/2)
        for (int e = tid; e < NPAIR + L / 2 + 1; e += NTHR) {
            if (e < NPAIR) {
                const int k = 1 + e / L;
                const int ky = e - (k - 1) * L;
                if (k == H / 2 && ky > L / 2) continue;
                const int kyn = ky == 0 ? 0 : L - ky;
                const int kn = H - k;
                const cplx<T> F1 = buf[ky * PS + lpad(k)];
                const cplx<T> F2 = buf[kyn * PS + lpad(kn)];
                // slot (ky, k): F1 with conj F2; slot (-ky, H-k): F2 with conj F1
                const cplx<T> w1 = cconj(tws[k]);   // W^-k
                const cplx<T> w2 = cconj(tws[kn]);  // W^-(H-k)
                const cplx<T> e1 = cadd(F1, cconj(F2)), o1 = cmul(csub(F1, cconj(F2)), w1);
                const cplx<T> e2 = cadd(F2, cconj(F1)), o2 = cmul(csub(F2, cconj(F1)), w2);
                buf[ky * PS + lpad(k)] = cplx<T>{e1.x - o1.y, e1.y + o1.x};
                if (kyn != ky || kn != k)
                    buf[kyn * PS + lpad(kn)] = cplx<T>{e2.x - o2.y, e2.y + o2.x};
            } else {
                const int ky = e - NPAIR;  // 0 .. L/2
                const int kyn = ky == 0 ? 0 : L - ky;
                const cplx<T> Fa0 = buf[ky * PS + lpad(0)], FaH = buf[ky * PS + lpad(H)];
                const cplx<T> Fb0 = buf[kyn * PS + lpad(0)], FbH = buf[kyn * PS + lpad(H)];
                const cplx<T> e1 = cadd(Fa0, cconj(FbH)), o1 = csub(Fa0, cconj(FbH));
                const cplx<T> e2 = cadd(Fb0, cconj(FaH)), o2 = csub(Fb0, cconj(FaH));
                buf[ky * PS + lpad(0)] = cplx<T>{e1.x - o1.y, e1.y + o1.x};
                if (kyn != ky) buf[kyn * PS + lpad(0)] = cplx<T>{e2.x - o2.y, e2.y + o2.x};
            }
        }
    }
    __syncthreads();
    auto col = [](int line, int e) { return e * PS + lpad(line); };
    lds_fft<T, L, true, H, NTHR, true>(buf, tws, tid, col);
    // along x; the last stage stores each complex Z'[y][j] as the real pair
    // v[y][2j], v[y][2j+1]
    cplx<T>* out = reinterpret_cast<cplx<T>*>(vout + (size_t)cz * L * L);
    const cplx<T>* lb = buf;
    auto ldl = [lb](int line, int e) { return lb[line * PS + lpad(e)]; };
    auto gst = [out](int line, int e, cplx<T> x) { st32(out, (unsigned)(line * H + e), x); };
    line_fft_io<T, H, true, L, PS, NTHR, false, true, false>(buf, twh, tid, ldl, gst);
}

template <typename T, int L>
hipError_t solve_sized(mb_grid* g, const T* v_in, const T* f, bool boxed, T* v_out,
                       hipStream_t s) {
    using G = Geo<T, L>;
    const bool steady = g->d.mode == MB_STEADY_STOKES;
    const double h = g->d.h;
    const double N = (double)g->N;
    cplx<T>* A = (cplx<T>*)g->d_spec;
    const cplx<T>* tw = (const cplx<T>*)g->d_tw;
    const T a = steady ? T(0) : (T)(g->d.rho / g->d.dt);
    const T b = steady ? T(0) : (T)(0.5 * g->d.eta / (h * h));
    const T* fin = boxed ? (const T*)g->d_box : f;
    const int nbox = g->tiles.nbox;
#define MB_XF(BX, ST)                                                                     \
    MB_LAUNCH(g, K_FFT_X_FWD, s, (k_x_fwd<T, L, BX, ST>), G::NBX * nbox, G::TX, 0, v_in, fin, \
              g->btiles, tw, a, b, A, g->d_psum)
    if (boxed) {
        if (steady) MB_XF(true, true);
        else MB_XF(true, false);
    } else {
        if (steady) MB_XF(false, true);
        else MB_XF(false, false);
    }
#undef MB_XF
    MB_LAUNCH(g, K_FFT_Y_FWD, s, (k_y<T, L, false>), 3 * L * G::NCHY * nbox, G::TY, 0, A,
              tw);
    const T c0 = steady ? T(0) : (T)(g->d.rho / g->d.dt * N);
    const T c1 = steady ? (T)(g->d.eta * N) : (T)(0.5 * g->d.eta * N);
    const double mv = steady ? 0.0 : 1.0 / N;
    const double mf = steady ? 0.0 : g->d.dt / g->d.rho / N;
    const int zm = (steady || g->d.zero_mean) ? 1 : 0;
    MB_LAUNCH(g, K_FFT_Z_SPECTRAL, s, (k_z_solve<T, L>), G::NC * (L / G::WZ) * nbox, G::TZ, 0,
              A, tw, (const cplx<T>*)g->d_dsym, (const T*)g->d_d2, c0, c1, zm,
              g->d_psum, G::NBX / 3, mv, mf);
    if constexpr (G::XY) {
        MB_LAUNCH(g, K_FFT_XY_INV, s, (k_xy_inv<T, L>), G::NBXY * nbox, G::TXY, 0, A, tw,
                  v_out);
    } else {
        MB_LAUNCH(g, K_FFT_Y_INV, s, (k_y<T, L, true>), 3 * L * G::NCHY * nbox, G::TY, 0, A,
                  tw);
        MB_LAUNCH(g, K_FFT_X_INV, s, (k_x_inv<T, L>), G::NBX * nbox, G::TX, 0, A, tw, v_out);
    }
    return hipGetLastError();
}

}  // namespace fft

#define MB_FFT_SIZES(X) \
    X(8) X(16) X(24) X(32) X(48) X(64) X(72) X(96) X(128) X(144) X(192) \
    X(216) X(256) X(288) X(384) X(432) X(512)

template <typename T>
hipError_t fluid_solve(mb_grid* g, const T* v_in, const T* f, T* v_out,
                       hipStream_t s, bool boxed) {
    switch (g->L) {
#define MB_CASE(n) \
    case n: return fft::solve_sized<T, n>(g, v_in, f, boxed, v_out, s);
        MB_FFT_SIZES(MB_CASE)
#undef MB_CASE
    }
    return hipErrorInvalidValue;
}

int fft_x_blocks(int L, int precision) {
    switch (L) {
#define MB_CASE(n) \
    case n: return precision == MB_MIXED ? fft::Geo<float, n>::NBX : fft::Geo<double, n>::NBX;
        MB_FFT_SIZES(MB_CASE)
#undef MB_CASE
    }
    return 0;
}

template hipError_t fluid_solve<float>(mb_grid*, const float*, const float*, float*, hipStream_t, bool);
template hipError_t fluid_solve<double>(mb_grid*, const double*, const double*, double*, hipStream_t, bool);

}  // namespace mb
