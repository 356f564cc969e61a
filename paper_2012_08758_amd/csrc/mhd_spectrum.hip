// Magnetic power spectrum E_B(k) of a run's current state (Section 5.3), on the device.
//
// B = curl A with the sixth-order first derivative is a circulant operator, so its
// discrete Fourier transform is B_hat(k) = i kappa(k) x A_hat(k), kappa_a the modified
// wavenumber of the first-derivative stencil along axis a.  The three A components are
// transformed in FP64 (whatever the run precision) by a mixed-radix Stockham FFT written
// here, one axis per pass, each pass streaming whole lines through LDS:
//   x: real lines, two per complex transform, unpacked to the half spectrum m = 0..nx/2;
//   y, z: complex lines strided in memory, P neighbouring lines per block so that every
//         global access is a run of P consecutive 16-byte values.
// A binning pass forms |kappa x A_hat|^2 (+ the mean field at k = 0), weights the half
// spectrum, and sums the energy into shells s - 1/2 <= |k|/dk < s + 1/2 with a
// segmented wave scan (shells grow monotonically along a line) into per-wave LDS
// accumulators, then per-block partials and a fixed-order final sum: the result is
// bit-reproducible.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mhd_host.h"

namespace mhd {
namespace spec {

constexpr int NT = 256;        // threads per block of the binning kernels
constexpr int NTF = 512;       // threads per block of the FFT kernels
constexpr int MAXN = 4096;     // longest transform
// complex FP64 values of one block's lines in LDS: LC_SHORT for lines of at most 1024
// points (next to a 16 KiB twiddle table), LC_LONG up to MAXN (64 KiB table)
constexpr int LC_SHORT = 4096;
constexpr int LC_LONG = 4096;
constexpr int MAXST = 16;      // most radix stages of one transform
constexpr int BIN_BLOCKS = 2048;

struct Plan {
    int n;         // transform length
    int lp;        // log2 of P, the number of lines one block transforms together
    int nst;       // number of radix stages
    int r[MAXST];  // radices in stage order
};

__device__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }

// R-point DFT o[k] = sum_q t[q] w_R^{qk}, w_R = exp(-2 pi i / R) = tw[n/R].
template <int R>
__device__ inline void small_dft(const double2 *t, double2 *o, const double2 *tw, int nr)
{
    if constexpr (R == 2) {
        o[0] = cadd(t[0], t[1]);
        o[1] = csub(t[0], t[1]);
    } else if constexpr (R == 4) {
        const double2 y0 = cadd(t[0], t[2]), y1 = csub(t[0], t[2]);
        const double2 y2 = cadd(t[1], t[3]), d = csub(t[1], t[3]);
        const double2 y3 = make_double2(d.y, -d.x);  // -i (t1 - t3)
        o[0] = cadd(y0, y2);
        o[2] = csub(y0, y2);
        o[1] = cadd(y1, y3);
        o[3] = csub(y1, y3);
    } else {
#pragma unroll
        for (int k = 0; k < R; k++) {
            double2 acc = t[0];
#pragma unroll
            for (int q = 1; q < R; q++) acc = cadd(acc, cmul(t[q], tw[((q * k) % R) * nr]));
            o[k] = acc;
        }
    }
}

// One in-place Stockham stage of radix R on P interleaved lines (element t of line p
// at buf[t * P + p]).  After the stages before it, index g + G_prev f holds the length-L
// transform f of the subsequence g (G_prev = n / L); this stage combines R of them:
//   out[g + G (f + L k)] = sum_q w_R^{qk} w_{LR}^{qf} in[g + G (q + R f)],  G = n / (L R).
// Every thread reads all its butterflies' inputs, the block synchronises, then writes.
template <int R, int LC>
__device__ inline void fft_stage(double2 *buf, const double2 *tw, int n, int lp, int L)
{
    constexpr int NB = (LC / R + NTF - 1) / NTF;
    const int G = n / (L * R);
    const int nr = n / R;
    const int nbf = nr << lp;
    const int pm = (1 << lp) - 1;
    double2 v[NB][R];
#pragma unroll
    for (int j = 0; j < NB; j++) {
        const int i = (int)threadIdx.x + j * NTF;
        if (i < nbf) {
            const int p = i & pm, b = i >> lp;
            const int f = b / G, g = b - f * G;
#pragma unroll
            for (int q = 0; q < R; q++) {
                double2 x = buf[((g + G * (q + R * f)) << lp) + p];
                if (q) x = cmul(x, tw[q * f * G]);
                v[j][q] = x;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NB; j++) {
        const int i = (int)threadIdx.x + j * NTF;
        if (i < nbf) {
            const int p = i & pm, b = i >> lp;
            const int f = b / G, g = b - f * G;
            double2 o[R];
            small_dft<R>(v[j], o, tw, nr);
#pragma unroll
            for (int k = 0; k < R; k++) buf[((g + G * (f + L * k)) << lp) + p] = o[k];
        }
    }
    __syncthreads();
}

template <int LC>
__device__ inline void run_stages(double2 *buf, const double2 *tw, const Plan &pl)
{
    int L = 1;
    for (int s = 0; s < pl.nst; s++) {
        const int r = pl.r[s];
        switch (r) {
            case 4: fft_stage<4, LC>(buf, tw, pl.n, pl.lp, L); break;
            case 2: fft_stage<2, LC>(buf, tw, pl.n, pl.lp, L); break;
            case 3: fft_stage<3, LC>(buf, tw, pl.n, pl.lp, L); break;
            case 5: fft_stage<5, LC>(buf, tw, pl.n, pl.lp, L); break;
            default: fft_stage<7, LC>(buf, tw, pl.n, pl.lp, L); break;
        }
        L *= r;
    }
}

// x pass: real lines of the three A components (run precision) -> half spectra in W.
// Real lines 2p and 2p+1 of the block travel as the real and imaginary part of
// complex line p and are separated after the transform:
//   X_a[m] = (Z[m] + conj Z[n-m]) / 2,  X_b[m] = -i (Z[m] - conj Z[n-m]) / 2.
template <typename T, int TW, int LC>
__global__ __launch_bounds__(NTF) void k_fft_x(const T *__restrict__ a0, const T *__restrict__ a1,
                                              const T *__restrict__ a2, double2 *__restrict__ W,
                                              long long cstride, long long nlines, int nh,
                                              const double2 *__restrict__ twg, Plan pl)
{
    __shared__ __align__(16) double2 buf[LC];
    __shared__ __align__(16) double2 tw[TW];
    const int c = blockIdx.y;
    const T *src = c == 0 ? a0 : (c == 1 ? a1 : a2);
    const int n = pl.n, lp = pl.lp;
    const long long line0 = (long long)blockIdx.x << (lp + 1);
    for (int i = threadIdx.x; i < n; i += NTF) tw[i] = twg[i];
    double *bd = reinterpret_cast<double *>(buf);
    // the block's 2P lines are one contiguous run of the array; (line, t) of element i
    // advance by a fixed step instead of a division per element
    const int tot = n << (lp + 1);
    const T *blk = src + line0 * n;
    const long long valid = (nlines - line0) * n;  // elements of the run inside the array
    {
        const int drl = NTF / n, dt = NTF - drl * n;
        int rl = (int)threadIdx.x / n, t = (int)threadIdx.x - rl * n;
        for (int i = threadIdx.x; i < tot; i += NTF) {
            const double v = i < valid ? (double)blk[i] : 0.0;
            bd[2 * ((t << lp) + (rl >> 1)) + (rl & 1)] = v;
            t += dt;
            rl += drl;
            if (t >= n) {
                t -= n;
                rl++;
            }
        }
    }
    __syncthreads();
    run_stages<LC>(buf, tw, pl);
    double2 *dst = W + c * cstride + line0 * nh;
    const int toth = nh << (lp + 1);
    const long long validh = (nlines - line0) * nh;
    {
        const int drl = NTF / nh, dm = NTF - drl * nh;
        int rl = (int)threadIdx.x / nh, m = (int)threadIdx.x - rl * nh;
        for (int i = threadIdx.x; i < toth; i += NTF) {
            if (i < validh) {
                const int p = rl >> 1;
                const double2 z = buf[(m << lp) + p];
                const double2 w = buf[((m == 0 ? 0 : n - m) << lp) + p];
                dst[i] = (rl & 1) ? make_double2(0.5 * (z.y + w.y), -0.5 * (z.x - w.x))
                                  : make_double2(0.5 * (z.x + w.x), 0.5 * (z.y - w.y));
            }
            m += dm;
            rl += drl;
            if (m >= nh) {
                m -= nh;
                rl++;
            }
        }
    }
}

// y and z passes: complex lines of length n with element stride S, in place.  Line
// (o, l) starts at o * S * n + l, l in [0, I); a block takes P neighbouring l.
template <int TW, int LC>
__global__ __launch_bounds__(NTF) void k_fft_s(double2 *__restrict__ W, long long cstride, long long S,
                                              long long I, int nchunk, const double2 *__restrict__ twg,
                                              Plan pl)
{
    __shared__ __align__(16) double2 buf[LC];
    __shared__ __align__(16) double2 tw[TW];
    const int n = pl.n, lp = pl.lp, pm = (1 << lp) - 1;
    const int o = blockIdx.x / nchunk, ch = blockIdx.x - o * nchunk;
    const long long l0 = (long long)ch << lp;
    double2 *base = W + blockIdx.y * cstride + (long long)o * S * n + l0;
    for (int i = threadIdx.x; i < n; i += NTF) tw[i] = twg[i];
    const int tot = n << lp;
    for (int i = threadIdx.x; i < tot; i += NTF) {
        const int p = i & pm, t = i >> lp;
        buf[i] = l0 + p < I ? base[p + t * S] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    run_stages<LC>(buf, tw, pl);
    for (int i = threadIdx.x; i < tot; i += NTF) {
        const int p = i & pm, t = i >> lp;
        if (l0 + p < I) base[p + t * S] = buf[i];
    }
}

struct BinArgs {
    long long cstride;     // complex values per component in W
    int nx, ny, nz, nh;
    int nsh, lpb;          // shells; (ky, kz) lines per block
    double rx, ry, rz;     // max(L) / L_a: wavenumber index -> units of dk
    double b0[3];          // Ncell * B_ext: the k = 0 coefficient of the mean field
};

// Energy per half-spectrum element, summed into shells.  Each wave owns one LDS
// accumulator array and walks its lines in 64-element chunks: within a chunk the
// shell index never decreases, so an inclusive segmented scan leaves each run's sum
// in its last lane, and those lanes (distinct shells) add into the wave's array.
template <int NSH>
__global__ __launch_bounds__(NT) void k_spec_bin(const double2 *__restrict__ W, const double *__restrict__ kx,
                                                 const double *__restrict__ ky, const double *__restrict__ kz,
                                                 BinArgs a, double *__restrict__ part)
{
    constexpr int NW = NT / 64;
    __shared__ double acc[NW][NSH];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < NW * NSH; i += NT) (&acc[0][0])[i] = 0.0;
    __syncthreads();
    const long long nlines = (long long)a.ny * a.nz;
    const long long L0 = (long long)blockIdx.x * a.lpb;
    const long long L1 = L0 + a.lpb < nlines ? L0 + a.lpb : nlines;
    for (long long line = L0 + wv; line < L1; line += NW) {
        const int jz = (int)(line / a.ny), jy = (int)(line - (long long)jz * a.ny);
        const int my = jy <= a.ny / 2 ? jy : jy - a.ny;
        const int mz = jz <= a.nz / 2 ? jz : jz - a.nz;
        const double ay = __dmul_rn((double)my, a.ry), az = __dmul_rn((double)mz, a.rz);
        const double y2 = __dmul_rn(ay, ay), z2 = __dmul_rn(az, az);
        const double kyv = ky[jy], kzv = kz[jz];
        const double2 *wx = W + line * a.nh, *wy = wx + a.cstride, *wz = wy + a.cstride;
        for (int m0 = 0; m0 < a.nh; m0 += 64) {
            const int m = m0 + lane;
            double e = 0.0;
            int s = -1;
            if (m < a.nh) {
                const double2 X = wx[m], Y = wy[m], Z = wz[m];
                const double kxv = kx[m];
                double2 cx = make_double2(kyv * Z.x - kzv * Y.x, kyv * Z.y - kzv * Y.y);
                double2 cy = make_double2(kzv * X.x - kxv * Z.x, kzv * X.y - kxv * Z.y);
                double2 cz = make_double2(kxv * Y.x - kyv * X.x, kxv * Y.y - kyv * X.y);
                if (line == 0 && m == 0) {
                    cx.x += a.b0[0];
                    cy.x += a.b0[1];
                    cz.x += a.b0[2];
                }
                e = cx.x * cx.x + cx.y * cx.y + cy.x * cy.x + cy.y * cy.y + cz.x * cz.x + cz.y * cz.y;
                if (m != 0 && 2 * m != a.nx) e *= 2.0;  // the conjugate half m' = nx - m
                const double ax = __dmul_rn((double)m, a.rx);
                const double q = __dadd_rn(__dadd_rn(__dmul_rn(ax, ax), y2), z2);
                s = (int)floor(__dadd_rn(__dsqrt_rn(q), 0.5));
                s = s < a.nsh ? s : a.nsh - 1;  // never above the corner's shell; kept in range regardless
            }
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const double eu = __shfl_up(e, off, 64);
                const int su = __shfl_up(s, off, 64);
                if (lane >= off && su == s) e += eu;
            }
            const int sn = __shfl_down(s, 1, 64);
            if (s >= 0 && (lane == 63 || sn != s)) acc[wv][s] += e;
        }
    }
    __syncthreads();
    for (int s = threadIdx.x; s < a.nsh; s += NT) {
        double t = acc[0][s];
#pragma unroll
        for (int w = 1; w < NW; w++) t += acc[w][s];
        part[(long long)blockIdx.x * a.nsh + s] = t;
    }
}

// out[s] = scale * sum over blocks of part[b][s], in a fixed order (shells s < cap).
__global__ __launch_bounds__(NT) void k_spec_final(const double *__restrict__ part, int nblk, int nsh,
                                                   double scale, double *__restrict__ out, int cap)
{
    __shared__ double sh[NT];
    const int s = blockIdx.x;
    double t = 0.0;
    for (int b = threadIdx.x; b < nblk; b += NT) t += part[(long long)b * nsh + s];
    sh[threadIdx.x] = t;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0 && s < cap) out[s] = sh[0] * scale;
}


// Twiddles exp(-2 pi i j / n) of the three axes and the modified wavenumbers of the
// first-derivative stencil, (45 sin w - 9 sin 2w + sin 3w) / (30 h) with w = 2 pi m / n,
// computed on the device (FP64 sincospi / sinpi; within an ulp or two of the host's
// extended-precision tables).  Block y = axis.
struct TableArgs {
    int n[3], nk[3];
    double ih30[3];     // 1 / (30 h)
    double2 *tw[3];
    double *kap[3];
};

__global__ __launch_bounds__(NT) void k_spec_tables(TableArgs a)
{
    const int ax = blockIdx.y;
    const int n = a.n[ax];
    const int j = blockIdx.x * NT + threadIdx.x;
    if (j < n) {
        double sv, cv;
        sincospi(2.0 * (double)j / (double)n, &sv, &cv);
        a.tw[ax][j] = make_double2(cv, -sv);
    }
    if (j < a.nk[ax]) {
        const double u = 2.0 * (double)j / (double)n;  // w / pi
        a.kap[ax][j] = (45.0 * sinpi(u) - 9.0 * sinpi(2.0 * u) + sinpi(3.0 * u)) * a.ih30[ax];
    }
}

// ------------------------------------------------------------------ host side

static int lds_lines(int n) { return n <= 1024 ? LC_SHORT : LC_LONG; }

// Radices 4, 2, 3, 5, 7 in that order; P = the most lines (a power of two, <= 64)
// whose values fit the block's LDS.  False if n has another prime factor or exceeds MAXN.
static bool make_plan(int n, Plan &pl)
{
    std::memset(&pl, 0, sizeof pl);
    if (n < 2 || n > MAXN) return false;
    pl.n = n;
    int m = n;
    for (int r : {4, 2, 3, 5, 7}) {
        while (m % r == 0) {
            if (pl.nst == MAXST) return false;
            pl.r[pl.nst++] = r;
            m /= r;
        }
    }
    if (m != 1) return false;
    while ((1 << (pl.lp + 1)) <= 64 && (n << (pl.lp + 1)) <= lds_lines(n)) pl.lp++;
    return true;
}

struct Geometry {
    int nx, ny, nz, nh, nsh;
    double dk, rx, ry, rz;
};

static Geometry geometry(const mhd_params &p)
{
    Geometry g;
    g.nx = p.nx;
    g.ny = p.ny;
    g.nz = p.nz;
    g.nh = p.nx / 2 + 1;
    const double lmax = std::max(p.lx, std::max(p.ly, p.lz));
    g.dk = 2.0 * M_PI / lmax;
    g.rx = lmax / p.lx;
    g.ry = lmax / p.ly;
    g.rz = lmax / p.lz;
    // shell of the corner wavevector (n_a / 2 per axis), same operation order as the bins
    // (squares in statements of their own, so that no multiply-add is contracted)
    const double ax = (double)(p.nx / 2) * g.rx, ay = (double)(p.ny / 2) * g.ry, az = (double)(p.nz / 2) * g.rz;
    const double x2 = ax * ax, y2 = ay * ay, z2 = az * az;
    g.nsh = (int)std::floor(std::sqrt((x2 + y2) + z2) + 0.5) + 1;
    return g;
}

// exp(-2 pi i j / n), j < n, evaluated in extended precision and rounded.
static void twiddles(int n, std::vector<double2> &out)
{
    out.resize(n);
    for (int j = 0; j < n; j++) {
        const long double th = 2.0L * 3.141592653589793238462643383279502884L * (long double)j / (long double)n;
        out[j] = make_double2((double)cosl(th), (double)-sinl(th));
    }
}

// Modified wavenumber of the sixth-order first derivative for index m of n points:
// (45 sin w - 9 sin 2w + sin 3w) / (30 h), w = 2 pi m / n.
static double kappa(int m, int n, double h)
{
    const long double w = 2.0L * 3.141592653589793238462643383279502884L * (long double)m / (long double)n;
    return (double)((45.0L * sinl(w) - 9.0L * sinl(2.0L * w) + sinl(3.0L * w)) / (30.0L * (long double)h));
}

struct Layout {
    size_t w, tw[3], kap[3], part, out, total;
    int nblk, lpb;
};

static Layout layout(const Geometry &g)
{
    Layout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, 256);
        return at;
    };
    const long long nlines = (long long)g.ny * g.nz;
    L.lpb = (int)std::max<long long>(4, (nlines + BIN_BLOCKS - 1) / BIN_BLOCKS);
    L.nblk = (int)((nlines + L.lpb - 1) / L.lpb);
    L.w = take(sizeof(double2) * 3 * (size_t)g.nh * g.ny * g.nz);
    L.tw[0] = take(sizeof(double2) * g.nx);
    L.tw[1] = take(sizeof(double2) * g.ny);
    L.tw[2] = take(sizeof(double2) * g.nz);
    L.kap[0] = take(sizeof(double) * g.nh);
    L.kap[1] = take(sizeof(double) * g.ny);
    L.kap[2] = take(sizeof(double) * g.nz);
    L.part = take(sizeof(double) * (size_t)L.nblk * g.nsh);
    L.out = take(sizeof(double) * g.nsh);
    L.total = off;
    return L;
}

static mhd_status ensure_workspace(mhd_ctx *c, const Geometry &g, const Layout &L)
{
    if (c->spec_ws && c->spec_bytes >= L.total) return MHD_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("spectrum: ") + hipGetErrorString(e));
    if (c->spec_ws) (void)hipFree(c->spec_ws);
    c->spec_ws = nullptr;
    c->spec_bytes = 0;
    e = hipMalloc(&c->spec_ws, L.total);
    if (e != hipSuccess) {
        c->spec_ws = nullptr;
        (void)hipGetLastError();
        return fail(MHD_E_OOM, "spectrum: workspace allocation of " + std::to_string(L.total) + " bytes failed");
    }
    c->spec_bytes = L.total;
    char *ws = static_cast<char *>(c->spec_ws);
    const int ns[3] = {g.nx, g.ny, g.nz};
    const double h[3] = {c->p.lx / g.nx, c->p.ly / g.ny, c->p.lz / g.nz};
    for (int a = 0; a < 3; a++) {
        std::vector<double2> tw;
        twiddles(ns[a], tw);
        const int nk = a == 0 ? g.nh : ns[a];
        std::vector<double> kap(nk);
        for (int m = 0; m < nk; m++) kap[m] = kappa(m, ns[a], h[a]);
        e = hipMemcpy(ws + L.tw[a], tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(ws + L.kap[a], kap.data(), sizeof(double) * nk, hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("spectrum: ") + hipGetErrorString(e));
    }
    return MHD_OK;
}

template <int TW, int LC>
static void launch_strided(double2 *W, long long cstride, long long S, long long I, long long O,
                           const double2 *tw, const Plan &pl, hipStream_t st)
{
    const int nchunk = (int)((I + (1LL << pl.lp) - 1) >> pl.lp);
    hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fft_s<TW, LC>), dim3((unsigned)(O * nchunk), 3), dim3(NTF), 0, st, W, cstride,
                       S, I, nchunk, tw, pl);
}

static mhd_status plan_all(const mhd_ctx *c, Geometry &g, Plan &px, Plan &py, Plan &pz)
{
    g = geometry(c->p);
    if (!make_plan(g.nx, px) || !make_plan(g.ny, py) || !make_plan(g.nz, pz))
        return fail(MHD_E_UNSUPPORTED, "spectrum: every grid side must be a product of 2, 3, 5 and 7, at most 4096");
    if (g.nsh > 4096) return fail(MHD_E_UNSUPPORTED, "spectrum: more than 4096 shells");
    return MHD_OK;
}

// The passes of one spectrum on the run's stream, in the workspace at ws (tables
// already in place); the first min(cap, nsh) shells land in the device array dout.
template <typename T>
static void launch_passes(const mhd_ctx *c, const Geometry &g, const Layout &L, const Plan &px, const Plan &py,
                          const Plan &pz, char *ws, double *dout, int cap)
{
    double2 *W = reinterpret_cast<double2 *>(ws + L.w);
    const double2 *tw[3] = {reinterpret_cast<double2 *>(ws + L.tw[0]), reinterpret_cast<double2 *>(ws + L.tw[1]),
                            reinterpret_cast<double2 *>(ws + L.tw[2])};
    const double *kap[3] = {reinterpret_cast<double *>(ws + L.kap[0]), reinterpret_cast<double *>(ws + L.kap[1]),
                            reinterpret_cast<double *>(ws + L.kap[2])};
    double *part = reinterpret_cast<double *>(ws + L.part);
    const long long cstride = (long long)g.nh * g.ny * g.nz;
    const long long nlines = (long long)g.ny * g.nz;
    const T *A[3] = {static_cast<const T *>(c->bufs[c->parity][4]), static_cast<const T *>(c->bufs[c->parity][5]),
                     static_cast<const T *>(c->bufs[c->parity][6])};
    hipStream_t s = c->stream;

    const unsigned nbx = (unsigned)((nlines + (2LL << px.lp) - 1) / (2LL << px.lp));
    if (g.nx <= 1024)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fft_x<T, 1024, LC_SHORT>), dim3(nbx, 3), dim3(NTF), 0, s, A[0], A[1], A[2], W,
                           cstride, nlines, g.nh, tw[0], px);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_fft_x<T, MAXN, LC_LONG>), dim3(nbx, 3), dim3(NTF), 0, s, A[0], A[1], A[2], W,
                           cstride, nlines, g.nh, tw[0], px);
    // y: lines along y at stride nh, nh of them per z-plane, nz planes
    if (g.ny <= 1024)
        launch_strided<1024, LC_SHORT>(W, cstride, g.nh, g.nh, g.nz, tw[1], py, s);
    else
        launch_strided<MAXN, LC_LONG>(W, cstride, g.nh, g.nh, g.nz, tw[1], py, s);
    // z: lines along z at stride nh*ny, one set of nh*ny lines
    const long long sz = (long long)g.nh * g.ny;
    if (g.nz <= 1024)
        launch_strided<1024, LC_SHORT>(W, cstride, sz, sz, 1, tw[2], pz, s);
    else
        launch_strided<MAXN, LC_LONG>(W, cstride, sz, sz, 1, tw[2], pz, s);

    BinArgs ba;
    ba.cstride = cstride;
    ba.nx = g.nx;
    ba.ny = g.ny;
    ba.nz = g.nz;
    ba.nh = g.nh;
    ba.nsh = g.nsh;
    ba.lpb = L.lpb;
    ba.rx = g.rx;
    ba.ry = g.ry;
    ba.rz = g.rz;
    const double ncell = (double)c->ncell;
    for (int a = 0; a < 3; a++) ba.b0[a] = ncell * c->p.bext[a];
    if (g.nsh <= 512)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_spec_bin<512>), dim3(L.nblk), dim3(NT), 0, s, W, kap[0], kap[1], kap[2],
                           ba, part);
    else
        hipLaunchKernelGGL(HIP_KERNEL_NAME(k_spec_bin<4096>), dim3(L.nblk), dim3(NT), 0, s, W, kap[0], kap[1],
                           kap[2], ba, part);
    const double vol = c->p.lx * c->p.ly * c->p.lz;
    const double scale = vol / (2.0 * g.dk * ncell * ncell);
    hipLaunchKernelGGL(k_spec_final, dim3(g.nsh), dim3(NT), 0, s, part, L.nblk, g.nsh, scale, dout, cap);
}

template <typename T>
static mhd_status run(mhd_ctx *c, double *out, int32_t cap, int32_t *nshell, double *dk)
{
    Geometry g;
    Plan px, py, pz;
    mhd_status st = plan_all(c, g, px, py, pz);
    if (st != MHD_OK) return st;
    if (nshell) *nshell = g.nsh;
    if (dk) *dk = g.dk;
    if (cap == 0) return MHD_OK;  // query only
    const Layout L = layout(g);
    st = ensure_workspace(c, g, L);
    if (st != MHD_OK) return st;
    char *ws = static_cast<char *>(c->spec_ws);
    double *dout = reinterpret_cast<double *>(ws + L.out);
    launch_passes<T>(c, g, L, px, py, pz, ws, dout, g.nsh);
    hipStream_t s = c->stream;
    hipError_t e = hipGetLastError();
    std::vector<double> host(g.nsh);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), dout, sizeof(double) * g.nsh, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("spectrum: ") + hipGetErrorString(e));
    if (out && cap > 0) std::memcpy(out, host.data(), sizeof(double) * (size_t)std::min<int32_t>(cap, g.nsh));
    return MHD_OK;
}


// ------------------------------------------------------------------ no-allocation variant
//
// For callers that may not allocate device memory (code under stream capture, serving
// loops): the workspace lives in one file-scope device array per GPU, reached through
// its address from hipGetSymbolAddress (the name itself is a host-side stand-in).  All
// calls on one GPU share it and it keeps the last call's contents; every pass writes
// the parts it reads later, so nothing needs clearing.  Calls that overlap on one GPU
// race on it.
constexpr size_t SCRATCH_BYTES = 64ull << 20;
static __device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[MAX_DEVICES] = {};

// the scratch address on the current device (looked up once per device)
static mhd_status scratch_base(char **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("spectrum_noalloc: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MHD_E_UNSUPPORTED, "spectrum_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(MHD_E_DEVICE, std::string("spectrum_noalloc: scratch address: ") + hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    *out = g_scratch_ptr[dev];
    return MHD_OK;
}

template <typename T>
static mhd_status run_noalloc(mhd_ctx *c, double *dout, int32_t cap, int32_t *nshell, double *dk)
{
    Geometry g;
    Plan px, py, pz;
    mhd_status st = plan_all(c, g, px, py, pz);
    if (st != MHD_OK) return st;
    if (nshell) *nshell = g.nsh;
    if (dk) *dk = g.dk;
    if (cap == 0) return MHD_OK;
    const Layout L = layout(g);
    if (L.total > SCRATCH_BYTES)
        return fail(MHD_E_UNSUPPORTED, "spectrum_noalloc: this grid needs a workspace of " + std::to_string(L.total) +
                                           " bytes, above the " + std::to_string(SCRATCH_BYTES) +
                                           "-byte scratch (use mhd_spectrum)");
    char *ws = nullptr;
    st = scratch_base(&ws);
    if (st != MHD_OK) return st;
    TableArgs ta;
    const int ns[3] = {g.nx, g.ny, g.nz};
    const double ls[3] = {c->p.lx, c->p.ly, c->p.lz};
    int nmax = 0;
    for (int a = 0; a < 3; a++) {
        ta.n[a] = ns[a];
        ta.nk[a] = a == 0 ? g.nh : ns[a];
        ta.ih30[a] = 1.0 / (30.0 * (ls[a] / ns[a]));
        ta.tw[a] = reinterpret_cast<double2 *>(ws + L.tw[a]);
        ta.kap[a] = reinterpret_cast<double *>(ws + L.kap[a]);
        nmax = std::max(nmax, ns[a]);
    }
    hipLaunchKernelGGL(k_spec_tables, dim3((nmax + NT - 1) / NT, 3), dim3(NT), 0, c->stream, ta);
    launch_passes<T>(c, g, L, px, py, pz, ws, dout, std::min<int32_t>(cap, g.nsh));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("spectrum_noalloc: ") + hipGetErrorString(e));
    return MHD_OK;
}

}  // namespace spec
}  // namespace mhd

using namespace mhd;

extern "C" {

mhd_status mhd_spectrum(mhd_ctx *c, double *out, int32_t cap, int32_t *nshell, double *dk)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (cap < 0 || (cap > 0 && !out)) return fail(MHD_E_INVALID, "out is NULL or cap < 0");
    return c->p.precision == MHD_FP64 ? spec::run<double>(c, out, cap, nshell, dk)
                                      : spec::run<float>(c, out, cap, nshell, dk);
}

mhd_status mhd_spectrum_noalloc(mhd_ctx *c, double *out_dev, int32_t cap, int32_t *nshell, double *dk)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (cap < 0 || (cap > 0 && !out_dev)) return fail(MHD_E_INVALID, "out_dev is NULL or cap < 0");
    return c->p.precision == MHD_FP64 ? spec::run_noalloc<double>(c, out_dev, cap, nshell, dk)
                                      : spec::run_noalloc<float>(c, out_dev, cap, nshell, dk);
}

mhd_status mhd_spectrum_shells(const mhd_params *p, int32_t *nshell, double *dk, size_t *workspace_bytes)
{
    mhd_status st = check_params(p);
    if (st != MHD_OK) return st;
    const spec::Geometry g = spec::geometry(*p);
    if (nshell) *nshell = g.nsh;
    if (dk) *dk = g.dk;
    if (workspace_bytes) *workspace_bytes = spec::layout(g).total;
    spec::Plan pl;
    if (!spec::make_plan(p->nx, pl) || !spec::make_plan(p->ny, pl) || !spec::make_plan(p->nz, pl))
        return fail(MHD_E_UNSUPPORTED, "spectrum: every grid side must be a product of 2, 3, 5 and 7, at most 4096");
    return MHD_OK;
}

mhd_status mhd_channel_growth_rate(const double *t, const double *e, int64_t n, double *lambda)
{
    if (!t || !e || !lambda) return fail(MHD_E_INVALID, "NULL argument");
    if (n < 2) return fail(MHD_E_INVALID, "need n >= 2 samples");
    double tm = 0.0, ym = 0.0;
    for (int64_t i = 0; i < n; i++) {
        if (!(e[i] > 0.0) || !std::isfinite(e[i]) || !std::isfinite(t[i]))
            return fail(MHD_E_INVALID, "channel energies must be finite and > 0, times finite");
        tm += t[i];
        ym += std::log(e[i]);
    }
    tm /= (double)n;
    ym /= (double)n;
    double sxy = 0.0, sxx = 0.0;
    for (int64_t i = 0; i < n; i++) {
        const double x = t[i] - tm;
        sxy += x * (std::log(e[i]) - ym);
        sxx += x * x;
    }
    if (!(sxx > 0.0)) return fail(MHD_E_INVALID, "all samples at the same time");
    *lambda = 0.5 * sxy / sxx;
    return MHD_OK;
}

}  // extern "C"
