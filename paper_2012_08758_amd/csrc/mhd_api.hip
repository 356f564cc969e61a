// C ABI of the MHD solver: contexts (single runs), forcing and initial-condition
// generation, diagnostics, tile-shape selection and autotuning, batched ensembles.
// The serving loop lives in mhd_server.hip.
#include "mhd.h"
#include "mhd_host.h"
#include "mhd_zmarch.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

namespace mhd {

thread_local std::string g_err;

mhd_status fail(mhd_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

// ------------------------------------------------------------------ tile shapes

const Shape SHAPES[NSHAPES] = {
    // register-staged kernel: any grid
    {16, 8, 4, 1, false},   // 0: 512 threads, halo box / cells = 6.0
    {32, 8, 4, 1, false},   // 1: 1024 threads, 5.2
    {8, 8, 4, 1, false},    // 2: 256 threads, small grids
    {16, 8, 8, 2, false},   // 3: 512 threads, 1024 cells, 4.2
    {32, 4, 4, 1, false},   // 4: 512 threads, 7.4
    {32, 4, 8, 2, false},   // 5: 512 threads, 1024 cells, 5.2
    // direct-to-LDS ring kernel: nx a multiple of 16 / sizeof(value), 16-byte aligned fields
    {16, 8, 4, 1, true},    // 6
    {32, 8, 4, 1, true},    // 7
    {8, 8, 4, 1, true},     // 8
    {16, 8, 8, 2, true},    // 9
    {32, 4, 4, 1, true},    // 10
    {32, 4, 8, 2, true},    // 11
    // z-marching column kernel (ring per field in LDS): the tile divides the grid
    {16, 8, 4, 1, true, true},  // 12: FP32 only (the FP64 rings do not fit the LDS)
    {8, 8, 4, 1, true, true},   // 13
    // z-marching kernel with register queues: nx % 32 == 0, ny % 8 == 0
    {32, 8, 1, 1, false, false, true},  // 14
    // the same, FP32 with nx % 64 == 0: substeps 1 and 2 on 64 x 8 tiles of 1024 threads
    {32, 8, 1, 1, false, false, true, true},  // 15
};

// the shape used when `shape` cannot run on a grid: march -> ring -> staged, same box
int shape_fallback(int shape)
{
    if (shape == SHAPE_ZMW) return SHAPE_ZM;
    if (shape == SHAPE_ZM) return 9;
    if (shape == 12) return 6;
    if (shape == 13) return 8;
    return SHAPES[shape].pipe ? shape - 6 : shape;
}

static bool march_lds_fits(int shape, int precision)
{
    const Shape &s = SHAPES[shape];
    if (s.tx == 16 && s.ty == 8 && s.tz == 4)
        return precision == MHD_FP64 ? MarchCfg<double, 16, 8, 4>::FITS : MarchCfg<float, 16, 8, 4>::FITS;
    if (s.tx == 8 && s.ty == 8 && s.tz == 4)
        return precision == MHD_FP64 ? MarchCfg<double, 8, 8, 4>::FITS : MarchCfg<float, 8, 8, 4>::FITS;
    return false;
}

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, int> g_tuned;  // (nx, ny, nz, prec) -> shape

bool shape_eligible(const mhd_params &p, int shape, bool aligned)
{
    if (shape < 0 || shape >= NSHAPES) return false;
    const Shape &s = SHAPES[shape];
    if (s.zm)
        return aligned && p.nx % s.tx == 0 && p.ny % s.ty == 0 && p.nx % (16 / p.precision) == 0 &&
               (!s.wide || (p.precision == MHD_FP32 && p.nx % ZM_WIDE_TX == 0));
    if (!s.pipe) return true;
    const int epl = 16 / p.precision;
    if (!(aligned && p.nx % epl == 0)) return false;
    if (!s.march) return true;
    return march_lds_fits(shape, p.precision) && p.nx % s.tx == 0 && p.ny % s.ty == 0 && p.nz % s.tz == 0 &&
           p.nx >= s.tx + 8 && p.ny >= s.ty + 6;
}

bool shape_fits(const mhd_params &p, int shape)
{
    const Shape &s = SHAPES[shape];
    return p.nx >= s.tx + 8 && p.ny >= s.ty + 6 && p.nz >= s.tz + 6;
}

int default_shape(const mhd_params &p, bool aligned, bool filled)
{
    int want = -1;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tuned.find(std::make_tuple(p.nx, p.ny, p.nz, p.precision));
        if (it != g_tuned.end()) want = it->second;
    }
    if (want < 0) {
        // measured at 512^3: 16x8x8/2 is the fastest FP64 ring shape, 32x4x8/2 the
        // fastest FP32 one; a small grid alone wants the small tile (more work-groups).
        // The z-marching kernel beats both once its columns and segments give at least
        // 1024 work-groups (256^3: 2.64 against 3.59 ms per step in FP64, 1.65 against
        // 1.81 in FP32; 512^3: 18.3 against 26.8 and 11.9 against 12.6); at 128^3 (128
        // work-groups) alone the ring kernel is faster, but in a batch that fills the chip
        // the z-marching kernel wins at any size (48 FP32 runs of 64^3 and 128^3: 13500
        // against 12090 run-steps per second).
        const double n = (double)p.nx * p.ny * p.nz;
        want = (n <= 64.0 * 64 * 64 && !filled) ? 8 : (p.precision == MHD_FP64 ? 9 : 11);
        if (shape_eligible(p, SHAPE_ZM, aligned) && (filled || run_ntiles(p, SHAPE_ZM) >= 1024)) {
            want = SHAPE_ZM;
            if (shape_eligible(p, SHAPE_ZMW, aligned)) want = SHAPE_ZMW;
        }
    }
    while (!shape_eligible(p, want, aligned)) want = shape_fallback(want);
    return want;
}

// ------------------------------------------------------------------ coefficients

// Williamson (1980) third-order 2N Runge-Kutta
static const double RK_A[3] = {0.0, -5.0 / 9.0, -153.0 / 128.0};
static const double RK_B[3] = {1.0 / 3.0, 15.0 / 16.0, 8.0 / 15.0};

template <typename T>
static void fill_coef(const mhd_params &p, Coef<T> &c, DCoef &dc)
{
    const double h[3] = {p.lx / p.nx, p.ly / p.ny, p.lz / p.nz};
    for (int a = 0; a < 3; a++) {
        c.ih1[a] = (T)(1.0 / h[a]);
        dc.ih1[a] = 1.0 / h[a];
        c.ih2[a] = (T)(1.0 / (h[a] * h[a]));
    }
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int q = 0; q < 3; q++) c.ihm[q] = (T)(1.0 / (4.0 * h[pa[q]] * h[pb[q]]));
    c.cs2 = (T)(p.cs * p.cs);
    c.nu = (T)p.nu;
    c.nu3 = (T)(p.nu / 3.0);
    c.nu2_3 = (T)(2.0 * p.nu / 3.0);
    c.eta = (T)p.eta;
    for (int a = 0; a < 3; a++) {
        c.bext[a] = (T)p.bext[a];
        dc.bext[a] = p.bext[a];
    }
    for (int a = 0; a < 3; a++) c.upw[a] = (T)(p.upwind / (60.0 * h[a]));
    const double w1[3] = {W1_1, W1_2, W1_3}, w2[4] = {W2_0, W2_1, W2_2, W2_3};
    for (int a = 0; a < 2; a++) {
        for (int k = 0; k < 3; k++) c.w1[a][k] = (T)(w1[k] / h[a]);
        for (int k = 0; k < 4; k++) c.w2[a][k] = (T)(w2[k] / (h[a] * h[a]));
    }
    for (int role = 0; role < 2; role++) {
        const double f = role == 0 ? p.nu / 3.0 : 1.0;
        for (int k = 0; k < 3; k++) {
            c.wm[role][k] = (T)(f * w2[k + 1] / (4.0 * h[0] * h[1]));
            for (int a = 0; a < 2; a++) c.wq[role][a][k] = (T)(f * w2[k + 1] / (4.0 * h[a] * h[2]));
        }
    }
    for (int s = 0; s < 3; s++) {
        c.bdt[s] = (T)(RK_B[s] * p.dt);
        c.brho[s] = s == 0 ? (T)0 : (T)(RK_B[s] * RK_A[s] / RK_B[s - 1]);
    }
}

// ------------------------------------------------------------------ forcing

static std::vector<std::array<int, 3>> shell_vectors(double kf)
{
    std::vector<std::array<int, 3>> out;
    const double lo2 = (kf - 0.5) * (kf - 0.5), hi2 = (kf + 0.5) * (kf + 0.5);
    const int m = (int)std::floor(kf + 0.5);
    for (int kx = -m; kx <= m; kx++)
        for (int ky = -m; ky <= m; ky++)
            for (int kz = -m; kz <= m; kz++) {
                const double q = (double)(kx * kx + ky * ky + kz * kz);
                if (q >= lo2 && q <= hi2) out.push_back({kx, ky, kz});
            }
    return out;
}

mhd_forcing random_forcing(double kf, double f0, double sigma, uint64_t seed, int64_t n)
{
    static thread_local double cached_kf = -1.0;
    static thread_local std::vector<std::array<int, 3>> shell;
    if (kf != cached_kf) {
        shell = shell_vectors(kf);
        cached_kf = kf;
    }
    mhd_forcing r;
    std::memset(&r, 0, sizeof r);
    r.sigma = sigma;
    r.f0 = f0;
    if (shell.empty()) {
        r.f0 = 0.0;
        r.k[0] = 1;
        r.e[1] = 1.0;
        return r;
    }
    const uint64_t key = sm_key(seed, 1);
    double u[8];
    for (int i = 0; i < 8; i++) u[i] = sm_unif(key, (uint64_t)(8 * n + i));
    size_t si = (size_t)(u[0] * (double)shell.size());
    if (si >= shell.size()) si = shell.size() - 1;
    const auto k = shell[si];
    const double kn = std::sqrt((double)(k[0] * k[0] + k[1] * k[1] + k[2] * k[2]));
    const double kh[3] = {k[0] / kn, k[1] / kn, k[2] / kn};
    bool found = false;
    double e[3] = {0, 0, 0};
    for (int cand = 0; cand < 2 && !found; cand++) {
        const double a = u[1 + 2 * cand], b = u[2 + 2 * cand];
        const double z = 2.0 * a - 1.0;
        const double s = std::sqrt(std::max(0.0, 1.0 - z * z));
        const double ph = 2.0 * M_PI * b;
        const double c[3] = {s * std::cos(ph), s * std::sin(ph), z};
        if (std::fabs(kh[0] * c[0] + kh[1] * c[1] + kh[2] * c[2]) <= 0.99) {
            e[0] = c[0]; e[1] = c[1]; e[2] = c[2];
            found = true;
        }
    }
    if (!found) {
        int ax = 0;
        for (int a = 1; a < 3; a++)
            if (std::fabs(kh[a]) < std::fabs(kh[ax])) ax = a;
        e[ax] = 1.0;
    }
    for (int a = 0; a < 3; a++) { r.k[a] = k[a]; r.e[a] = e[a]; }
    r.phi = M_PI * (2.0 * u[5] - 1.0);
    return r;
}

mhd_status check_forcing(const mhd_forcing &f)
{
    if (!std::isfinite(f.phi) || !std::isfinite(f.sigma) || !std::isfinite(f.f0))
        return fail(MHD_E_INVALID, "forcing: non-finite phi, sigma or f0");
    if (f.f0 == 0.0) return MHD_OK;
    const double kk = (double)f.k[0] * f.k[0] + (double)f.k[1] * f.k[1] + (double)f.k[2] * f.k[2];
    if (kk == 0.0) return fail(MHD_E_INVALID, "forcing: k = 0");
    const double ee = f.e[0] * f.e[0] + f.e[1] * f.e[1] + f.e[2] * f.e[2];
    if (!(std::fabs(ee - 1.0) < 1e-6)) return fail(MHD_E_INVALID, "forcing: e is not a unit vector");
    const double ke = f.k[0] * f.e[0] + f.k[1] * f.e[1] + f.k[2] * f.e[2];
    if (!(1.0 - ke * ke / kk > 1e-12)) return fail(MHD_E_INVALID, "forcing: e is parallel to k");
    return MHD_OK;
}

// Write one step's forcing block: the two real vectors a, b with
// f = a cos(theta) + b sin(theta), and per-axis phase tables whose product is
// exp(i theta), theta = K.x + phi.  From Eqs. forcing, fnorm and feigen:
// f = Re{N f_k e^{i theta}} = N Re(f_k) cos - N Im(f_k) sin, with
// Re f_k = K x (K x e) / D and Im f_k = -sigma |K| (K x e) / D.
// cos and sin of 2 pi m / n, m = 0..n-1 (interleaved): the phases of one axis for any
// integer wave number are a permutation of this table
static std::vector<double> unit_circle(int n)
{
    std::vector<double> u(2 * (size_t)n);
    for (int m = 0; m < n; m++) {
        const double th = 2.0 * M_PI * (double)m / (double)n;
        u[2 * (size_t)m] = std::cos(th);
        u[2 * (size_t)m + 1] = std::sin(th);
    }
    return u;
}

// The forcing block of one step: head a, b (f = a cos(theta) + b sin(theta) with theta =
// k.x + phi), the on-flag, then per axis the (cos, sin) of k_a x_a (x also + phi) at every
// index, gathered from the axis's unit-circle table (u[a], from unit_circle(n_a)) and, for
// x, rotated by phi.
template <typename T>
static void forcing_block(const mhd_params &p, const mhd_forcing &f, T *blk, const std::vector<double> *u)
{
    constexpr int W = FSLOT<T>;
    for (int i = 0; i < FHEAD; i++) blk[i] = (T)0;
    T *Ex = blk + FHEAD, *Ey = Ex + W * p.nx, *Ez = Ey + W * p.ny;
    for (int i = 0; i < W * (p.nx + p.ny + p.nz); i++) Ex[i] = (T)0;
    if (f.f0 == 0.0) return;
    const double L[3] = {p.lx, p.ly, p.lz};
    double K[3];
    for (int a = 0; a < 3; a++) K[a] = 2.0 * M_PI * f.k[a] / L[a];
    const double kk = K[0] * K[0] + K[1] * K[1] + K[2] * K[2];
    const double kn = std::sqrt(kk);
    const double ke = K[0] * f.e[0] + K[1] * f.e[1] + K[2] * f.e[2];
    const double kxe[3] = {K[1] * f.e[2] - K[2] * f.e[1], K[2] * f.e[0] - K[0] * f.e[2],
                           K[0] * f.e[1] - K[1] * f.e[0]};
    const double kkxe[3] = {K[1] * kxe[2] - K[2] * kxe[1], K[2] * kxe[0] - K[0] * kxe[2],
                            K[0] * kxe[1] - K[1] * kxe[0]};
    const double D = std::sqrt(1.0 + f.sigma * f.sigma) * kk * std::sqrt(1.0 - ke * ke / kk);
    const double N = f.f0 * p.cs * std::sqrt(kn * p.cs / p.dt);
    for (int a = 0; a < 3; a++) {
        blk[a] = (T)(N * kkxe[a] / D);
        blk[3 + a] = (T)(N * f.sigma * kn * kxe[a] / D);
    }
    blk[6] = (T)1;
    const int n[3] = {p.nx, p.ny, p.nz};
    T *tab[3] = {Ex, Ey, Ez};
    const double cp = std::cos(f.phi), sp = std::sin(f.phi);
    for (int a = 0; a < 3; a++) {
        const int64_t na = n[a];
        const double *U = u[a].data();
        for (int64_t i = 0; i < na; i++) {
            int64_t m = ((int64_t)f.k[a] * i) % na;
            if (m < 0) m += na;
            const double c = U[2 * m], sn = U[2 * m + 1];
            tab[a][W * i] = (T)(a == 0 ? c * cp - sn * sp : c);
            tab[a][W * i + 1] = (T)(a == 0 ? sn * cp + c * sp : sn);
        }
    }
}

int forcing_stride(const mhd_params &p)
{
    // head, then one 16-byte slot per index of each axis; blocks start 64-byte aligned
    int s = FHEAD + (16 / p.precision) * (p.nx + p.ny + p.nz);
    return (s + 7) & ~7;
}

// ------------------------------------------------------------------ validation

mhd_status check_params(const mhd_params *p)
{
    if (!p) return fail(MHD_E_INVALID, "params is NULL");
    if (p->nx < 8 || p->ny < 8 || p->nz < 8) return fail(MHD_E_INVALID, "grid: every n must be >= 8");
    if (p->nx > 65535 || p->ny > 65535 || p->nz > 65535) return fail(MHD_E_INVALID, "grid: n > 65535");
    if ((double)p->nx * p->ny * p->nz >= 4294967296.0) return fail(MHD_E_INVALID, "grid: more than 2^32 cells");
    if (p->precision != MHD_FP32 && p->precision != MHD_FP64)
        return fail(MHD_E_INVALID, "precision must be MHD_FP32 (4) or MHD_FP64 (8)");
    if (!(p->lx > 0 && p->ly > 0 && p->lz > 0)) return fail(MHD_E_INVALID, "box lengths must be > 0");
    if (!(p->dt > 0) || !std::isfinite(p->dt)) return fail(MHD_E_INVALID, "dt must be finite and > 0");
    if (!(p->nu >= 0) || !(p->eta >= 0) || !(p->cs >= 0)) return fail(MHD_E_INVALID, "nu, eta, cs must be >= 0");
    if (!std::isfinite(p->nu) || !std::isfinite(p->eta) || !std::isfinite(p->cs))
        return fail(MHD_E_INVALID, "nu, eta, cs must be finite");
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(p->bext[a])) return fail(MHD_E_INVALID, "bext must be finite");
    if (!(p->upwind >= 0) || !std::isfinite(p->upwind)) return fail(MHD_E_INVALID, "upwind must be finite and >= 0");
    return MHD_OK;
}

// ------------------------------------------------------------------ tiles

// Tiles of a run in the order the work-groups should meet them.  The (x, y) columns
// of tiles are grouped into patches of a few times as many columns as one XCD runs
// at once; a patch is walked through z one level at a time.  Tiles running together
// then share their x/y halo lines in L2, and the z halo of one level is still in
// L2 when the next level reads it.  (In plain z-y-x order the z neighbours of a tile
// are thousands of tiles away and every z halo is fetched from HBM again.)
// tir (the partials slot) stays the natural z-y-x index.
// z-segments of a marching run: enough work-groups to fill the chip (one resident per
// CU), each segment a whole number of slabs of at least two slabs
int march_segment(const mhd_params &p, int shape)
{
    const Shape &s = SHAPES[shape];
    if (!s.march) return 0;
    const long ncol = (long)(p.nx / s.tx) * (p.ny / s.ty);
    int nseg = 1;
    while (ncol * nseg < 1024 && p.nz % (2 * nseg * s.tz) == 0 && p.nz / (2 * nseg) >= 2 * s.tz) nseg *= 2;
    return p.nz / nseg;
}

// z-segments of a zm run: the columns times the segments make at least 2048 work-groups
// (eight per CU at one per CU) while a segment keeps at least 64 planes, so that the six
// planes of warm-up per segment cost little
int zm_segment(const mhd_params &p)
{
    const Shape &s = SHAPES[SHAPE_ZM];
    const long ncol = (long)(p.nx / s.tx) * (p.ny / s.ty);
    int nseg = 1;
    while (ncol * nseg < 2048 && p.nz / (2 * nseg) >= 64) nseg *= 2;
    return (p.nz + nseg - 1) / nseg;
}

// z-marching columns of tw x 8 cells in z-segments of zm_segment(p) planes, in patches
// of 32 columns (the work-groups resident on one XCD at a time), so that neighbouring
// columns march side by side and share their x/y halo lines in L2
static void zm_tiles(const mhd_params &p, int tw, int run, std::vector<TileEnt> &out)
{
    const int ty_ = SHAPES[SHAPE_ZM].ty;
    const int ntx = p.nx / tw, nty = p.ny / ty_, seg = zm_segment(p), nseg = (p.nz + seg - 1) / seg;
    int px = 1;
    while (px * 2 <= ntx && px * px * 2 <= 32) px *= 2;
    const int py = std::max(1, std::min(nty, 32 / px));
    for (int sg = 0; sg < nseg; sg++)
        for (int pY = 0; pY < nty; pY += py)
            for (int pX = 0; pX < ntx; pX += px)
                for (int ty = pY; ty < std::min(nty, pY + py); ty++)
                    for (int tx = pX; tx < std::min(ntx, pX + px); tx++) {
                        TileEnt t;
                        t.run = run;
                        t.xy = (tx * tw) | ((ty * ty_) << 16);
                        t.z0 = sg * seg;
                        t.tir = tx + ntx * (ty + nty * sg);
                        out.push_back(t);
                    }
}

void run_tiles_wide(const mhd_params &p, int run, std::vector<TileEnt> &out) { zm_tiles(p, ZM_WIDE_TX, run, out); }

int run_ntiles_wide(const mhd_params &p)
{
    const int seg = zm_segment(p);
    return (p.nx / ZM_WIDE_TX) * (p.ny / SHAPES[SHAPE_ZM].ty) * ((p.nz + seg - 1) / seg);
}

void run_tiles(const mhd_params &p, int shape, int run, std::vector<TileEnt> &out)
{
    const Shape &s = SHAPES[shape];
    if (s.zm) {
        zm_tiles(p, s.tx, run, out);
        return;
    }
    if (s.march) {
        // columns in patches of ~32 (the work-groups resident on one XCD at a time), so
        // that columns marching side by side share their x/y halo lines in L2
        const int ntx = p.nx / s.tx, nty = p.ny / s.ty, seg = march_segment(p, shape), nseg = p.nz / seg;
        int px = 1;
        while (px * 2 <= ntx && px * px * 2 <= 32) px *= 2;
        const int py = std::max(1, std::min(nty, 32 / px));
        for (int pY = 0; pY < nty; pY += py)
            for (int pX = 0; pX < ntx; pX += px)
                for (int sg = 0; sg < nseg; sg++)
                    for (int ty = pY; ty < std::min(nty, pY + py); ty++)
                        for (int tx = pX; tx < std::min(ntx, pX + px); tx++) {
                            TileEnt t;
                            t.run = run;
                            t.xy = (tx * s.tx) | ((ty * s.ty) << 16);
                            t.z0 = sg * seg;
                            t.tir = tx + ntx * (ty + nty * sg);
                            out.push_back(t);
                        }
        return;
    }
    const int ntx = (p.nx + s.tx - 1) / s.tx, nty = (p.ny + s.ty - 1) / s.ty, ntz = (p.nz + s.tz - 1) / s.tz;
    // columns per patch: about twice the work-groups resident on one XCD (32 CUs x 1-2
    // groups).  At 512^3 this ran 0.4 % (FP64) and 1.2 % (FP32) faster than one XCD's
    // worth and 3 % faster than half of it; the patch's aspect ratio mattered less.
    const int target = p.precision == MHD_FP64 ? 64 : 128;
    int px = 1;
    while (px * 2 <= ntx && px * px * 2 <= target) px *= 2;
    int py = std::max(1, std::min(nty, target / px));
    for (int pY = 0; pY < nty; pY += py)
        for (int pX = 0; pX < ntx; pX += px)
            for (int tz = 0; tz < ntz; tz++)
                for (int ty = pY; ty < std::min(nty, pY + py); ty++)
                    for (int tx = pX; tx < std::min(ntx, pX + px); tx++) {
                        TileEnt t;
                        t.run = run;
                        t.xy = (tx * s.tx) | ((ty * s.ty) << 16);
                        t.z0 = tz * s.tz;
                        t.tir = tx + ntx * (ty + nty * tz);
                        out.push_back(t);
                    }
}

// Offset of the ring kernel's tile grid in x.  A halo-box row spans TX + 8 values;
// where it falls on 128-byte lines decides how many lines the row costs, and line
// requests in flight per CU are what bound the staging rate.  Choose, among offsets
// that keep 16-byte vectors aligned, the one that touches the fewest lines over a
// row of tiles (rows assumed to start on a line, as they do when nx * size is a
// multiple of 128).  The staged kernel uses no offset.
int x_shift(const mhd_params &p, int shape)
{
    const Shape &s = SHAPES[shape];
    if (s.zm) {  // the kernel wraps every copy fully: any offset that keeps vectors aligned
        const int es = p.precision, epl = 16 / es, L = 128 / es;
        const int ntx = p.nx / s.tx;
        int best = 0;
        long bestc = -1;
        for (int xs = 0; xs < L; xs += epl) {
            long cnt = 0;
            for (int t = 0; t < ntx; t++) {
                int prev = -1;
                for (int e = t * s.tx + xs - 4; e < t * s.tx + xs + s.tx + 4; e++) {
                    const int line = (((e % p.nx) + p.nx) % p.nx) / L;
                    if (line != prev) cnt++;
                    prev = line;
                }
            }
            if (bestc < 0 || cnt < bestc) {
                bestc = cnt;
                best = xs;
            }
        }
        return best;
    }
    if (!s.pipe || !shape_fits(p, shape)) return 0;
    const int es = p.precision, epl = 16 / es, L = 128 / es;
    const int ntx = (p.nx + s.tx - 1) / s.tx;
    int best = 0;
    long bestc = -1;
    // every box must stay within one period past nx: the kernel wraps indices once
    for (int xs = 0; xs < L && ntx * s.tx + xs + 4 <= 2 * p.nx; xs += epl) {
        long cnt = 0;
        for (int t = 0; t < ntx; t++) {
            int prev = -1;
            for (int e = t * s.tx + xs - 4; e < t * s.tx + xs + s.tx + 4; e++) {
                const int line = (((e % p.nx) + p.nx) % p.nx) / L;
                if (line != prev) cnt++;
                prev = line;
            }
        }
        if (bestc < 0 || cnt < bestc) {
            bestc = cnt;
            best = xs;
        }
    }
    return best;
}

int run_ntiles(const mhd_params &p, int shape)
{
    const Shape &s = SHAPES[shape];
    if (s.zm) {
        const int seg = zm_segment(p);
        return (p.nx / s.tx) * (p.ny / s.ty) * ((p.nz + seg - 1) / seg);
    }
    if (s.march) return (p.nx / s.tx) * (p.ny / s.ty) * (p.nz / march_segment(p, shape));
    return ((p.nx + s.tx - 1) / s.tx) * ((p.ny + s.ty - 1) / s.ty) * ((p.nz + s.tz - 1) / s.tz);
}

// Work-groups are dispatched round-robin over the 8 XCDs (block b -> XCD b mod 8),
// and each XCD has its own L2.  Reorder so that XCD g receives a contiguous run of
// tiles in natural order: neighbouring tiles, which share halo lines, then meet
// in the same L2.
std::vector<TileEnt> xcd_order(const std::vector<TileEnt> &nat)
{
    const size_t T = nat.size();
    const size_t NX = 8;
    std::vector<TileEnt> out(T);
    size_t start = 0;
    for (size_t g = 0; g < NX; g++) {
        const size_t cnt = (T > g) ? (T - g + NX - 1) / NX : 0;  // blocks b < T with b % 8 == g
        for (size_t m = 0; m < cnt; m++) out[NX * m + g] = nat[start + m];
        start += cnt;
    }
    return out;
}

// ------------------------------------------------------------------ launches

template <typename T, int TX, int TY, int TZ, int CZ>
static hipError_t launch_shape(int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles, int step,
                               hipStream_t st)
{
    constexpr int W = 2;  // minimum waves per SIMD: at most 256 VGPRs
    const dim3 grid(ntiles), block(TX * TY * (TZ / CZ));
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 0, true, true, W>), grid, block, 0, st, runs, tiles, step); break;
    case 1: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 1, false, true, W>), grid, block, 0, st, runs, tiles, step); break;
    case 2: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 2, false, true, W>), grid, block, 0, st, runs, tiles, step); break;
    case 4: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 0, true, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
    case 5: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 1, false, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
    case 6: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 2, false, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
    default: hipLaunchKernelGGL((k_substep<T, TX, TY, TZ, CZ, 0, true, false, W>), grid, block, 0, st, runs, tiles, step); break;
    }
    return hipGetLastError();
}

template <typename T, int TX, int TY, int TZ, int CZ, bool FIT>
static hipError_t launch_pipe(int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles, int step,
                              hipStream_t st)
{
    constexpr int W = pipe_waves<T, TX, TY, TZ, CZ>();
    const dim3 grid(ntiles), block(TX * TY * (TZ / CZ));
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 0, true, true, W, FIT>), grid, block, 0, st, runs, tiles, step); break;
    case 1: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 1, false, true, W, FIT>), grid, block, 0, st, runs, tiles, step); break;
    case 2: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 2, false, true, W, FIT>), grid, block, 0, st, runs, tiles, step); break;
    case 4: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 0, true, true, W, FIT, true>), grid, block, 0, st, runs, tiles, step); break;
    case 5: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 1, false, true, W, FIT, true>), grid, block, 0, st, runs, tiles, step); break;
    case 6: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 2, false, true, W, FIT, true>), grid, block, 0, st, runs, tiles, step); break;
    default: hipLaunchKernelGGL((k_pipe<T, TX, TY, TZ, CZ, 0, true, false, W, FIT>), grid, block, 0, st, runs, tiles, step); break;
    }
    return hipGetLastError();
}

template <typename T, int TX, int TY, int TZ, int CZ>
static hipError_t launch_pipe_fit(bool fit, int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles,
                                  int step, hipStream_t st)
{
    return fit ? launch_pipe<T, TX, TY, TZ, CZ, true>(kind, runs, tiles, ntiles, step, st)
               : launch_pipe<T, TX, TY, TZ, CZ, false>(kind, runs, tiles, ntiles, step, st);
}

template <typename T, int TX, int TY, int TZ>
static hipError_t launch_march(int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles, int step,
                               hipStream_t st)
{
    if constexpr (!MarchCfg<T, TX, TY, TZ>::FITS) {
        return hipErrorInvalidValue;
    } else {
        constexpr int NT = TX * TY * TZ;
        constexpr int W = NT >= 512 ? 2 : 1;  // one work-group per CU (LDS)
        const dim3 grid(ntiles), block(NT);
        switch (kind) {
        case 0: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 0, true, true, W>), grid, block, 0, st, runs, tiles, step); break;
        case 1: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 1, false, true, W>), grid, block, 0, st, runs, tiles, step); break;
        case 2: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 2, false, true, W>), grid, block, 0, st, runs, tiles, step); break;
        case 4: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 0, true, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
        case 5: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 1, false, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
        case 6: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 2, false, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
        default: hipLaunchKernelGGL((k_march<T, TX, TY, TZ, 0, true, false, W>), grid, block, 0, st, runs, tiles, step); break;
        }
        return hipGetLastError();
    }
}

// z-marching kernel: FP64 at two waves per SIMD (256 registers, one 160 KB work-group
// per CU), FP32 at four (128 registers, two 80 KB work-groups per CU) except substep 1,
// whose FP64 diagnostics need more registers than that (two waves per SIMD)
template <typename T>
static hipError_t launch_zm(int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles, const TileEnt *wtiles,
                            int nwtiles, int step, hipStream_t st)
{
    constexpr int W = sizeof(T) == 8 ? 2 : 4;
    constexpr int WD = 2;
    if constexpr (sizeof(T) == 4) {
        // substeps 1 and 2 on 64-wide tiles: one 1024-thread work-group per CU (the LDS
        // holds one), whose sixteen waves stay in step at every plane
        if (wtiles && nwtiles > 0 && (kind == 1 || kind == 2 || kind == 5 || kind == 6)) {
            const dim3 grid(nwtiles), block(ZmCfg<T, ZM_WIDE_TX>::NT);
            switch (kind) {
            case 1: hipLaunchKernelGGL((k_zm<T, 1, false, true, 4, false, ZM_WIDE_TX>), grid, block, 0, st, runs, wtiles, step); break;
            case 2: hipLaunchKernelGGL((k_zm<T, 2, false, true, 4, false, ZM_WIDE_TX>), grid, block, 0, st, runs, wtiles, step); break;
            case 5: hipLaunchKernelGGL((k_zm<T, 1, false, true, 4, true, ZM_WIDE_TX>), grid, block, 0, st, runs, wtiles, step); break;
            default: hipLaunchKernelGGL((k_zm<T, 2, false, true, 4, true, ZM_WIDE_TX>), grid, block, 0, st, runs, wtiles, step); break;
            }
            return hipGetLastError();
        }
    }
    const dim3 grid(ntiles), block(ZmCfg<T>::NT);
    switch (kind) {
    case 0: hipLaunchKernelGGL((k_zm<T, 0, true, true, WD>), grid, block, 0, st, runs, tiles, step); break;
    case 1: hipLaunchKernelGGL((k_zm<T, 1, false, true, W>), grid, block, 0, st, runs, tiles, step); break;
    case 2: hipLaunchKernelGGL((k_zm<T, 2, false, true, W>), grid, block, 0, st, runs, tiles, step); break;
    case 4: hipLaunchKernelGGL((k_zm<T, 0, true, true, WD, true>), grid, block, 0, st, runs, tiles, step); break;
    case 5: hipLaunchKernelGGL((k_zm<T, 1, false, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
    case 6: hipLaunchKernelGGL((k_zm<T, 2, false, true, W, true>), grid, block, 0, st, runs, tiles, step); break;
    default: hipLaunchKernelGGL((k_zm<T, 0, true, false, WD>), grid, block, 0, st, runs, tiles, step); break;
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_substep(int shape, bool fit, int kind, const RunDesc<T> *runs, const TileEnt *tiles, int ntiles,
                          const TileEnt *wtiles, int nwtiles, int step, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    if (SHAPES[shape].zm) return launch_zm<T>(kind, runs, tiles, ntiles, wtiles, nwtiles, step, st);
    switch (shape) {
    case 0: return launch_shape<T, 16, 8, 4, 1>(kind, runs, tiles, ntiles, step, st);
    case 1: return launch_shape<T, 32, 8, 4, 1>(kind, runs, tiles, ntiles, step, st);
    case 2: return launch_shape<T, 8, 8, 4, 1>(kind, runs, tiles, ntiles, step, st);
    case 3: return launch_shape<T, 16, 8, 8, 2>(kind, runs, tiles, ntiles, step, st);
    case 4: return launch_shape<T, 32, 4, 4, 1>(kind, runs, tiles, ntiles, step, st);
    case 5: return launch_shape<T, 32, 4, 8, 2>(kind, runs, tiles, ntiles, step, st);
    case 6: return launch_pipe_fit<T, 16, 8, 4, 1>(fit, kind, runs, tiles, ntiles, step, st);
    case 7: return launch_pipe_fit<T, 32, 8, 4, 1>(fit, kind, runs, tiles, ntiles, step, st);
    case 8: return launch_pipe_fit<T, 8, 8, 4, 1>(fit, kind, runs, tiles, ntiles, step, st);
    case 9: return launch_pipe_fit<T, 16, 8, 8, 2>(fit, kind, runs, tiles, ntiles, step, st);
    case 10: return launch_pipe_fit<T, 32, 4, 4, 1>(fit, kind, runs, tiles, ntiles, step, st);
    case 11: return launch_pipe_fit<T, 32, 4, 8, 2>(fit, kind, runs, tiles, ntiles, step, st);
    case 12: return launch_march<T, 16, 8, 4>(kind, runs, tiles, ntiles, step, st);
    default: return launch_march<T, 8, 8, 4>(kind, runs, tiles, ntiles, step, st);
    }
}

int run_nb2(const mhd_params &p, int shape) { return (run_ntiles(p, shape) + FIN_CHUNK - 1) / FIN_CHUNK; }

template <typename T>
hipError_t launch_finalize(const RunDesc<T> *runs, int nruns, int max_nb2, int step, hipStream_t st)
{
    if (nruns <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_finalize1<T>), dim3(nruns, max_nb2), dim3(256), 0, st, runs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_finalize2<T>), dim3(nruns), dim3(64), 0, st, runs, step);
    return hipGetLastError();
}

template hipError_t launch_substep<float>(int, bool, int, const RunDesc<float> *, const TileEnt *, int, const TileEnt *, int,
                                          int, hipStream_t);
template hipError_t launch_substep<double>(int, bool, int, const RunDesc<double> *, const TileEnt *, int, const TileEnt *, int,
                                           int, hipStream_t);
template hipError_t launch_finalize<float>(const RunDesc<float> *, int, int, int, hipStream_t);
template hipError_t launch_finalize<double>(const RunDesc<double> *, int, int, int, hipStream_t);

// ------------------------------------------------------------------ context

size_t ctx_footprint(const mhd_params &p)
{
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    const size_t fb = field_spacing(n, p.precision);
    const int nt = run_ntiles(p, default_shape(p));
    return 14 * fb + (size_t)(nt + run_nb2(p, default_shape(p))) * DIAGW * 8 +
           (size_t)CHUNK * forcing_stride(p) * p.precision +
           (size_t)CHUNK * DREC * 8 + 4096;
}

static_assert(sizeof(RunDesc<double>) <= 1024 && sizeof(RunDesc<float>) <= 1024,
              "run descriptor must fit its 1 KiB device slot");

static mhd_status ctx_alloc_aux(mhd_ctx *c)
{
    const size_t fbytes = (size_t)CHUNK * c->fstride * c->p.precision;
    const size_t rbytes = (size_t)CHUNK * DREC * sizeof(double);
    const size_t pbytes = (size_t)c->ntiles * DIAGW * sizeof(double);
    const size_t p2bytes = (size_t)c->nb2 * DIAGW * sizeof(double);
    const size_t dbytes = 1024;
    const size_t tbytes = (size_t)c->ntiles * sizeof(TileEnt);
    const size_t wbytes = (size_t)c->ntiles_w * sizeof(TileEnt);
    c->aux_bytes = align_up(fbytes, 256) + align_up(rbytes, 256) + align_up(pbytes, 256) + align_up(p2bytes, 256) +
                   align_up(dbytes, 256) + align_up(tbytes, 256) + align_up(wbytes, 256);
    if (hipMalloc(&c->aux, c->aux_bytes) != hipSuccess) return fail(MHD_E_OOM, "device allocation (aux) failed");
    char *b = (char *)c->aux;
    c->d_forcing = b; b += align_up(fbytes, 256);
    c->d_records = (double *)b; b += align_up(rbytes, 256);
    c->d_partials = (double *)b; b += align_up(pbytes, 256);
    c->d_partials2 = (double *)b; b += align_up(p2bytes, 256);
    c->d_desc = b; b += align_up(dbytes, 256);
    c->d_tiles = (TileEnt *)b; b += align_up(tbytes, 256);
    c->d_tiles_w = c->ntiles_w > 0 ? (TileEnt *)b : nullptr;
    c->h_stage_bytes = fbytes + dbytes;
    if (hipHostMalloc(&c->h_stage, c->h_stage_bytes, hipHostMallocDefault) != hipSuccess)
        return fail(MHD_E_OOM, "pinned host allocation failed");
    if (hipEventCreateWithFlags(&c->stage_evt, hipEventDisableTiming) != hipSuccess)
        return fail(MHD_E_DEVICE, "hipEventCreate failed");
    std::vector<TileEnt> nat;
    run_tiles(c->p, c->shape, 0, nat);
    std::vector<TileEnt> ord = xcd_order(nat);
    if (hipMemcpy(c->d_tiles, ord.data(), tbytes, hipMemcpyHostToDevice) != hipSuccess)
        return fail(MHD_E_DEVICE, "tile table upload failed");
    if (c->ntiles_w > 0) {
        nat.clear();
        run_tiles_wide(c->p, 0, nat);
        ord = xcd_order(nat);
        if (hipMemcpy(c->d_tiles_w, ord.data(), wbytes, hipMemcpyHostToDevice) != hipSuccess)
            return fail(MHD_E_DEVICE, "tile table upload failed");
    }
    return MHD_OK;
}

mhd_status ctx_init(mhd_ctx *c, const mhd_params *p, void *stream, void *const *bufs, int shape)
{
    c->p = *p;
    c->ncell = (size_t)p->nx * p->ny * p->nz;
    c->stream = (hipStream_t)stream;
    c->fstride = forcing_stride(*p);
    const size_t fb = field_spacing(c->ncell, p->precision);
    bool aligned = true;
    if (bufs) {
        for (int s = 0; s < 2; s++)
            for (int f = 0; f < NF; f++) {
                c->bufs[s][f] = bufs[s * NF + f];
                if (!c->bufs[s][f]) return fail(MHD_E_INVALID, "borrowed buffer is NULL");
                if ((uintptr_t)c->bufs[s][f] % (uintptr_t)p->precision != 0)
                    return fail(MHD_E_INVALID, "borrowed buffer is not aligned to its value size");
                aligned = aligned && ((uintptr_t)c->bufs[s][f] % 16 == 0);
            }
    } else {
        if (hipMalloc(&c->mem, 14 * fb) != hipSuccess) return fail(MHD_E_OOM, "device allocation of the state failed");
        c->owns = true;
        for (int s = 0; s < 2; s++)
            for (int f = 0; f < NF; f++) c->bufs[s][f] = (char *)c->mem + (size_t)(s * NF + f) * fb;
        if (hipMemsetAsync(c->mem, 0, 14 * fb, c->stream) != hipSuccess)
            return fail(MHD_E_DEVICE, "clearing the state failed");
    }
    // tile shape: the requested one if this grid and these buffers can use it, else the
    // (tuned or default) choice; ring shapes fall back to the staged kernel of the same box
    if (shape >= 0)
        while (!shape_eligible(*p, shape, aligned)) shape = shape_fallback(shape);
    c->shape = shape >= 0 ? shape : default_shape(*p, aligned);
    c->fit = SHAPES[c->shape].pipe && shape_fits(*p, c->shape);
    c->xs = x_shift(*p, c->shape);
    c->seg = SHAPES[c->shape].zm ? zm_segment(*p) : march_segment(*p, c->shape);
    c->ntiles = run_ntiles(*p, c->shape);
    c->ntiles_w = SHAPES[c->shape].wide ? run_ntiles_wide(*p) : 0;
    c->nb2 = run_nb2(*p, c->shape);
    {
        int dev = 0, khz = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            c->clock_hz = 1e3 * (double)khz;
    }
    mhd_status st = ctx_alloc_aux(c);
    if (st != MHD_OK) return st;
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(MHD_E_DEVICE, "stream sync failed");
    return MHD_OK;
}

void ctx_release(mhd_ctx *c)
{
    if (c->stream || true) hipStreamSynchronize(c->stream);
    if (c->owns && c->mem) hipFree(c->mem);
    if (c->aux) hipFree(c->aux);
    if (c->spec_ws) hipFree(c->spec_ws);
    c->spec_ws = nullptr;
    c->spec_bytes = 0;
    if (c->h_stage) hipHostFree(c->h_stage);
    if (c->stage_evt) hipEventDestroy(c->stage_evt);
    c->mem = c->aux = c->h_stage = nullptr;
    c->stage_evt = nullptr;
}

// Forcing record of the context's global step n.
mhd_status ctx_forcing_at(mhd_ctx *c, int64_t n, mhd_forcing &f)
{
    if (c->fmode == 0) {
        std::memset(&f, 0, sizeof f);
        f.k[0] = 1;
        f.e[1] = 1.0;
        return MHD_OK;
    }
    if (c->fmode == 2) {
        f = random_forcing(c->kf, c->f0, c->sigma, c->fseed, n);
        return MHD_OK;
    }
    const int64_t i = n - c->sched_start;
    if (i < 0 || i >= (int64_t)c->sched.size())
        return fail(MHD_E_INVALID, "step " + std::to_string(n) + " is outside the forcing schedule");
    f = c->sched[(size_t)i];
    return MHD_OK;
}

template <typename T>
void fill_desc(const mhd_ctx *c, RunDesc<T> &d, int parity0, int64_t step0, const T *forcing, double *records,
               double *partials, int first_tile)
{
    std::memset(&d, 0, sizeof d);
    for (int s = 0; s < 2; s++)
        for (int f = 0; f < NF; f++) d.buf[s][f] = (T *)c->bufs[s][f];
    d.nx = c->p.nx;
    d.ny = c->p.ny;
    d.nz = c->p.nz;
    d.parity0 = parity0;
    d.first_tile = first_tile;
    d.ntiles = c->ntiles;
    d.fstride = c->fstride;
    d.xs = c->xs;
    d.seg = c->seg;
    fill_coef<T>(c->p, d.c, d.dc);
    d.forcing = forcing;
    d.partials = partials;
    d.partials2 = c->d_partials2;
    d.nb2 = c->nb2;
    d.records = records;
    d.step0 = (double)step0;
    d.dt = c->p.dt;
}
template void fill_desc<float>(const mhd_ctx *, RunDesc<float> &, int, int64_t, const float *, double *, double *, int);
template void fill_desc<double>(const mhd_ctx *, RunDesc<double> &, int, int64_t, const double *, double *, double *, int);

// Write the forcing blocks of steps [n0, n0+m) into host memory dst.
mhd_status ctx_forcing_blocks(mhd_ctx *c, int64_t n0, int64_t m, void *dst)
{
    const int n[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (int a = 0; a < 3; a++)
        if (c->unit[a].size() != 2 * (size_t)n[a]) c->unit[a] = unit_circle(n[a]);
    for (int64_t s = 0; s < m; s++) {
        mhd_forcing f;
        mhd_status st = ctx_forcing_at(c, n0 + s, f);
        if (st != MHD_OK) return st;
        st = check_forcing(f);
        if (st != MHD_OK) return st;
        if (c->p.precision == MHD_FP64)
            forcing_block<double>(c->p, f, (double *)dst + (size_t)s * c->fstride, c->unit);
        else
            forcing_block<float>(c->p, f, (float *)dst + (size_t)s * c->fstride, c->unit);
    }
    return MHD_OK;
}

// Move device records into the host list (synchronises the stream).
mhd_status ctx_drain(mhd_ctx *c)
{
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(MHD_E_DEVICE, "device error while stepping");
    if (c->rcount == 0) return MHD_OK;
    std::vector<double> tmp((size_t)c->rcount * DREC);
    if (hipMemcpy(tmp.data(), c->d_records, tmp.size() * sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
        return fail(MHD_E_DEVICE, "copying diagnostics failed");
    for (int64_t i = 0; i < c->rcount; i++) {
        const double *r = &tmp[(size_t)i * DREC];
        mhd_diag d;
        d.step = (int64_t)r[0];
        d.t = r[1];
        d.em = r[2];
        d.ek = r[3];
        d.urms = r[4];
        d.brms = r[5];
        d.umax = r[6];
        d.lnrho_mean = r[7];
        d.b_mean[0] = r[8];
        d.b_mean[1] = r[9];
        d.b_mean[2] = r[10];
        d.nonfinite = (int64_t)r[11];  /* an exact count, carried as a double on the device */
        d.t_device = r[12] / c->clock_hz;
        c->host_diag.push_back(d);
    }
    c->rcount = 0;
    return MHD_OK;
}

// Stage (forcing blocks, descriptor) through pinned memory and enqueue the upload.
template <typename T>
static mhd_status ctx_stage(mhd_ctx *c, int64_t m, bool diag_only)
{
    if (hipEventSynchronize(c->stage_evt) != hipSuccess) return fail(MHD_E_DEVICE, "staging event failed");
    char *h = (char *)c->h_stage;
    const size_t fbytes = (size_t)m * c->fstride * sizeof(T);
    if (!diag_only) {
        mhd_status st = ctx_forcing_blocks(c, c->step, m, h);
        if (st != MHD_OK) return st;
    }
    RunDesc<T> d;
    fill_desc<T>(c, d, c->parity, c->step, (const T *)c->d_forcing, c->d_records + (size_t)c->rcount * DREC,
                 c->d_partials, 0);
    char *hd = h + (size_t)CHUNK * c->fstride * sizeof(T);
    std::memcpy(hd, &d, sizeof d);
    if (!diag_only && fbytes)
        if (hipMemcpyAsync(c->d_forcing, h, fbytes, hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return fail(MHD_E_DEVICE, "forcing upload failed");
    if (hipMemcpyAsync(c->d_desc, hd, sizeof d, hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return fail(MHD_E_DEVICE, "descriptor upload failed");
    if (hipEventRecord(c->stage_evt, c->stream) != hipSuccess) return fail(MHD_E_DEVICE, "event record failed");
    return MHD_OK;
}

// launch kinds 0-2 are the three substeps, 4-6 the same with upwinding
static int upwind_kind(const mhd_params &p) { return p.upwind != 0.0 ? 4 : 0; }

template <typename T>
static mhd_status ctx_step_t(mhd_ctx *c, int64_t nsteps)
{
    const int upk = upwind_kind(c->p);
    while (nsteps > 0) {
        const int64_t m = std::min<int64_t>(nsteps, CHUNK);
        if (c->rcount + m > CHUNK) {
            mhd_status st = ctx_drain(c);
            if (st != MHD_OK) return st;
        }
        mhd_status st = ctx_stage<T>(c, m, false);
        if (st != MHD_OK) return st;
        const RunDesc<T> *d = (const RunDesc<T> *)c->d_desc;
        for (int64_t s = 0; s < m; s++) {
            hipError_t e = launch_substep<T>(c->shape, c->fit, 0 + upk, d, c->d_tiles, c->ntiles, c->d_tiles_w, c->ntiles_w, (int)s, c->stream);
            if (e == hipSuccess) e = launch_finalize<T>(d, 1, c->nb2, (int)s, c->stream);
            if (e == hipSuccess) e = launch_substep<T>(c->shape, c->fit, 1 + upk, d, c->d_tiles, c->ntiles, c->d_tiles_w, c->ntiles_w, (int)s, c->stream);
            if (e == hipSuccess) e = launch_substep<T>(c->shape, c->fit, 2 + upk, d, c->d_tiles, c->ntiles, c->d_tiles_w, c->ntiles_w, (int)s, c->stream);
            if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
        }
        c->rcount += m;
        c->parity ^= (int)(m & 1);
        c->step += m;
        nsteps -= m;
    }
    return MHD_OK;
}

// Same as ctx_step_t, with events around each launch (timing for the roofline).
template <typename T>
static mhd_status ctx_step_timed_t(mhd_ctx *c, int64_t nsteps, double kms[4], double *step_ms)
{
    std::vector<hipEvent_t> ev;
    auto fail_ev = [&](const std::string &m) {
        for (auto e : ev) (void)hipEventDestroy(e);
        return fail(MHD_E_DEVICE, m);
    };
    double acc[4] = {0, 0, 0, 0};
    int64_t done = 0;
    const int upk = upwind_kind(c->p);
    while (nsteps > 0) {
        const int64_t m = std::min<int64_t>(nsteps, CHUNK);
        if (c->rcount + m > CHUNK) {
            mhd_status st = ctx_drain(c);
            if (st != MHD_OK) return st;
        }
        mhd_status st = ctx_stage<T>(c, m, false);
        if (st != MHD_OK) return st;
        for (auto e : ev) (void)hipEventDestroy(e);
        ev.assign((size_t)(5 * m), nullptr);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess) return fail_ev("hipEventCreate failed");
        const RunDesc<T> *d = (const RunDesc<T> *)c->d_desc;
        for (int64_t s = 0; s < m; s++) {
            hipEvent_t *E = &ev[(size_t)(5 * s)];
            hipError_t e = hipEventRecord(E[0], c->stream);
            if (e == hipSuccess) e = launch_substep<T>(c->shape, c->fit, 0 + upk, d, c->d_tiles, c->ntiles, c->d_tiles_w, c->ntiles_w, (int)s, c->stream);
            if (e == hipSuccess) e = hipEventRecord(E[1], c->stream);
            if (e == hipSuccess) e = launch_finalize<T>(d, 1, c->nb2, (int)s, c->stream);
            if (e == hipSuccess) e = hipEventRecord(E[2], c->stream);
            if (e == hipSuccess) e = launch_substep<T>(c->shape, c->fit, 1 + upk, d, c->d_tiles, c->ntiles, c->d_tiles_w, c->ntiles_w, (int)s, c->stream);
            if (e == hipSuccess) e = hipEventRecord(E[3], c->stream);
            if (e == hipSuccess) e = launch_substep<T>(c->shape, c->fit, 2 + upk, d, c->d_tiles, c->ntiles, c->d_tiles_w, c->ntiles_w, (int)s, c->stream);
            if (e == hipSuccess) e = hipEventRecord(E[4], c->stream);
            if (e != hipSuccess) return fail_ev(std::string("launch failed: ") + hipGetErrorString(e));
        }
        if (hipStreamSynchronize(c->stream) != hipSuccess) return fail_ev("device error while stepping");
        for (int64_t s = 0; s < m; s++) {
            hipEvent_t *E = &ev[(size_t)(5 * s)];
            float t01, t12, t23, t34;
            if (hipEventElapsedTime(&t01, E[0], E[1]) != hipSuccess || hipEventElapsedTime(&t12, E[1], E[2]) != hipSuccess ||
                hipEventElapsedTime(&t23, E[2], E[3]) != hipSuccess || hipEventElapsedTime(&t34, E[3], E[4]) != hipSuccess)
                return fail_ev("hipEventElapsedTime failed");
            acc[0] += t01;
            acc[3] += t12;
            acc[1] += t23;
            acc[2] += t34;
            if (step_ms) step_ms[done + s] = (double)t01 + t12 + t23 + t34;
        }
        c->rcount += m;
        c->parity ^= (int)(m & 1);
        c->step += m;
        nsteps -= m;
        done += m;
    }
    for (auto e : ev) (void)hipEventDestroy(e);
    for (int i = 0; i < 4; i++) kms[i] = done ? acc[i] / (double)done : 0.0;
    return MHD_OK;
}

template <typename T>
static mhd_status ctx_reduce_t(mhd_ctx *c)
{
    if (c->rcount + 1 > CHUNK) {
        mhd_status st = ctx_drain(c);
        if (st != MHD_OK) return st;
    }
    mhd_status st = ctx_stage<T>(c, 0, true);
    if (st != MHD_OK) return st;
    const RunDesc<T> *d = (const RunDesc<T> *)c->d_desc;
    hipError_t e = launch_substep<T>(c->shape, c->fit, 3, d, c->d_tiles, c->ntiles, nullptr, 0, 0, c->stream);
    if (e == hipSuccess) e = launch_finalize<T>(d, 1, c->nb2, 0, c->stream);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("kernel launch failed: ") + hipGetErrorString(e));
    c->rcount += 1;
    return MHD_OK;
}

mhd_status ctx_step(mhd_ctx *c, int64_t n)
{
    return c->p.precision == MHD_FP64 ? ctx_step_t<double>(c, n) : ctx_step_t<float>(c, n);
}

// ln rho = 0, u = 0, A = the seed field of (seed, amp), into the current buffer set,
// generated on the device in the context's stream (ordered before its next step).
template <typename T>
static mhd_status ctx_init_seed_t(mhd_ctx *c, uint64_t seed, double amp)
{
    SeedArgs<T> a;
    for (int f = 0; f < NF; f++) a.f[f] = (T *)c->bufs[c->parity][f];
    for (int k = 0; k < 3; k++) a.key[k] = sm_key(seed, 104 + k);
    a.amp = amp;
    a.n = c->ncell;
    const uint64_t npair = (a.n + 1) / 2;
    const unsigned grid = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>((npair + 255) / 256, 4096));
    hipLaunchKernelGGL(k_seed<T>, dim3(grid), dim3(256), 0, c->stream, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("seed kernel launch failed: ") + hipGetErrorString(e));
    return MHD_OK;
}

mhd_status ctx_init_seed(mhd_ctx *c, uint64_t seed, double amp)
{
    return c->p.precision == MHD_FP64 ? ctx_init_seed_t<double>(c, seed, amp) : ctx_init_seed_t<float>(c, seed, amp);
}

}  // namespace mhd

using namespace mhd;

// ====================================================================== C ABI

extern "C" {

const char *mhd_last_error(void) { return g_err.c_str(); }

static mhd_status create_common(const mhd_params *p, void *const *bufs, void *stream, mhd_ctx **out)
{
    if (!out) return fail(MHD_E_INVALID, "out is NULL");
    *out = nullptr;
    mhd_status st = check_params(p);
    if (st != MHD_OK) return st;
    mhd_ctx *c = new (std::nothrow) mhd_ctx();
    if (!c) return fail(MHD_E_OOM, "host allocation failed");
    st = ctx_init(c, p, stream, bufs, -1);
    if (st != MHD_OK) {
        ctx_release(c);
        delete c;
        return st;
    }
    *out = c;
    return MHD_OK;
}

mhd_status mhd_create(const mhd_params *p, void *hip_stream, mhd_ctx **out)
{
    return create_common(p, nullptr, hip_stream, out);
}

mhd_status mhd_create_borrowed(const mhd_params *p, void *const bufs[14], void *hip_stream, mhd_ctx **out)
{
    if (!bufs) return fail(MHD_E_INVALID, "bufs is NULL");
    return create_common(p, bufs, hip_stream, out);
}

mhd_status mhd_destroy(mhd_ctx *c)
{
    if (!c) return MHD_OK;
    if (c->in_batch) return fail(MHD_E_INVALID, "context belongs to a batch");
    ctx_release(c);
    delete c;
    return MHD_OK;
}

mhd_status mhd_set_field(mhd_ctx *c, int field, const void *src, int on_device)
{
    if (!c || !src) return fail(MHD_E_INVALID, "NULL argument");
    if (field < 0 || field >= NF) return fail(MHD_E_INVALID, "field index out of range");
    const size_t bytes = c->ncell * c->p.precision;
    hipError_t e = hipMemcpyAsync(c->bufs[c->parity][field], src, bytes,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("set_field: ") + hipGetErrorString(e));
    return MHD_OK;
}

mhd_status mhd_get_field(mhd_ctx *c, int field, void *dst, int on_device)
{
    if (!c || !dst) return fail(MHD_E_INVALID, "NULL argument");
    if (field < 0 || field >= NF) return fail(MHD_E_INVALID, "field index out of range");
    const size_t bytes = c->ncell * c->p.precision;
    hipError_t e = hipMemcpyAsync(dst, c->bufs[c->parity][field], bytes,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess && !on_device) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("get_field: ") + hipGetErrorString(e));
    return MHD_OK;
}

mhd_status mhd_field_ptr(mhd_ctx *c, int field, void **dptr)
{
    if (!c || !dptr) return fail(MHD_E_INVALID, "NULL argument");
    if (field < 0 || field >= NF) return fail(MHD_E_INVALID, "field index out of range");
    *dptr = c->bufs[c->parity][field];
    return MHD_OK;
}

mhd_status mhd_init_seed(mhd_ctx *c, uint64_t seed, double a_noise)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (!std::isfinite(a_noise)) return fail(MHD_E_INVALID, "a_noise must be finite");
    return ctx_init_seed(c, seed, a_noise);
}

mhd_status mhd_set_forcing(mhd_ctx *c, const mhd_forcing *recs, int64_t n)
{
    if (!c || (!recs && n > 0) || n < 0) return fail(MHD_E_INVALID, "bad forcing schedule arguments");
    for (int64_t i = 0; i < n; i++) {
        mhd_status st = check_forcing(recs[i]);
        if (st != MHD_OK) return fail(st, "record " + std::to_string(i) + ": " + g_err);
    }
    c->sched.assign(recs, recs + n);
    c->sched_start = c->step;
    c->fmode = 1;
    return MHD_OK;
}

mhd_status mhd_set_forcing_random(mhd_ctx *c, double kf, double f0, double sigma, uint64_t seed)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (!(kf >= 1.0) || !std::isfinite(kf)) return fail(MHD_E_INVALID, "kf must be >= 1");
    if (!std::isfinite(f0) || !std::isfinite(sigma)) return fail(MHD_E_INVALID, "f0 and sigma must be finite");
    c->fmode = 2;
    c->kf = kf;
    c->f0 = f0;
    c->sigma = sigma;
    c->fseed = seed;
    return MHD_OK;
}

mhd_status mhd_clear_forcing(mhd_ctx *c)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    c->fmode = 0;
    c->sched.clear();
    return MHD_OK;
}

mhd_status mhd_step(mhd_ctx *c, int64_t nsteps)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (c->in_batch) return fail(MHD_E_INVALID, "context belongs to a batch: use mhd_batch_run");
    if (nsteps < 0) return fail(MHD_E_INVALID, "nsteps < 0");
    return ctx_step(c, nsteps);
}

mhd_status mhd_step_timed(mhd_ctx *c, int64_t nsteps, double kernel_ms[4], double *step_ms)
{
    if (!c || !kernel_ms) return fail(MHD_E_INVALID, "NULL argument");
    if (c->in_batch) return fail(MHD_E_INVALID, "context belongs to a batch: use mhd_batch_run");
    if (nsteps < 0) return fail(MHD_E_INVALID, "nsteps < 0");
    return c->p.precision == MHD_FP64 ? ctx_step_timed_t<double>(c, nsteps, kernel_ms, step_ms)
                                      : ctx_step_timed_t<float>(c, nsteps, kernel_ms, step_ms);
}

mhd_status mhd_reduce(mhd_ctx *c)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    return c->p.precision == MHD_FP64 ? ctx_reduce_t<double>(c) : ctx_reduce_t<float>(c);
}

mhd_status mhd_get_diag(mhd_ctx *c, mhd_diag *out, int64_t cap, int64_t *n_out)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    mhd_status st = ctx_drain(c);
    if (st != MHD_OK) return st;
    const int64_t n = (int64_t)c->host_diag.size();
    if (n_out) *n_out = n;
    if (out && cap > 0) std::memcpy(out, c->host_diag.data(), (size_t)std::min(n, cap) * sizeof(mhd_diag));
    return MHD_OK;
}

mhd_status mhd_clear_diag(mhd_ctx *c)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    mhd_status st = ctx_drain(c);
    if (st != MHD_OK) return st;
    c->host_diag.clear();
    return MHD_OK;
}

mhd_status mhd_get_time(mhd_ctx *c, int64_t *step, double *t)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (step) *step = c->step;
    if (t) *t = (double)c->step * c->p.dt;
    return MHD_OK;
}

mhd_status mhd_sync(mhd_ctx *c)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return fail(MHD_E_DEVICE, std::string("device error: ") + hipGetErrorString(e));
    return MHD_OK;
}

mhd_status mhd_growth_rate(const mhd_diag *d, int64_t n, int64_t i0, int64_t i1, double *lambda)
{
    if (!d || !lambda) return fail(MHD_E_INVALID, "NULL argument");
    if (i0 < 0 || i1 > n || i1 - i0 < 2) return fail(MHD_E_INVALID, "need 0 <= i0, i1 <= n, i1 - i0 >= 2");
    double tm = 0.0, ym = 0.0;
    for (int64_t i = i0; i < i1; i++) {
        if (!(d[i].brms > 0.0)) return fail(MHD_E_INVALID, "brms must be > 0 for the fit");
        tm += d[i].t;
        ym += std::log(d[i].brms);
    }
    tm /= (double)(i1 - i0);
    ym /= (double)(i1 - i0);
    double sxy = 0.0, sxx = 0.0;
    for (int64_t i = i0; i < i1; i++) {
        const double x = d[i].t - tm;
        sxy += x * (std::log(d[i].brms) - ym);
        sxx += x * x;
    }
    if (!(sxx > 0.0)) return fail(MHD_E_INVALID, "all records at the same time");
    *lambda = sxy / sxx;
    return MHD_OK;
}

static void shape_name(int shape, char *buf, size_t len)
{
    const Shape &s = SHAPES[shape];
    if (s.zm)
        std::snprintf(buf, len, "%dx%d+zm", s.wide ? ZM_WIDE_TX : s.tx, s.ty);
    else
        std::snprintf(buf, len, "%dx%dx%d/%d%s", s.tx, s.ty, s.tz, s.cz, s.march ? "+march" : (s.pipe ? "+ring" : ""));
}

mhd_status mhd_tile_config(const mhd_params *p, char *buf, size_t len)
{
    mhd_status st = check_params(p);
    if (st != MHD_OK) return st;
    if (!buf || len == 0) return fail(MHD_E_INVALID, "buffer is NULL");
    shape_name(default_shape(*p), buf, len);
    return MHD_OK;
}

mhd_status mhd_ctx_tile_config(const mhd_ctx *c, char *buf, size_t len)
{
    if (!c) return fail(MHD_E_INVALID, "ctx is NULL");
    if (!buf || len == 0) return fail(MHD_E_INVALID, "buffer is NULL");
    shape_name(c->shape, buf, len);
    return MHD_OK;
}

mhd_status mhd_forcing_draw(double kf, double f0, double sigma, uint64_t seed, int64_t n, mhd_forcing *out)
{
    if (!out || n < 0) return fail(MHD_E_INVALID, "bad arguments");
    if (!(kf >= 1.0) || !std::isfinite(kf)) return fail(MHD_E_INVALID, "kf must be >= 1");
    *out = random_forcing(kf, f0, sigma, seed, n);
    return MHD_OK;
}

int32_t mhd_num_tile_shapes(void) { return NSHAPES; }

mhd_status mhd_tile_shape_name(int32_t i, char *buf, size_t len)
{
    if (i < 0 || i >= NSHAPES || !buf || len == 0) return fail(MHD_E_INVALID, "bad tile shape index or buffer");
    shape_name(i, buf, len);
    return MHD_OK;
}

mhd_status mhd_set_tile_shape(const mhd_params *p, int32_t i)
{
    mhd_status st = check_params(p);
    if (st != MHD_OK) return st;
    if (i < -1 || i >= NSHAPES) return fail(MHD_E_INVALID, "tile shape index out of range");
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto key = std::make_tuple(p->nx, p->ny, p->nz, p->precision);
    if (i < 0) g_tuned.erase(key);
    else g_tuned[key] = i;
    return MHD_OK;
}

mhd_status mhd_autotune(const mhd_params *p, int reps, void *hip_stream, double *best_ms)
{
    mhd_status st = check_params(p);
    if (st != MHD_OK) return st;
    if (reps < 1) return fail(MHD_E_INVALID, "reps must be >= 1");
    hipStream_t s = (hipStream_t)hip_stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(MHD_E_DEVICE, "hipEventCreate failed");
    int best = -1;
    double bt = 1e300;
    for (int sh = 0; sh < NSHAPES; sh++) {
        if (!shape_eligible(*p, sh, true)) continue;
        mhd_ctx *c = new mhd_ctx();
        st = ctx_init(c, p, hip_stream, nullptr, sh);
        if (st == MHD_OK) st = ctx_step(c, 1);  // warm-up
        if (st == MHD_OK && hipEventRecord(e0, s) != hipSuccess) st = fail(MHD_E_DEVICE, "event record failed");
        if (st == MHD_OK) st = ctx_step(c, reps);
        if (st == MHD_OK && hipEventRecord(e1, s) != hipSuccess) st = fail(MHD_E_DEVICE, "event record failed");
        float ms = 0.f;
        if (st == MHD_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
            st = fail(MHD_E_DEVICE, "timing failed");
        ctx_release(c);
        delete c;
        if (st != MHD_OK) break;
        const double per = ms / reps;
        if (per < bt) {
            bt = per;
            best = sh;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != MHD_OK) return st;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple(p->nx, p->ny, p->nz, p->precision)] = best;
    }
    if (best_ms) *best_ms = bt;
    return MHD_OK;
}

}  // extern "C"
