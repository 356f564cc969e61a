// Device-side data structures and kernels of the MHD solver (gfx950).
//
// One launch = one RK3 substep of every run in a tile list.  Each work-group owns a
// TX x TY x TZ box of cells of one run (or, in the marching kernel, a TX x TY column
// of one z-segment).  The seven fields pass through LDS one at a time (box + 3-cell
// halo, periodic indices wrapped while staging), the next fields streaming in while
// the current one is differentiated: through registers in k_substep, by direct-to-
// LDS loads into a ring of three boxes in k_pipe, into per-field plane rings in
// k_march.  Every right-hand-side term is folded into per-cell accumulators as soon
// as the fields it needs have passed, so registers hold ~23 values per cell instead
// of ~60 derivatives.  The RK3 update is fused: the output of substep s overwrites,
// cell by cell, the buffer holding substep s-2.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mhd {

// Pointers that the kernels dereference are cast to the global address space, so
// loads and stores are global_* (vector-memory counter only) instead of flat_*
// (which also occupy the LDS counter and serialise against LDS reads).
template <typename T>
using G = __attribute__((address_space(1))) T;

constexpr int NF = 7;
constexpr int DIAGW = 10;  // per-tile partials: |B|^2, |u|^2, rho|u|^2, lnrho, Bx, By, Bz, max|u|^2, nonfinite, spare
constexpr int DREC = 13;   // record: step, t, em, ek, urms, brms, umax, <lnrho>, <Bx>, <By>, <Bz>, nonfinite,
                           // device wall clock (ticks) when the record was written
constexpr int FHEAD = 8;   // forcing block head: a[3], b[3], on, spare

// Forcing phase tables hold (cos, sin) of one index in a 16-byte slot (FP32 pads
// with two zeros), so that the ring kernel can copy them with 16-byte vectors.
template <typename T>
constexpr int FSLOT = 16 / (int)sizeof(T);

// Sixth-order central weights (exact for polynomials of degree 6 / 7): first
// derivative, offsets 1..3; second derivative, offsets 0..3.  The kernels take
// them as compile-time constants (materialised by scalar moves, never loaded) and
// scale each derivative by the run's inverse spacing.
constexpr double W1_1 = 3.0 / 4.0, W1_2 = -3.0 / 20.0, W1_3 = 1.0 / 60.0;
constexpr double W2_0 = -49.0 / 18.0, W2_1 = 3.0 / 2.0, W2_2 = -3.0 / 20.0, W2_3 = 1.0 / 90.0;

template <typename T>
struct Coef {
    T ih1[3];     // 1 / h_axis
    T ih2[3];     // 1 / h_axis^2
    T ihm[3];     // 1 / (4 h_a h_b), pair 0 = xy, 1 = xz, 2 = yz
    T cs2, nu, nu3, nu2_3, eta;
    T bext[3];
    T bdt[3];     // beta_s * dt
    T brho[3];    // beta_s * alpha_s / beta_{s-1} (0 for s = 0)
    T upw[3];     // upwinding of the continuity advection: c / (60 h_axis)
    // the same stencil weights scaled by the inverse spacings, x and y (z-marching kernel)
    T w1[2][3];   // W1_s / h_axis, s = 1..3
    T w2[2][4];   // W2_s / h_axis^2, s = 0..3
    // per thread role of that kernel (0: ln rho and u, whose mixed derivatives enter
    // the viscous term with nu / 3; 1: A, whose enter the current density as they are)
    T wm[2][3];     // diagonal x-y derivative: W2_s / (4 h_x h_y), s = 1..3
    T wq[2][2][3];  // diagonal x-z, y-z derivatives: W2_s / (4 h_a h_z), a = x, y
};

struct DCoef {      // FP64 inverse spacings and mean field, for the diagnostics
    double ih1[3];
    double bext[3];
};

// The coefficients that the passes use, read once per work-group and held in scalar
// registers for the whole kernel.  Without the pin the compiler re-reads them from
// memory inside every pass, and each such scalar read must be waited for with the
// counter that also tracks the pass's LDS reads, which serialises the pass.
template <typename T>
struct KRegs {
    T ih1[3], ih2[3], ihm[3];
    T cs2, nu, nu3, nu2_3, eta;

    __device__ __forceinline__ void load(const Coef<T> &c)
    {
#pragma unroll
        for (int a = 0; a < 3; a++) { ih1[a] = c.ih1[a]; ih2[a] = c.ih2[a]; ihm[a] = c.ihm[a]; }
        cs2 = c.cs2; nu = c.nu; nu3 = c.nu3; nu2_3 = c.nu2_3; eta = c.eta;
#pragma unroll
        for (int a = 0; a < 3; a++) asm volatile("" : "+s"(ih1[a]), "+s"(ih2[a]), "+s"(ihm[a]));
        asm volatile("" : "+s"(cs2), "+s"(nu), "+s"(nu3), "+s"(nu2_3), "+s"(eta));
    }
};

// with the upwinding coefficients (kernels instantiated with upwinding only)
template <typename T>
struct KRegsU : KRegs<T> {
    T upw[3];

    __device__ __forceinline__ void load(const Coef<T> &c)
    {
        KRegs<T>::load(c);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            upw[a] = c.upw[a];
            asm volatile("" : "+s"(upw[a]));
        }
    }
};

template <typename T, bool UPW>
using KRegsFor = typename std::conditional<UPW, KRegsU<T>, KRegs<T>>::type;

template <typename T>
struct RunDesc {
    T *buf[2][NF];
    int nx, ny, nz, parity0;
    int first_tile, ntiles, fstride, xs;  // xs: x offset of the tile grid (ring kernel only)
    Coef<T> c;
    DCoef dc;
    const T *forcing;   // per batch step: FHEAD values then Ex, Ey, Ez (FSLOT values per index)
    double *partials;   // [ntiles][DIAGW]
    double *partials2;  // [nb2][DIAGW]: second level of the diagnostic reduction
    int nb2;            // blocks of the first finalize level (FIN_CHUNK partials each)
    int seg;            // z-marching kernel: planes per z-segment of a column
    double *records;    // [batch step][DREC]
    double step0;       // global step index of batch step 0
    double dt;
};

struct TileEnt {
    int run;
    int xy;    // x0 | (y0 << 16)
    int z0;
    int tir;   // tile index within its run (partials slot)
};

template <typename T>
__device__ __forceinline__ T sd1(const T *s, int st, T ih)
{
    return ih * (T(W1_1) * (s[st] - s[-st]) + T(W1_2) * (s[2 * st] - s[-2 * st]) + T(W1_3) * (s[3 * st] - s[-3 * st]));
}

template <typename T>
__device__ __forceinline__ T sd2(const T *s, int st, T ih2)
{
    return ih2 * (T(W2_0) * s[0] + T(W2_1) * (s[st] + s[-st]) + T(W2_2) * (s[2 * st] + s[-2 * st]) +
                  T(W2_3) * (s[3 * st] + s[-3 * st]));
}

// seven-point sixth difference (h^6 times the sixth derivative, to leading order)
template <typename T>
__device__ __forceinline__ T sd6(const T *s, int st)
{
    return T(-20) * s[0] + T(15) * (s[st] + s[-st]) + T(-6) * (s[2 * st] + s[-2 * st]) + (s[3 * st] + s[-3 * st]);
}

// d_a d_b from the (a+b) and (a-b) diagonals
template <typename T>
__device__ __forceinline__ T sdm(const T *s, int sa, int sb, T ihm)
{
    const int p = sa + sb, q = sa - sb;
    return ihm * (T(W2_1) * ((s[p] + s[-p]) - (s[q] + s[-q])) +
                  T(W2_2) * ((s[2 * p] + s[-2 * p]) - (s[2 * q] + s[-2 * q])) +
                  T(W2_3) * ((s[3 * p] + s[-3 * p]) - (s[3 * q] + s[-3 * q])));
}

// first derivative of FP32 values evaluated in FP64
__device__ __forceinline__ double sd1d(const float *s, int st, double ih)
{
    return ih * (W1_1 * ((double)s[st] - (double)s[-st]) + W1_2 * ((double)s[2 * st] - (double)s[-2 * st]) +
                 W1_3 * ((double)s[3 * st] - (double)s[-3 * st]));
}

__device__ __forceinline__ bool finite_v(float v) { return __builtin_isfinite(v); }
__device__ __forceinline__ bool finite_v(double v) { return __builtin_isfinite(v); }

__device__ __forceinline__ int wrapi(int v, int n)
{
    int r = v % n;
    return r < 0 ? r + n : r;
}

// Per-cell accumulators of one thread (CZ cells along z).
template <typename T, int CZ>
struct Cells {
    T v[CZ][NF];        // centre values
    T g[CZ][3];         // grad ln rho
    T B[CZ][3], J[CZ][3];
    T R[CZ][NF];        // right-hand side accumulators
    double Bd[CZ][3];   // FP64 curl, for the diagnostics
    T old[CZ][NF];      // state of substep s-2 at the cells (filled early by the ring kernel)
    T pend[CZ][3];      // u-first order: d_y u_x, d_z u_x, d_z u_y until u_y / u_z are known
    T up6[CZ][3];       // upwinding, u-first order: sixth differences of ln rho until u is known
    bool have_old = false;
};

template <int A, int SY, int SZ>
struct Stride {
    static constexpr int v = A == 0 ? 1 : (A == 1 ? SY : SZ);
};

// index of the mixed pair {a, b}: xy -> 0, xz -> 1, yz -> 2
template <int A, int B>
struct Pair {
    static constexpr int v = (A + B == 1) ? 0 : ((A + B == 2) ? 1 : 2);
};

// Pin the accumulators in registers at this point of the program.  Without it the
// optimiser sinks each pass's arithmetic to the final update and keeps the raw LDS
// reads of every pass alive (and spilled) until then.
template <typename T, int CZ>
__device__ __forceinline__ void pin(Cells<T, CZ> &C)
{
#pragma unroll
    for (int c = 0; c < CZ; c++) {
#pragma unroll
        for (int f = 0; f < NF; f++) asm volatile("" : "+v"(C.R[c][f]), "+v"(C.v[c][f]));
#pragma unroll
        for (int a = 0; a < 3; a++) asm volatile("" : "+v"(C.g[c][a]), "+v"(C.B[c][a]), "+v"(C.J[c][a]), "+v"(C.Bd[c][a]));
    }
}

template <typename T, int CZ>
__device__ __forceinline__ void pin_up6(Cells<T, CZ> &C)
{
#pragma unroll
    for (int c = 0; c < CZ; c++) asm volatile("" : "+v"(C.up6[c][0]), "+v"(C.up6[c][1]), "+v"(C.up6[c][2]));
}

template <typename T, int CZ>
__device__ __forceinline__ void pin_pend(Cells<T, CZ> &C, int n)
{
#pragma unroll
    for (int c = 0; c < CZ; c++)
#pragma unroll
        for (int a = 0; a < 3; a++)
            if (a < n) asm volatile("" : "+v"(C.pend[c][a]));
}

// Fold the derivatives of field F at this thread's cells into the accumulators.
// Fields pass in the order ln rho, A_x, A_y, A_z, u_x, u_y, u_z.
// UFIRST: the ring kernel's order ln rho, u_x, u_y, u_z, A_x, A_y, A_z, in which every
// centre value comes from its own field's box: the advection products whose velocity
// component has not passed yet are held as their derivative (pend) and completed in
// the later u passes, and -u.grad ln rho is added once u_z has passed.
// UPW: upwinding of the continuity advection, -(u_a d_a ln rho) gains
// + c |u_a| delta6_a ln rho / (60 h_a) (added once u is known).
template <typename T, int F, int SY, int SZ, int CZ, bool DIAG, bool UFIRST = false, bool UPW = false, class KR>
__device__ __forceinline__ void absorb(Cells<T, CZ> &C, const T *S, const int (&cidx)[CZ], const KR &K,
                                       const DCoef &dc)
{
    constexpr int s0 = 1, s1 = SY, s2 = SZ;
#pragma unroll
    for (int c = 0; c < CZ; c++) {
        const T *s = S + cidx[c];
        if constexpr (F == 0) {
            C.g[c][0] = sd1(s, s0, K.ih1[0]);
            C.g[c][1] = sd1(s, s1, K.ih1[1]);
            C.g[c][2] = sd1(s, s2, K.ih1[2]);
            if constexpr (UFIRST)
                C.v[c][0] = s[0];
            else
                C.R[c][0] -= C.v[c][1] * C.g[c][0] + C.v[c][2] * C.g[c][1] + C.v[c][3] * C.g[c][2];
            if constexpr (UPW) {
                const T q0 = sd6(s, s0), q1 = sd6(s, s1), q2 = sd6(s, s2);
                if constexpr (UFIRST) {
                    C.up6[c][0] = q0;
                    C.up6[c][1] = q1;
                    C.up6[c][2] = q2;
                } else {
                    C.R[c][0] += K.upw[0] * fabs(C.v[c][1]) * q0 + K.upw[1] * fabs(C.v[c][2]) * q1 +
                                 K.upw[2] * fabs(C.v[c][3]) * q2;
                }
            }
            C.R[c][1] -= K.cs2 * C.g[c][0];
            C.R[c][2] -= K.cs2 * C.g[c][1];
            C.R[c][3] -= K.cs2 * C.g[c][2];
        } else if constexpr (F >= 4) {
            constexpr int m = F - 4;  // A_m
            constexpr int b1 = (m + 1) % 3, b2 = (m + 2) % 3;  // the other two axes, cyclic
            constexpr int st1 = Stride<b1, SY, SZ>::v, st2 = Stride<b2, SY, SZ>::v, stm = Stride<m, SY, SZ>::v;
            C.v[c][F] = s[0];
            const T d2m = sd2(s, stm, K.ih2[m]);
            const T d21 = sd2(s, st1, K.ih2[b1]);
            const T d22 = sd2(s, st2, K.ih2[b2]);
            C.R[c][F] += K.eta * (d2m + d21 + d22);
            // j_m = sum_{b != m} (d_m d_b A_b - d_b d_b A_m): the second part here
            C.J[c][m] -= d21 + d22;
            // j_b += d_b d_m A_m for b != m
            C.J[c][b1] += sdm(s, st1, stm, K.ihm[Pair<b1, m>::v]);
            C.J[c][b2] += sdm(s, st2, stm, K.ihm[Pair<b2, m>::v]);
            // B = curl A: A_m enters B_{b1} with + d_{b2} A_m and B_{b2} with - d_{b1} A_m
            const T e1 = sd1(s, st1, K.ih1[b1]);
            const T e2 = sd1(s, st2, K.ih1[b2]);
            C.B[c][b1] += e2;
            C.B[c][b2] -= e1;
            if constexpr (DIAG) {  // FP64 curl for the diagnostics (recomputed for FP32 states)
                if constexpr (sizeof(T) == 8) {
                    C.Bd[c][b1] += (double)e2;
                    C.Bd[c][b2] -= (double)e1;
                } else {
                    C.Bd[c][b1] += sd1d(s, st2, dc.ih1[b2]);
                    C.Bd[c][b2] -= sd1d(s, st1, dc.ih1[b1]);
                }
            }
            if constexpr (F == 6) {
                // A complete (B started from the imposed field): Lorentz force and induction
                const T rinv = exp(-C.v[c][0]);
                const T *Bv = C.B[c], *Jv = C.J[c], *u = &C.v[c][1];
                C.R[c][1] += rinv * (Jv[1] * Bv[2] - Jv[2] * Bv[1]);
                C.R[c][2] += rinv * (Jv[2] * Bv[0] - Jv[0] * Bv[2]);
                C.R[c][3] += rinv * (Jv[0] * Bv[1] - Jv[1] * Bv[0]);
                C.R[c][4] += u[1] * Bv[2] - u[2] * Bv[1];
                C.R[c][5] += u[2] * Bv[0] - u[0] * Bv[2];
                C.R[c][6] += u[0] * Bv[1] - u[1] * Bv[0];
            }
        } else {
            constexpr int m = F - 1;  // u_m
            constexpr int b1 = (m + 1) % 3, b2 = (m + 2) % 3;
            constexpr int st1 = Stride<b1, SY, SZ>::v, st2 = Stride<b2, SY, SZ>::v, stm = Stride<m, SY, SZ>::v;
            T du[3];
            du[m] = sd1(s, stm, K.ih1[m]);
            du[b1] = sd1(s, st1, K.ih1[b1]);
            du[b2] = sd1(s, st2, K.ih1[b2]);
            const T d2m = sd2(s, stm, K.ih2[m]);
            const T lap = d2m + sd2(s, st1, K.ih2[b1]) + sd2(s, st2, K.ih2[b2]);
            const T *g = C.g[c], *u = &C.v[c][1];
            // viscous: nu lap u_m + nu/3 d_m d_m u_m; advection; strain row m
            T rm = K.nu * lap + K.nu3 * d2m;
            if constexpr (UFIRST) {
                C.v[c][F] = s[0];
                if constexpr (m == 0) {
                    rm -= u[0] * du[0];
                    C.pend[c][0] = du[1];
                    C.pend[c][1] = du[2];
                } else if constexpr (m == 1) {
                    C.R[c][1] -= u[1] * C.pend[c][0];
                    rm -= u[0] * du[0] + u[1] * du[1];
                    C.pend[c][2] = du[2];
                } else {
                    C.R[c][1] -= u[2] * C.pend[c][1];
                    C.R[c][2] -= u[2] * C.pend[c][2];
                    rm -= u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
                    C.R[c][0] -= u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
                    if constexpr (UPW)
                        C.R[c][0] += K.upw[0] * fabs(u[0]) * C.up6[c][0] + K.upw[1] * fabs(u[1]) * C.up6[c][1] +
                                     K.upw[2] * fabs(u[2]) * C.up6[c][2];
                }
            } else {
                rm -= u[0] * du[0] + u[1] * du[1] + u[2] * du[2];
            }
            rm += K.nu * (du[0] * g[0] + du[1] * g[1] + du[2] * g[2]);
            C.R[c][1 + m] += rm;
            C.R[c][0] -= du[m];
            // strain column m and trace part, for every component a
#pragma unroll
            for (int a = 0; a < 3; a++) C.R[c][1 + a] += K.nu * du[a] * g[m] - K.nu2_3 * du[m] * g[a];
            // grad div u: d_a d_m u_m for a != m
            C.R[c][1 + b1] += K.nu3 * sdm(s, st1, stm, K.ihm[Pair<b1, m>::v]);
            C.R[c][1 + b2] += K.nu3 * sdm(s, st2, stm, K.ihm[Pair<b2, m>::v]);
        }
    }
    pin(C);
}

template <typename T, int NL, int NT, int VOL>
__device__ __forceinline__ void stage_load(T (&stage)[NL], const G<T> *src, const uint32_t (&gofs)[NL])
{
#pragma unroll
    for (int k = 0; k < NL; k++) stage[k] = src[gofs[k]];
}

template <typename T, int NL, int NT, int VOL>
__device__ __forceinline__ void stage_store(T *dst, const T (&stage)[NL], int tid)
{
#pragma unroll
    for (int k = 0; k < NL; k++) {
        const int q = tid + k * NT;
        if (k < NL - 1 || q < VOL) dst[q] = stage[k];
    }
}

// One DPP move of a double (two 32-bit halves); lanes without a source read 0, the
// identity of both reductions below (the maxima are of non-negative values).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum (or maximum) over the 64 lanes of a wave, valid in lane 63: shifts right by 1,
// 2, 4, 8 within each row of 16 lanes, then row 0/2 totals broadcast into rows 1/3
// (row_bcast:15), then the row 1 total into rows 2 and 3 (row_bcast:31).
template <bool MAX>
__device__ __forceinline__ double wave_reduce(double v)
{
    auto op = [](double a, double b) { return MAX ? fmax(a, b) : a + b; };
    v = op(v, dpp_move<0x111, 0xF>(v));
    v = op(v, dpp_move<0x112, 0xF>(v));
    v = op(v, dpp_move<0x114, 0xF>(v));
    v = op(v, dpp_move<0x118, 0xF>(v));
    v = op(v, dpp_move<0x142, 0xA>(v));
    v = op(v, dpp_move<0x143, 0xC>(v));
    return v;
}

// Forcing, RK3 update and diagnostic partials of this thread's cells (shared by
// both substep kernels).  `red` is LDS scratch of at least 9 doubles per wave,
// free once every thread has passed the preceding barrier.
template <typename T, int CZ, int NT, int SUB, bool DIAG, bool STORE, bool FORCE = true>
__device__ __forceinline__ void finish(Cells<T, CZ> &C, const RunDesc<T> &r, const TileEnt &te, const Coef<T> &K,
                                       const DCoef &dc, const bool (&inside)[CZ], const uint32_t (&gcell)[CZ],
                                       const int (&gpos)[CZ][3], G<T> *const (&out)[NF], double *red, int step,
                                       int tid)
{
    if constexpr (STORE) {
        // forcing (held fixed over the step's substeps)
        const G<T> *fs = (const G<T> *)r.forcing + (size_t)step * (size_t)r.fstride;
        if (FORCE && fs[6] != T(0)) {
            constexpr int W = FSLOT<T>;
            const G<T> *Ex = fs + FHEAD, *Ey = Ex + W * r.nx, *Ez = Ey + W * r.ny;
#pragma unroll
            for (int c = 0; c < CZ; c++) {
                if (!inside[c]) continue;
                const int gx = gpos[c][0], gy = gpos[c][1], gz = gpos[c][2];
                const T xr = Ex[W * gx], xi = Ex[W * gx + 1];
                const T yr = Ey[W * gy], yi = Ey[W * gy + 1];
                const T zr = Ez[W * gz], zi = Ez[W * gz + 1];
                const T pr = xr * yr - xi * yi, pi = xr * yi + xi * yr;
                const T cr = pr * zr - pi * zi, ci = pr * zi + pi * zr;
#pragma unroll
                for (int a = 0; a < 3; a++) C.R[c][1 + a] += fs[a] * cr + fs[3 + a] * ci;
            }
        }

        const T bdt = K.bdt[SUB], brho = K.brho[SUB];
#pragma unroll
        for (int c = 0; c < CZ; c++) {
            if (!inside[c]) continue;
#pragma unroll
            for (int f = 0; f < NF; f++) {
                T o;
                if constexpr (SUB == 0) {
                    o = C.v[c][f] + bdt * C.R[c][f];
                } else {
                    const T old = C.have_old ? C.old[c][f] : T(out[f][gcell[c]]);
                    o = C.v[c][f] + brho * (C.v[c][f] - old) + bdt * C.R[c][f];
                }
                out[f][gcell[c]] = o;
            }
        }
    }

    if constexpr (DIAG) {
        double acc[9];
#pragma unroll
        for (int q = 0; q < 9; q++) acc[q] = 0.0;
#pragma unroll
        for (int c = 0; c < CZ; c++) {
            if (!inside[c]) continue;
            const double bx = C.Bd[c][0] + dc.bext[0], by = C.Bd[c][1] + dc.bext[1], bz = C.Bd[c][2] + dc.bext[2];
            const double ux = (double)C.v[c][1], uy = (double)C.v[c][2], uz = (double)C.v[c][3];
            const double u2 = ux * ux + uy * uy + uz * uz;
            const double b2 = bx * bx + by * by + bz * bz;
            acc[0] += b2;
            acc[1] += u2;
            acc[2] += exp((double)C.v[c][0]) * u2;
            acc[3] += (double)C.v[c][0];
            acc[4] += bx;
            acc[5] += by;
            acc[6] += bz;
            acc[7] = fmax(acc[7], u2);
            bool ok = true;
#pragma unroll
            for (int f = 0; f < NF; f++) ok = ok && finite_v(C.v[c][f]);
            acc[8] += ok ? 0.0 : 1.0;
        }
        // wave reduction with DPP row moves (VALU only, no LDS traffic), totals in lane
        // 63; then across waves through LDS (fixed order: deterministic)
#pragma unroll
        for (int q = 0; q < 9; q++) acc[q] = (q == 7) ? wave_reduce<true>(acc[q]) : wave_reduce<false>(acc[q]);
        constexpr int NW = NT / 64;
        __syncthreads();
        const int wave = tid / 64, lane = tid % 64;
        if (lane == 63) {
#pragma unroll
            for (int q = 0; q < 9; q++) red[wave * 9 + q] = acc[q];
        }
        __syncthreads();
        if (tid < 9) {
            double sum = red[tid];
            for (int w = 1; w < NW; w++) sum = (tid == 7) ? fmax(sum, red[w * 9 + tid]) : sum + red[w * 9 + tid];
            ((G<double> *)r.partials)[(size_t)te.tir * DIAGW + tid] = sum;
        }
    }
}

template <typename T, int TX, int TY, int TZ, int CZ, int SUB, bool DIAG, bool STORE, int WPE, bool UPW = false>
__global__ void __launch_bounds__(TX * TY * (TZ / CZ), WPE)
k_substep(const RunDesc<T> *__restrict__ runs, const TileEnt *__restrict__ tiles, int step)
{
    constexpr int NT = TX * TY * (TZ / CZ);
    constexpr int XW = TX + 6, YW = TY + 6, ZW = TZ + 6;
    constexpr int VOL = XW * YW * ZW;
    constexpr int NL = (VOL + NT - 1) / NT;
    constexpr int SY = XW, SZ = XW * YW;
    constexpr int ZS = TZ / CZ;  // z distance between a thread's cells

    __shared__ __align__(16) T lds[2][VOL];

    const TileEnt te = tiles[blockIdx.x];
    const RunDesc<T> &r = runs[te.run];
    const int nx = r.nx, ny = r.ny, nz = r.nz;
    const int x0 = te.xy & 0xffff, y0 = te.xy >> 16, z0 = te.z0;
    const int par = (r.parity0 + step) & 1;
    // substep 0 and the diagnostic pass read X, substep 1 reads Y, substep 2 reads X
    const int in_set = (SUB == 1) ? (par ^ 1) : par;
    const int out_set = (SUB == 1) ? par : (par ^ 1);
    const G<T> *in[NF];
    G<T> *out[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        in[f] = (const G<T> *)r.buf[in_set][f];
        out[f] = (G<T> *)r.buf[out_set][f];
    }

    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz0 = tid / (TX * TY);

    // global offsets of this thread's share of the halo box (same for every field)
    uint32_t gofs[NL];
#pragma unroll
    for (int k = 0; k < NL; k++) {
        int q = tid + k * NT;
        if (q >= VOL) q = VOL - 1;
        const int qx = q % XW, qy = (q / XW) % YW, qz = q / SZ;
        const int gx = wrapi(x0 - 3 + qx, nx), gy = wrapi(y0 - 3 + qy, ny), gz = wrapi(z0 - 3 + qz, nz);
        gofs[k] = (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz);
    }

    // this thread's cells
    int cidx[CZ];
    uint32_t gcell[CZ];
    bool inside[CZ];
#pragma unroll
    for (int c = 0; c < CZ; c++) {
        const int lz = lz0 + c * ZS;
        cidx[c] = (lz + 3) * SZ + (ly + 3) * SY + (lx + 3);
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        inside[c] = gx < nx && gy < ny && gz < nz;
        gcell[c] = inside[c] ? (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz) : 0u;
    }

    Cells<T, CZ> C;
#pragma unroll
    for (int c = 0; c < CZ; c++) {
#pragma unroll
        for (int f = 0; f < NF; f++) C.R[c][f] = T(0);
#pragma unroll
        for (int a = 0; a < 3; a++) { C.B[c][a] = r.c.bext[a]; C.J[c][a] = T(0); C.Bd[c][a] = 0.0; }
        // u and ln rho at the cell are needed by every pass: read them first
        C.v[c][0] = in[0][gcell[c]];
        C.v[c][1] = in[1][gcell[c]];
        C.v[c][2] = in[2][gcell[c]];
        C.v[c][3] = in[3][gcell[c]];
    }

    KRegsFor<T, UPW> K;
    K.load(r.c);
    const DCoef &dc = r.dc;
    T stage[NL];

    stage_load<T, NL, NT, VOL>(stage, in[0], gofs);
    stage_store<T, NL, NT, VOL>(lds[0], stage, tid);
    __syncthreads();
    // Each pass: issue the next field's loads, differentiate the current field out
    // of LDS, then write the staged values.  The scheduling fences keep the compiler
    // from hoisting the LDS writes (and their wait on the loads) above the compute.
    stage_load<T, NL, NT, VOL>(stage, in[4], gofs);
    __builtin_amdgcn_sched_barrier(0);
    absorb<T, 0, SY, SZ, CZ, DIAG, false, UPW>(C, lds[0], cidx, K, dc);
    __builtin_amdgcn_sched_barrier(0);
    stage_store<T, NL, NT, VOL>(lds[1], stage, tid);
    __syncthreads();
    stage_load<T, NL, NT, VOL>(stage, in[5], gofs);
    __builtin_amdgcn_sched_barrier(0);
    absorb<T, 4, SY, SZ, CZ, DIAG, false, UPW>(C, lds[1], cidx, K, dc);
    __builtin_amdgcn_sched_barrier(0);
    stage_store<T, NL, NT, VOL>(lds[0], stage, tid);
    __syncthreads();
    stage_load<T, NL, NT, VOL>(stage, in[6], gofs);
    __builtin_amdgcn_sched_barrier(0);
    absorb<T, 5, SY, SZ, CZ, DIAG, false, UPW>(C, lds[0], cidx, K, dc);
    __builtin_amdgcn_sched_barrier(0);
    stage_store<T, NL, NT, VOL>(lds[1], stage, tid);
    __syncthreads();
    stage_load<T, NL, NT, VOL>(stage, in[1], gofs);
    __builtin_amdgcn_sched_barrier(0);
    absorb<T, 6, SY, SZ, CZ, DIAG, false, UPW>(C, lds[1], cidx, K, dc);
    __builtin_amdgcn_sched_barrier(0);
    stage_store<T, NL, NT, VOL>(lds[0], stage, tid);
    __syncthreads();
    if constexpr (STORE) {
        stage_load<T, NL, NT, VOL>(stage, in[2], gofs);
        __builtin_amdgcn_sched_barrier(0);
        absorb<T, 1, SY, SZ, CZ, DIAG, false, UPW>(C, lds[0], cidx, K, dc);
        __builtin_amdgcn_sched_barrier(0);
        stage_store<T, NL, NT, VOL>(lds[1], stage, tid);
        __syncthreads();
        stage_load<T, NL, NT, VOL>(stage, in[3], gofs);
        __builtin_amdgcn_sched_barrier(0);
        absorb<T, 2, SY, SZ, CZ, DIAG, false, UPW>(C, lds[1], cidx, K, dc);
        __builtin_amdgcn_sched_barrier(0);
        stage_store<T, NL, NT, VOL>(lds[0], stage, tid);
        __syncthreads();
        absorb<T, 3, SY, SZ, CZ, DIAG, false, UPW>(C, lds[0], cidx, K, dc);

    }
    int gpos[CZ][3];
#pragma unroll
    for (int c = 0; c < CZ; c++) {
        gpos[c][0] = x0 + lx;
        gpos[c][1] = y0 + ly;
        gpos[c][2] = z0 + lz0 + c * ZS;
    }
    finish<T, CZ, NT, SUB, DIAG, STORE>(C, r, te, r.c, dc, inside, gcell, gpos, out,
                                          reinterpret_cast<double *>(&lds[1][0]), step, tid);
}

// ------------------------------------------------------------------ pipelined variant
//
// Same arithmetic as k_substep, different staging: the halo box of each field is
// copied HBM -> LDS by the direct-to-LDS loads of gfx950 (global_load_lds_dwordx4,
// 16 bytes per lane, no registers involved) into a ring of three buffers, two
// fields ahead of the one being differentiated, so about twice the bytes are in
// flight per CU and no VGPRs hold staged data.  Completion is tracked with explicit
// vmcnt waits before plain s_barriers (a full __syncthreads would wait for every
// outstanding load, including the prefetches).  The box starts at x0-4 so that
// each 16-byte vector holds whole, contiguous elements of one row; this needs
// nx % (16 / sizeof(T)) == 0 and 16-byte aligned field arrays (checked on the host).

typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) const void gconst_void_t;

// s_waitcnt that limits only vmcnt (gfx9 encoding: vmcnt in bits 3:0 and 15:14,
// expcnt 6:4 and lgkmcnt 11:8 left at their maxima)
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit counter");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
}

// barrier for the ring: this wave's copies up to the limit have landed; all waves
// have finished the previous pass
template <int N>
__device__ __forceinline__ void ring_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    wait_vmcnt<N>();
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

template <typename T, int NV, int NT, int EPL>
__device__ __forceinline__ void ring_copy(const G<T> *src, T *buf, const uint32_t (&voff)[NV], int wave)
{
    const G<char> *base = (const G<char> *)src;
#pragma unroll
    for (int v = 0; v < NV; v++)
        __builtin_amdgcn_global_load_lds((gconst_void_t *)(base + voff[v]),
                                         (lds_void_t *)(buf + (v * NT + wave * 64) * EPL), 16, 0, 0);
}

// wait for this wave's LDS reads, then the work-group barrier
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0), vmcnt and expcnt unrestricted
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Direct-to-LDS copies issued per wave: every wave of a work-group issues the same
// number, so that the vmcnt waits of the ring hold for each wave.
template <typename T, int TX, int TY, int TZ, int NT, int NFI>
struct Interior {
    static constexpr int EPL = 16 / (int)sizeof(T);
    static constexpr int NCELL = TX * TY * TZ, IV = NCELL / EPL;
    static constexpr int NI = (NFI * IV + NT - 1) / NT;  // copies per wave
    static_assert(IV % 64 == 0, "each wave's vectors lie in one field");

    // the values of fields src[0..NFI) at the tile's cells; field k lands at
    // area + k * NCELL, cells x fastest.  Cells past the grid edge read a clamped,
    // valid address (their values are never used).
    // (the sources are separate scalars, not an array: a dynamically indexed array of
    // pointers would be placed in scratch memory)
    static __device__ __forceinline__ void copy(const G<T> *s0, const G<T> *s1, const G<T> *s2, const G<T> *s3,
                                                T *area, int wave, int lane, int x0s, int y0, int z0, int nx, int ny,
                                                int nz)
    {
        static_assert(NFI >= 1 && NFI <= 4, "up to four fields");
#pragma unroll
        for (int i = 0; i < NI; i++) {
            int qb = i * NT + wave * 64;                // first vector of this wave (uniform)
            if (qb > NFI * IV - 64) qb = NFI * IV - 64;  // spare waves repeat the last vectors
            const int f = qb / IV;
            const G<T> *base = f == 0 ? s0 : (f == 1 ? s1 : (f == 2 ? s2 : s3));
            const int c0 = (qb - f * IV + lane) * EPL;
            const int x = c0 % TX, y = (c0 / TX) % TY, z = c0 / (TX * TY);
            // x0s + x < 2 nx for the tile's own cells, but a tile wider than the grid
            // (TX > nx) reaches further: wrap fully, so that every lane's 16-byte vector
            // lies inside the field (x0s, x and nx are multiples of EPL)
            const int gx = (x0s + x) % nx;
            const int gy = min(y0 + y, ny - 1), gz = min(z0 + z, nz - 1);
            const uint32_t off = (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz);
            __builtin_amdgcn_global_load_lds((gconst_void_t *)(base + off), (lds_void_t *)(area + qb * EPL), 16, 0, 0);
        }
    }
};

// The step's forcing head and the phase-table slots of the tile's x, y and z indices
// (one copy per wave, all waves writing the same values to the same place).
template <typename T, int TX, int TY, int TZ>
struct ForcingSlots {
    static constexpr int EPL = 16 / (int)sizeof(T), HV = FHEAD / EPL;
    static constexpr int NFV = HV + TX + TY + TZ;
    static_assert(NFV <= 64, "one vector per lane");
    static_assert(FSLOT<T> == EPL, "one table index per vector");

    static __device__ __forceinline__ void copy(const G<T> *fs, T *area, int lane, int x0s, int y0, int z0, int nx,
                                                int ny, int nz)
    {
        const G<T> *Ex = fs + FHEAD, *Ey = Ex + EPL * nx, *Ez = Ey + EPL * ny;
        const G<T> *p = fs;
        int j = lane;
        if (j < HV) {
            p = fs + j * EPL;
        } else if ((j -= HV) < TX) {
            p = Ex + EPL * ((x0s + j) % nx);  // full wrap: TX may exceed nx
        } else if ((j -= TX) < TY) {
            p = Ey + EPL * min(y0 + j, ny - 1);
        } else if ((j -= TY) < TZ) {
            p = Ez + EPL * min(z0 + j, nz - 1);
        }
        __builtin_amdgcn_global_load_lds((gconst_void_t *)p, (lds_void_t *)area, 16, 0, 0);
    }

    // f = a cos(theta) + b sin(theta) at this thread's cells, into the momentum sums
    template <int CZ, int ZS>
    static __device__ __forceinline__ void add(Cells<T, CZ> &C, const T *F, int lx, int ly, int lz0)
    {
        if (!(F[6] != T(0))) return;
        const T *ex = F + (HV + lx) * EPL, *ey = F + (HV + TX + ly) * EPL;
#pragma unroll
        for (int c = 0; c < CZ; c++) {
            const T *ez = F + (HV + TX + TY + lz0 + c * ZS) * EPL;
            const T pr = ex[0] * ey[0] - ex[1] * ey[1], pi = ex[0] * ey[1] + ex[1] * ey[0];
            const T cr = pr * ez[0] - pi * ez[1], ci = pr * ez[1] + pi * ez[0];
#pragma unroll
            for (int q = 0; q < 3; q++) C.R[c][1 + q] += F[q] * cr + F[3 + q] * ci;
        }
    }
};

// LDS bytes of the ring kernel (three ring buffers)
template <typename T, int TX, int TY, int TZ, int CZ>
constexpr int pipe_lds_bytes()
{
    constexpr int NT = TX * TY * (TZ / CZ), EPL = 16 / (int)sizeof(T);
    constexpr int NVEC = (TX + 8) * (TY + 6) * (TZ + 6) / EPL;
    return 3 * ((NVEC + NT - 1) / NT) * NT * 16;
}

// Minimum waves per SIMD the ring kernel is compiled for (its register budget is
// 512 / this).  FP64 kernels need up to 256 registers: 2.  FP32 kernels: as many whole
// work-groups as the LDS holds, up to 6 waves per SIMD (one-cell kernels fit in 80
// registers: three 512-thread groups of 48 KB; two-cell kernels in 128: two groups of
// 72 KB; more would force spills).
template <typename T, int TX, int TY, int TZ, int CZ>
constexpr int pipe_waves()
{
    if (sizeof(T) != 4) return 2;
    constexpr int wpb = TX * TY * (TZ / CZ) / 64;
    constexpr int lds = pipe_lds_bytes<T, TX, TY, TZ, CZ>();
    int best = 2;
    for (int b = 1; b * lds <= 160 * 1024; b++) {
        const int w = b * wpb;
        if (w % 4 == 0 && w / 4 <= 6 && w / 4 > best) best = w / 4;
    }
    return best;
}

// Every read of the pipeline is a direct-to-LDS copy, which the compiler's wait
// analysis does not see; a register load issued before such copies would get a
// full drain (vmcnt(0)) in front of its first use, stalling the prefetch.  So the
// forcing slots and the s-2 state also travel through LDS, in ring buffers that are
// free at that moment, the centre values are read from the fields' own boxes, and
// every wait is explicit:
//   start: forcing slots -> buffer 2, field 0 -> 0, field 1 -> 1
//   pass 0: forcing from buffer 2, barrier, field 2 -> 2
//   passes 1-4: the next field two ahead; pass 5: s-2 state of ln rho, u -> 1;
//   pass 6: s-2 state of A -> 2; then the update reads them from LDS.
template <typename T, int TX, int TY, int TZ, int CZ, int SUB, bool DIAG, bool STORE, int WPE, bool FIT,
          bool UPW = false>
__global__ void __launch_bounds__(TX * TY * (TZ / CZ), WPE)
k_pipe(const RunDesc<T> *__restrict__ runs, const TileEnt *__restrict__ tiles, int step)
{
    constexpr int NT = TX * TY * (TZ / CZ);
    constexpr int EPL = 16 / (int)sizeof(T);
    constexpr int XW = TX + 8, YW = TY + 6, ZW = TZ + 6;
    constexpr int VOL = XW * YW * ZW;
    constexpr int NVEC = VOL / EPL;
    constexpr int NV = (NVEC + NT - 1) / NT;
    constexpr int BUF = NV * NT * EPL;
    constexpr int SY = XW, SZ = XW * YW;
    constexpr int ZS = TZ / CZ;
    constexpr int NCELL = TX * TY * TZ;
    using Old1 = Interior<T, TX, TY, TZ, NT, 4>;
    using Old2 = Interior<T, TX, TY, TZ, NT, 3>;
    using Frc = ForcingSlots<T, TX, TY, TZ>;
    static_assert(XW % EPL == 0 && TX % EPL == 0, "rows must hold whole vectors");
    static_assert(NT % 64 == 0, "whole waves");
    static_assert(64 * EPL <= BUF && 4 * NCELL <= BUF, "forcing slots and the s-2 state fit a ring buffer");
    static_assert(2 * NV + 1 < 64 && Old1::NI + Old2::NI < 64, "vmcnt is a 6-bit counter");
    static_assert(!(DIAG && SUB != 0), "diagnostics are taken in substep 0 only");

    __shared__ __align__(16) T lds[3][BUF];

    const TileEnt te = tiles[blockIdx.x];
    const RunDesc<T> &r = runs[te.run];
    const int nx = r.nx, ny = r.ny, nz = r.nz;
    // the tile grid is offset by xs cells in x (periodic), which places the rows of
    // the halo box on fewer 128-byte lines; x0 is the unshifted origin
    const int x0 = te.xy & 0xffff, y0 = te.xy >> 16, z0 = te.z0, x0s = x0 + r.xs;
    const int par = (r.parity0 + step) & 1;
    const int in_set = (SUB == 1) ? (par ^ 1) : par;
    const int out_set = (SUB == 1) ? par : (par ^ 1);
    const G<T> *in[NF];
    G<T> *out[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        in[f] = (const G<T> *)r.buf[in_set][f];
        out[f] = (G<T> *)r.buf[out_set][f];
    }

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz0 = tid / (TX * TY);

    // byte offsets of this thread's vectors of the halo box (same for every field)
    uint32_t voff[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        int qv = v * NT + tid;
        if (qv >= NVEC) qv = NVEC - 1;  // padding lanes re-read a valid vector
        const int q = qv * EPL;
        const int bx = q % XW, by = (q / XW) % YW, bz = q / SZ;
        int gx = x0s - 4 + bx, gy = y0 - 3 + by, gz = z0 - 3 + bz;
        if constexpr (FIT) {  // the box spans at most one period per axis
            gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
            gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
            gz += gz < 0 ? nz : (gz >= nz ? -nz : 0);
        } else {
            gx = wrapi(gx, nx);
            gy = wrapi(gy, ny);
            gz = wrapi(gz, nz);
        }
        voff[v] = (uint32_t)sizeof(T) * ((uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz));
    }
    // ln rho, u_x and A_x enter only through derivatives along the axes and in the xy and
    // xz planes: their boxes need no row that lies outside the tile in both y and z (the
    // four 3x3 corner blocks of rows).  Those vectors re-read an address another lane of
    // the same wave instruction reads anyway (or, if the whole instruction is corner rows,
    // one common address), so they add no line requests; the instruction count, and with
    // it every wait count, is unchanged.  Their LDS slots hold unused values.
    uint32_t voffx[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        int qv = v * NT + tid;
        if (qv >= NVEC) qv = NVEC - 1;
        const int q = qv * EPL;
        const int by = (q / XW) % YW, bz = q / SZ;
        const bool corner = (by < 3 || by >= 3 + TY) && (bz < 3 || bz >= 3 + TZ);
        const uint64_t need = __ballot(!corner);
        const int src = need ? __ffsll((unsigned long long)need) - 1 : 0;
        const uint32_t sub = __shfl(voff[v], src, 64);
        voffx[v] = corner ? sub : voff[v];
    }

    int cidx[CZ];
#pragma unroll
    for (int c = 0; c < CZ; c++) cidx[c] = (lz0 + c * ZS + 3) * SZ + (ly + 3) * SY + (lx + 4);

    KRegsFor<T, UPW> K;
    K.load(r.c);
    const DCoef &dc = r.dc;

    // fields pass in memory order ln rho, u_x, u_y, u_z, A_x, A_y, A_z (field k lives in
    // ring buffer k % 3 and is requested two passes ahead); each centre value comes
    // from its own field's box
    if constexpr (STORE)
        Frc::copy((const G<T> *)r.forcing + (size_t)step * (size_t)r.fstride, lds[2], lane, x0s, y0, z0, nx, ny, nz);
    ring_copy<T, NV, NT, EPL>(in[0], lds[0], voffx, wave);
    ring_copy<T, NV, NT, EPL>(in[1], lds[1], voffx, wave);

    Cells<T, CZ> C;
    ring_barrier<NV>();
#pragma unroll
    for (int c = 0; c < CZ; c++) {
#pragma unroll
        for (int f = 0; f < NF; f++) C.R[c][f] = T(0);
#pragma unroll
        for (int a = 0; a < 3; a++) { C.B[c][a] = r.c.bext[a]; C.J[c][a] = T(0); C.Bd[c][a] = 0.0; }
    }
    if constexpr (STORE) Frc::template add<CZ, ZS>(C, lds[2], lx, ly, lz0);
    pin(C);
    lds_barrier();  // buffer 2 (forcing slots) is read out
    ring_copy<T, NV, NT, EPL>(in[2], lds[2], voff, wave);
    absorb<T, 0, SY, SZ, CZ, DIAG, true, UPW>(C, lds[0], cidx, K, dc);
    if constexpr (UPW) pin_up6(C);

    ring_barrier<NV>();
    ring_copy<T, NV, NT, EPL>(in[3], lds[0], voff, wave);
    absorb<T, 1, SY, SZ, CZ, DIAG, true, UPW>(C, lds[1], cidx, K, dc);
    pin_pend(C, 2);
    if constexpr (UPW) pin_up6(C);

    ring_barrier<NV>();
    ring_copy<T, NV, NT, EPL>(in[4], lds[1], voffx, wave);
    absorb<T, 2, SY, SZ, CZ, DIAG, true, UPW>(C, lds[2], cidx, K, dc);
    pin_pend(C, 3);
    if constexpr (UPW) pin_up6(C);

    ring_barrier<NV>();
    ring_copy<T, NV, NT, EPL>(in[5], lds[2], voff, wave);
    absorb<T, 3, SY, SZ, CZ, DIAG, true, UPW>(C, lds[0], cidx, K, dc);

    ring_barrier<NV>();
    ring_copy<T, NV, NT, EPL>(in[6], lds[0], voff, wave);
    absorb<T, 4, SY, SZ, CZ, DIAG, true, UPW>(C, lds[1], cidx, K, dc);

    ring_barrier<NV>();
    if constexpr (STORE && SUB != 0)  // buffer 1 (A_x) is read out: the s-2 state of ln rho, u
        Old1::copy(out[0], out[1], out[2], out[3], lds[1], wave, lane, x0s, y0, z0, nx, ny, nz);
    absorb<T, 5, SY, SZ, CZ, DIAG, true, UPW>(C, lds[2], cidx, K, dc);

    if constexpr (STORE && SUB != 0) {
        ring_barrier<Old1::NI>();
        // buffer 2 (A_y) is read out: the s-2 state of A
        Old2::copy(out[4], out[5], out[6], out[6], lds[2], wave, lane, x0s, y0, z0, nx, ny, nz);
    } else {
        ring_barrier<0>();
    }
    absorb<T, 6, SY, SZ, CZ, DIAG, true, UPW>(C, lds[0], cidx, K, dc);
    // the cells' global positions, computed here so that they hold no registers during
    // the passes
    __builtin_amdgcn_sched_barrier(0);
    int icell[CZ];
    uint32_t gcell[CZ];
    bool inside[CZ];
    int gpos[CZ][3];
#pragma unroll
    for (int c = 0; c < CZ; c++) {
        const int lz = lz0 + c * ZS;
        icell[c] = lx + TX * (ly + TY * lz);
        gpos[c][0] = x0s + lx >= nx ? x0s + lx - nx : x0s + lx;
        gpos[c][1] = y0 + ly;
        gpos[c][2] = z0 + lz;
        inside[c] = x0 + lx < nx && gpos[c][1] < ny && gpos[c][2] < nz;
        gcell[c] = inside[c] ? (uint32_t)gpos[c][0] + (uint32_t)nx * ((uint32_t)gpos[c][1] + (uint32_t)ny * (uint32_t)gpos[c][2])
                             : 0u;
    }
    if constexpr (STORE && SUB != 0) {
        ring_barrier<0>();
#pragma unroll
        for (int c = 0; c < CZ; c++) {
#pragma unroll
            for (int f = 0; f < 4; f++) C.old[c][f] = lds[1][f * NCELL + icell[c]];
#pragma unroll
            for (int f = 4; f < NF; f++) C.old[c][f] = lds[2][(f - 4) * NCELL + icell[c]];
        }
        C.have_old = true;
    }
    __builtin_amdgcn_sched_barrier(0);
    finish<T, CZ, NT, SUB, DIAG, STORE, false>(C, r, te, r.c, dc, inside, gcell, gpos, out,
                                                 reinterpret_cast<double *>(&lds[1][0]), step, tid);
}

// ------------------------------------------------------------------ z-marching variant
//
// A work-group owns one TX x TY column of one run and marches through a z-segment in
// slabs of TZ planes (one cell per thread).  Every field keeps a ring of TZ + 6
// planes in LDS, the planes z-3 .. z+TZ+2 of the current slab.  Once a field's pass
// of a slab is done its TZ oldest planes are dead, and the next slab's TZ planes are
// requested into their slots, six passes ahead of use.  Planes shared by consecutive
// slabs therefore come from memory once; only the x and y halos are re-read, by the
// neighbouring columns (which march at the same time, so they meet in L2).  The
// z-stencil reaches into the ring through seven per-thread plane pointers.
//
// Terms that need a field at the cell before its pass has come (the advection of
// ln rho and u, the induction u x B) are kept as their factors and added at the end
// of the slab, so that the pipeline needs no out-of-order waits.

template <typename T, int SY>
struct PlaneAcc {
    const T *zp[7];  // this cell's (x, y) in the planes z-3 .. z+3
    template <int DX, int DY, int DZ>
    __device__ __forceinline__ T get() const
    {
        return zp[DZ + 3][DX + DY * SY];
    }
};

template <int AX, int M>
struct Ax {
    static constexpr int x = AX == 0 ? M : 0, y = AX == 1 ? M : 0, z = AX == 2 ? M : 0;
};

template <typename T, int AX, class A>
__device__ __forceinline__ T gd1(const A &a, T ih)
{
    using P1 = Ax<AX, 1>;
    using P2 = Ax<AX, 2>;
    using P3 = Ax<AX, 3>;
    return ih * (T(W1_1) * (a.template get<P1::x, P1::y, P1::z>() - a.template get<-P1::x, -P1::y, -P1::z>()) +
                 T(W1_2) * (a.template get<P2::x, P2::y, P2::z>() - a.template get<-P2::x, -P2::y, -P2::z>()) +
                 T(W1_3) * (a.template get<P3::x, P3::y, P3::z>() - a.template get<-P3::x, -P3::y, -P3::z>()));
}

template <typename T, int AX, class A>
__device__ __forceinline__ T gd2(const A &a, T ih2)
{
    using P1 = Ax<AX, 1>;
    using P2 = Ax<AX, 2>;
    using P3 = Ax<AX, 3>;
    return ih2 * (T(W2_0) * a.template get<0, 0, 0>() +
                  T(W2_1) * (a.template get<P1::x, P1::y, P1::z>() + a.template get<-P1::x, -P1::y, -P1::z>()) +
                  T(W2_2) * (a.template get<P2::x, P2::y, P2::z>() + a.template get<-P2::x, -P2::y, -P2::z>()) +
                  T(W2_3) * (a.template get<P3::x, P3::y, P3::z>() + a.template get<-P3::x, -P3::y, -P3::z>()));
}

template <int AX, class A>
__device__ __forceinline__ double gd1d(const A &a, double ih)
{
    using P1 = Ax<AX, 1>;
    using P2 = Ax<AX, 2>;
    using P3 = Ax<AX, 3>;
    auto d = [&](auto v) { return (double)v; };
    return ih * (W1_1 * (d(a.template get<P1::x, P1::y, P1::z>()) - d(a.template get<-P1::x, -P1::y, -P1::z>())) +
                 W1_2 * (d(a.template get<P2::x, P2::y, P2::z>()) - d(a.template get<-P2::x, -P2::y, -P2::z>())) +
                 W1_3 * (d(a.template get<P3::x, P3::y, P3::z>()) - d(a.template get<-P3::x, -P3::y, -P3::z>())));
}

template <typename T, int AX, class A>
__device__ __forceinline__ T gd6(const A &a)
{
    using P1 = Ax<AX, 1>;
    using P2 = Ax<AX, 2>;
    using P3 = Ax<AX, 3>;
    return T(-20) * a.template get<0, 0, 0>() +
           T(15) * (a.template get<P1::x, P1::y, P1::z>() + a.template get<-P1::x, -P1::y, -P1::z>()) +
           T(-6) * (a.template get<P2::x, P2::y, P2::z>() + a.template get<-P2::x, -P2::y, -P2::z>()) +
           (a.template get<P3::x, P3::y, P3::z>() + a.template get<-P3::x, -P3::y, -P3::z>());
}

// d_a d_b from the (a+b) and (a-b) diagonals
template <typename T, int AA, int AB, class A>
__device__ __forceinline__ T gdm(const A &a, T ihm)
{
    constexpr int px = Ax<AA, 1>::x + Ax<AB, 1>::x, py = Ax<AA, 1>::y + Ax<AB, 1>::y, pz = Ax<AA, 1>::z + Ax<AB, 1>::z;
    constexpr int qx = Ax<AA, 1>::x - Ax<AB, 1>::x, qy = Ax<AA, 1>::y - Ax<AB, 1>::y, qz = Ax<AA, 1>::z - Ax<AB, 1>::z;
    return ihm * (T(W2_1) * ((a.template get<px, py, pz>() + a.template get<-px, -py, -pz>()) -
                             (a.template get<qx, qy, qz>() + a.template get<-qx, -qy, -qz>())) +
                  T(W2_2) * ((a.template get<2 * px, 2 * py, 2 * pz>() + a.template get<-2 * px, -2 * py, -2 * pz>()) -
                             (a.template get<2 * qx, 2 * qy, 2 * qz>() + a.template get<-2 * qx, -2 * qy, -2 * qz>())) +
                  T(W2_3) * ((a.template get<3 * px, 3 * py, 3 * pz>() + a.template get<-3 * px, -3 * py, -3 * pz>()) -
                             (a.template get<3 * qx, 3 * qy, 3 * qz>() + a.template get<-3 * qx, -3 * qy, -3 * qz>())));
}

// per-cell accumulators of the marching kernel
template <typename T>
struct CellM {
    T v[NF];      // centre values
    T g[3];       // grad ln rho
    T B[3], J[3];
    T R[NF];
    T du[3][3];   // du[m][a] = d_a u_m, for the advection added at the end
    T up6[3];     // upwinding: sixth differences of ln rho, added at the end
    double Bd[3];
};

template <typename T>
__device__ __forceinline__ void pin_up6(CellM<T> &C)
{
    asm volatile("" : "+v"(C.up6[0]), "+v"(C.up6[1]), "+v"(C.up6[2]));
}

template <typename T>
__device__ __forceinline__ void pin(CellM<T> &C)
{
#pragma unroll
    for (int f = 0; f < NF; f++) asm volatile("" : "+v"(C.R[f]), "+v"(C.v[f]));
#pragma unroll
    for (int a = 0; a < 3; a++) {
        asm volatile("" : "+v"(C.g[a]), "+v"(C.B[a]), "+v"(C.J[a]), "+v"(C.Bd[a]));
        asm volatile("" : "+v"(C.du[a][0]), "+v"(C.du[a][1]), "+v"(C.du[a][2]));
    }
}

// Fold field F's derivatives at this cell into the accumulators (same terms as
// absorb, with the advection and induction deferred).
template <typename T, int F, bool DIAG, bool UPW, class A, class KR>
__device__ __forceinline__ void absorb_m(CellM<T> &C, const A &s, const KR &K, const DCoef &dc)
{
    if constexpr (F == 0) {
        C.v[0] = s.template get<0, 0, 0>();
        C.g[0] = gd1<T, 0>(s, K.ih1[0]);
        C.g[1] = gd1<T, 1>(s, K.ih1[1]);
        C.g[2] = gd1<T, 2>(s, K.ih1[2]);
        if constexpr (UPW) {
            C.up6[0] = gd6<T, 0>(s);
            C.up6[1] = gd6<T, 1>(s);
            C.up6[2] = gd6<T, 2>(s);
        }
        C.R[1] -= K.cs2 * C.g[0];
        C.R[2] -= K.cs2 * C.g[1];
        C.R[3] -= K.cs2 * C.g[2];
    } else if constexpr (F >= 4) {
        constexpr int m = F - 4;
        constexpr int b1 = (m + 1) % 3, b2 = (m + 2) % 3;
        C.v[F] = s.template get<0, 0, 0>();
        const T d2m = gd2<T, m>(s, K.ih2[m]);
        const T d21 = gd2<T, b1>(s, K.ih2[b1]);
        const T d22 = gd2<T, b2>(s, K.ih2[b2]);
        C.R[F] += K.eta * (d2m + d21 + d22);
        C.J[m] -= d21 + d22;
        C.J[b1] += gdm<T, b1, m>(s, K.ihm[Pair<b1, m>::v]);
        C.J[b2] += gdm<T, b2, m>(s, K.ihm[Pair<b2, m>::v]);
        const T e1 = gd1<T, b1>(s, K.ih1[b1]);
        const T e2 = gd1<T, b2>(s, K.ih1[b2]);
        C.B[b1] += e2;
        C.B[b2] -= e1;
        if constexpr (DIAG) {  // FP64 curl for the diagnostics (recomputed for FP32 states)
            if constexpr (sizeof(T) == 8) {
                C.Bd[b1] += (double)e2;
                C.Bd[b2] -= (double)e1;
            } else {
                C.Bd[b1] += gd1d<b2>(s, dc.ih1[b2]);
                C.Bd[b2] -= gd1d<b1>(s, dc.ih1[b1]);
            }
        }
        if constexpr (F == 6) {  // A complete: Lorentz force (ln rho is known)
            const T rinv = exp(-C.v[0]);
            const T *Bv = C.B, *Jv = C.J;
            C.R[1] += rinv * (Jv[1] * Bv[2] - Jv[2] * Bv[1]);
            C.R[2] += rinv * (Jv[2] * Bv[0] - Jv[0] * Bv[2]);
            C.R[3] += rinv * (Jv[0] * Bv[1] - Jv[1] * Bv[0]);
        }
    } else {
        constexpr int m = F - 1;
        constexpr int b1 = (m + 1) % 3, b2 = (m + 2) % 3;
        C.v[F] = s.template get<0, 0, 0>();
        T du[3];
        du[m] = gd1<T, m>(s, K.ih1[m]);
        du[b1] = gd1<T, b1>(s, K.ih1[b1]);
        du[b2] = gd1<T, b2>(s, K.ih1[b2]);
        const T d2m = gd2<T, m>(s, K.ih2[m]);
        const T lap = d2m + gd2<T, b1>(s, K.ih2[b1]) + gd2<T, b2>(s, K.ih2[b2]);
        const T *g = C.g;
        T rm = K.nu * lap + K.nu3 * d2m;
        rm += K.nu * (du[0] * g[0] + du[1] * g[1] + du[2] * g[2]);
        C.R[1 + m] += rm;
        C.R[0] -= du[m];
#pragma unroll
        for (int a = 0; a < 3; a++) C.R[1 + a] += K.nu * du[a] * g[m] - K.nu2_3 * du[m] * g[a];
        C.R[1 + b1] += K.nu3 * gdm<T, b1, m>(s, K.ihm[Pair<b1, m>::v]);
        C.R[1 + b2] += K.nu3 * gdm<T, b2, m>(s, K.ihm[Pair<b2, m>::v]);
#pragma unroll
        for (int a = 0; a < 3; a++) C.du[m][a] = du[a];
    }
    pin(C);
    if constexpr (UPW) pin_up6(C);
}

// Planes [za, za + n) of one field into its ring (slot of plane z: (z - zbase) mod P),
// one 16-byte vector per lane, every wave issuing the same number of copies.  A plane
// slot holds SLOTV vectors (whole waves); lanes past the plane's PV vectors and waves
// past the last plane repeat valid reads into their own (padding or repeated) slot.
template <typename T, int TX, int TY, int NT, int P, int SLOTV, int NPL>
__device__ __forceinline__ void plane_copy(const G<T> *src, T *ring, int za, int zbase, int wave, int lane, int x0s,
                                           int y0, int nx, int ny, int nz)
{
    constexpr int EPL = 16 / (int)sizeof(T);
    constexpr int XW = TX + 8, YW = TY + 6, PV = XW * YW / EPL;
    constexpr int NI = (NPL * SLOTV + NT - 1) / NT;
#pragma unroll
    for (int i = 0; i < NI; i++) {
        const int qb = i * NT + wave * 64;  // wave-uniform
        int k = qb / SLOTV;
        const int vb = qb - k * SLOTV;
        if (k >= NPL) k = NPL - 1;
        const int z = za + k;
        int slot = (z - zbase) % P;
        slot += slot < 0 ? P : 0;
        int gz = z % nz;
        gz += gz < 0 ? nz : 0;
        int v = vb + lane;
        if (v >= PV) v = 0;
        const int e = v * EPL, row = e / XW, col = e - row * XW;
        int gx = x0s - 4 + col, gy = y0 - 3 + row;
        gx += gx < 0 ? nx : (gx >= nx ? -nx : 0);
        gy += gy < 0 ? ny : (gy >= ny ? -ny : 0);
        const uint32_t off = (uint32_t)gx + (uint32_t)nx * ((uint32_t)gy + (uint32_t)ny * (uint32_t)gz);
        __builtin_amdgcn_global_load_lds((gconst_void_t *)(src + off),
                                         (lds_void_t *)(ring + slot * SLOTV * EPL + vb * EPL), 16, 0, 0);
    }
}

// LDS layout and copy counts of the marching kernel
template <typename T, int TX, int TY, int TZ>
struct MarchCfg {
    static constexpr int NT = TX * TY * TZ, EPL = 16 / (int)sizeof(T);
    static constexpr int XW = TX + 8, YW = TY + 6, SY = XW;
    static constexpr int PV = XW * YW / EPL;
    static constexpr int SLOTV = (PV + 63) / 64 * 64;  // plane slot, whole waves of vectors
    static constexpr int SLOT = SLOTV * EPL;           // elements
    static constexpr int P = TZ + 6;                   // planes per field ring
    static constexpr int RING = P * SLOT;
    static constexpr int ND = (TZ * SLOTV + NT - 1) / NT;  // copies per wave, one field, one slab
    static constexpr int IV = NT / EPL;
    static constexpr int LDS_ELEMS = NF * RING + NF * NT + 64 * EPL;
    static constexpr int LDS_BYTES = LDS_ELEMS * (int)sizeof(T);
    static constexpr bool FITS = LDS_BYTES <= 160 * 1024;
};

template <typename T, int TX, int TY, int TZ, int SUB, bool DIAG, bool STORE, int WPE, bool UPW = false>
__global__ void __launch_bounds__(TX * TY * TZ, WPE)
k_march(const RunDesc<T> *__restrict__ runs, const TileEnt *__restrict__ tiles, int step)
{
    using M = MarchCfg<T, TX, TY, TZ>;
    constexpr int NT = M::NT, EPL = M::EPL, SY = M::SY, P = M::P, SLOT = M::SLOT, RING = M::RING;
    constexpr int ND = M::ND;
    using Old = Interior<T, TX, TY, TZ, NT, 4>;
    using Old3 = Interior<T, TX, TY, TZ, NT, 3>;
    using Frc = ForcingSlots<T, TX, TY, TZ>;
    constexpr bool OLDS = STORE && SUB != 0;
    constexpr int NO = OLDS ? Old::NI + Old3::NI : 0;  // s-2 state copies per slab
    constexpr int NFC = STORE ? 1 : 0;                 // forcing-slot copy per slab
    constexpr int ES = STORE ? NF : 0;                 // stores per slab
    static_assert(M::FITS, "rings, s-2 state and forcing slots fit the LDS");
    static_assert(M::XW % EPL == 0 && TX % EPL == 0, "rows must hold whole vectors");
    static_assert(5 * ND + ES + NO + NFC < 64, "vmcnt is a 6-bit counter");
    static_assert(!(DIAG && SUB != 0), "diagnostics are taken in substep 0 only");

    __shared__ __align__(16) T lds[M::LDS_ELEMS];
    T *const old_area = lds + NF * RING;
    T *const frc = old_area + NF * NT;

    const TileEnt te = tiles[blockIdx.x];
    const RunDesc<T> &r = runs[te.run];
    const int nx = r.nx, ny = r.ny, nz = r.nz;
    const int x0 = te.xy & 0xffff, y0 = te.xy >> 16, zs0 = te.z0, x0s = x0 + r.xs;
    const int nslab = r.seg / TZ;
    const int zbase = zs0 - 3;
    const int par = (r.parity0 + step) & 1;
    const int in_set = (SUB == 1) ? (par ^ 1) : par;
    const int out_set = (SUB == 1) ? par : (par ^ 1);
    const G<T> *in[NF];
    G<T> *out[NF];
#pragma unroll
    for (int f = 0; f < NF; f++) {
        in[f] = (const G<T> *)r.buf[in_set][f];
        out[f] = (G<T> *)r.buf[out_set][f];
    }
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int gxc = x0s + lx >= nx ? x0s + lx - nx : x0s + lx, gyc = y0 + ly;
    const int xyoff = (ly + 3) * SY + (lx + 4);

    KRegsFor<T, UPW> K;
    K.load(r.c);
    const DCoef &dc = r.dc;
    const G<T> *fblk = (const G<T> *)r.forcing + (size_t)step * (size_t)r.fstride;

    // field at each position of the pass order (ln rho, A, u) and its ring
    constexpr int SEQ[NF] = {0, 4, 5, 6, 1, 2, 3};
    auto ring = [&](int pos) { return lds + pos * RING; };
    auto planes = [&](int pos, int za, auto nplc) {
        constexpr int NPL = decltype(nplc)::value;
        plane_copy<T, TX, TY, NT, P, M::SLOTV, NPL>(in[SEQ[pos]], ring(pos), za, zbase, wave, lane, x0s, y0, nx, ny,
                                                   nz);
    };
    using TZc = std::integral_constant<int, TZ>;
    using Pc = std::integral_constant<int, P>;

    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; q++) acc[q] = 0.0;

    // prologue: every field's first window
#pragma unroll
    for (int pos = 0; pos < NF; pos++) planes(pos, zbase, Pc{});

    for (int sl = 0; sl < nslab; sl++) {
        const bool first = sl == 0;
        const int z0 = zs0 + sl * TZ;
        const int w = (sl * TZ) % P;  // ring slot of plane z0 - 3
        int zoff[7];
#pragma unroll
        for (int k = 0; k < 7; k++) {
            int sk = w + lz + k;
            sk -= sk >= P ? P : 0;
            sk -= sk >= P ? P : 0;
            zoff[k] = sk * SLOT + xyoff;
        }
        auto acc_for = [&](int pos) {
            PlaneAcc<T, SY> a;
#pragma unroll
            for (int k = 0; k < 7; k++) a.zp[k] = ring(pos) + zoff[k];
            return a;
        };
        auto wait_bar = [&](auto wc) {
            constexpr int WN = decltype(wc)::value;
            if (first) ring_barrier<0>();
            else ring_barrier<WN>();
        };
        CellM<T> C;
#pragma unroll
        for (int f = 0; f < NF; f++) C.R[f] = T(0);
#pragma unroll
        for (int a = 0; a < 3; a++) {
            C.B[a] = r.c.bext[a];
            C.J[a] = T(0);
            C.Bd[a] = 0.0;
        }

        // pass 0: ln rho; the last field's planes of this slab, the s-2 state
        wait_bar(std::integral_constant<int, 5 * ND + NFC + ES>{});
        if (!first) planes(6, z0 + TZ + 3 - TZ, TZc{});
        if constexpr (OLDS) {
            Old::copy(out[0], out[1], out[2], out[3], old_area, wave, lane, x0s, y0, z0, nx, ny, nz);
            Old3::copy(out[4], out[5], out[6], out[6], old_area + 4 * NT, wave, lane, x0s, y0, z0, nx, ny, nz);
        }
        absorb_m<T, 0, DIAG, UPW>(C, acc_for(0), K, dc);

        // pass 1: A_x; ln rho's next planes, this slab's forcing slots
        wait_bar(std::integral_constant<int, 5 * ND + ES + NO>{});
        planes(0, z0 + TZ + 3, TZc{});
        if constexpr (STORE) Frc::copy(fblk, frc, lane, x0s, y0, z0, nx, ny, nz);
        absorb_m<T, 4, DIAG, UPW>(C, acc_for(1), K, dc);

        wait_bar(std::integral_constant<int, 5 * ND + ES + NO + NFC>{});
        planes(1, z0 + TZ + 3, TZc{});
        absorb_m<T, 5, DIAG, UPW>(C, acc_for(2), K, dc);

        wait_bar(std::integral_constant<int, 5 * ND + ES + NO + NFC>{});
        planes(2, z0 + TZ + 3, TZc{});
        absorb_m<T, 6, DIAG, UPW>(C, acc_for(3), K, dc);

        wait_bar(std::integral_constant<int, 5 * ND + ES + NO + NFC>{});
        planes(3, z0 + TZ + 3, TZc{});
        absorb_m<T, 1, DIAG, UPW>(C, acc_for(4), K, dc);

        wait_bar(std::integral_constant<int, 5 * ND + ES + NO + NFC>{});
        planes(4, z0 + TZ + 3, TZc{});
        absorb_m<T, 2, DIAG, UPW>(C, acc_for(5), K, dc);

        wait_bar(std::integral_constant<int, 5 * ND + NO + NFC>{});
        planes(5, z0 + TZ + 3, TZc{});
        absorb_m<T, 3, DIAG, UPW>(C, acc_for(6), K, dc);

        // the end of the slab: deferred terms, forcing, RK update
        wait_bar(std::integral_constant<int, 5 * ND>{});
        const T *u = &C.v[1];
#pragma unroll
        for (int m = 0; m < 3; m++) C.R[1 + m] -= u[0] * C.du[m][0] + u[1] * C.du[m][1] + u[2] * C.du[m][2];
        C.R[0] -= u[0] * C.g[0] + u[1] * C.g[1] + u[2] * C.g[2];
        if constexpr (UPW)
            C.R[0] += K.upw[0] * fabs(u[0]) * C.up6[0] + K.upw[1] * fabs(u[1]) * C.up6[1] +
                      K.upw[2] * fabs(u[2]) * C.up6[2];
        C.R[4] += u[1] * C.B[2] - u[2] * C.B[1];
        C.R[5] += u[2] * C.B[0] - u[0] * C.B[2];
        C.R[6] += u[0] * C.B[1] - u[1] * C.B[0];
        const int gzc = z0 + lz;
        const uint32_t gcell = (uint32_t)gxc + (uint32_t)nx * ((uint32_t)gyc + (uint32_t)ny * (uint32_t)gzc);
        if constexpr (STORE) {
            if (frc[6] != T(0)) {
                constexpr int HV = Frc::HV;
                const T *ex = frc + (HV + lx) * EPL, *ey = frc + (HV + TX + ly) * EPL,
                        *ez = frc + (HV + TX + TY + lz) * EPL;
                const T pr = ex[0] * ey[0] - ex[1] * ey[1], pi = ex[0] * ey[1] + ex[1] * ey[0];
                const T cr = pr * ez[0] - pi * ez[1], ci = pr * ez[1] + pi * ez[0];
#pragma unroll
                for (int q = 0; q < 3; q++) C.R[1 + q] += frc[q] * cr + frc[3 + q] * ci;
            }
            const T bdt = r.c.bdt[SUB], brho = r.c.brho[SUB];
#pragma unroll
            for (int f = 0; f < NF; f++) {
                T o;
                if constexpr (SUB == 0) {
                    o = C.v[f] + bdt * C.R[f];
                } else {
                    const T old = old_area[f * NT + tid];
                    o = C.v[f] + brho * (C.v[f] - old) + bdt * C.R[f];
                }
                out[f][gcell] = o;
            }
        }
        if constexpr (DIAG) {
            const double bx = C.Bd[0] + dc.bext[0], by = C.Bd[1] + dc.bext[1], bz = C.Bd[2] + dc.bext[2];
            const double ux = (double)C.v[1], uy = (double)C.v[2], uz = (double)C.v[3];
            const double u2 = ux * ux + uy * uy + uz * uz;
            acc[0] += bx * bx + by * by + bz * bz;
            acc[1] += u2;
            acc[2] += exp((double)C.v[0]) * u2;
            acc[3] += (double)C.v[0];
            acc[4] += bx;
            acc[5] += by;
            acc[6] += bz;
            acc[7] = fmax(acc[7], u2);
            bool ok = true;
#pragma unroll
            for (int f = 0; f < NF; f++) ok = ok && finite_v(C.v[f]);
            acc[8] += ok ? 0.0 : 1.0;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    // no copy may still be writing into this work-group's LDS when it ends
    ring_barrier<0>();
    if constexpr (DIAG) {
#pragma unroll
        for (int q = 0; q < 9; q++) acc[q] = (q == 7) ? wave_reduce<true>(acc[q]) : wave_reduce<false>(acc[q]);
        double *red = reinterpret_cast<double *>(old_area);
        if (lane == 63) {
#pragma unroll
            for (int q = 0; q < 9; q++) red[wave * 9 + q] = acc[q];
        }
        __syncthreads();
        if (tid < 9) {
            double sum = red[tid];
            for (int wv = 1; wv < NT / 64; wv++) sum = (tid == 7) ? fmax(sum, red[wv * 9 + tid]) : sum + red[wv * 9 + tid];
            ((G<double> *)r.partials)[(size_t)te.tir * DIAGW + tid] = sum;
        }
    }
}

// Per-run reduction of the tile partials into one diagnostic record, in two launches
// with a fixed assignment of partials to threads and fixed-order combines (so the
// result is the same every run): level 1 sums FIN_CHUNK consecutive tile partials per
// block with compensated sums, level 2 combines the level-1 results of a run.
constexpr int FIN_CHUNK = 1024;

__device__ __forceinline__ void csum_add(double &s, double &c, double x)
{
    const double u = s + x;
    c += (fabs(s) >= fabs(x)) ? ((s - u) + x) : ((x - u) + s);
    s = u;
}

// sums (q != 7) or maxima (q == 7) of 9 values per item, over items [lo, hi)
// strided by blockDim, reduced through LDS in a fixed tree
template <int NTH>
__device__ __forceinline__ void block_reduce9(const G<double> *src, int lo, int hi, double (*sh)[10], double *out)
{
    const int t = threadIdx.x;
    double s[9], cmp[9];
#pragma unroll
    for (int q = 0; q < 9; q++) { s[q] = 0.0; cmp[q] = 0.0; }
    for (int i = lo + t; i < hi; i += NTH) {
        const G<double> *p = src + (size_t)i * DIAGW;
#pragma unroll
        for (int q = 0; q < 9; q++) {
            const double x = p[q];
            if (q == 7) s[q] = fmax(s[q], x);
            else csum_add(s[q], cmp[q], x);
        }
    }
#pragma unroll
    for (int q = 0; q < 9; q++) sh[t][q] = (q == 7) ? s[q] : s[q] + cmp[q];
    __syncthreads();
    for (int w = NTH / 2; w >= 1; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int q = 0; q < 9; q++) sh[t][q] = (q == 7) ? fmax(sh[t][q], sh[t + w][q]) : sh[t][q] + sh[t + w][q];
        }
        __syncthreads();
    }
    if (t < 9) out[t] = sh[0][t];
}

template <typename T>
__global__ void __launch_bounds__(256) k_finalize1(const RunDesc<T> *__restrict__ runs)
{
    const RunDesc<T> &r = runs[blockIdx.x];
    const int b = blockIdx.y;
    if (b >= r.nb2) return;
    __shared__ double sh[256][10];
    __shared__ double res[9];
    const int lo = b * FIN_CHUNK, hi = min(r.ntiles, lo + FIN_CHUNK);
    block_reduce9<256>((const G<double> *)r.partials, lo, hi, sh, res);
    __syncthreads();
    if (threadIdx.x < 9) ((G<double> *)r.partials2)[(size_t)b * DIAGW + threadIdx.x] = res[threadIdx.x];
}

template <typename T>
__global__ void __launch_bounds__(64) k_finalize2(const RunDesc<T> *__restrict__ runs, int step)
{
    const RunDesc<T> &r = runs[blockIdx.x];
    __shared__ double sh[64][10];
    __shared__ double res[9];
    block_reduce9<64>((const G<double> *)r.partials2, 0, r.nb2, sh, res);
    __syncthreads();
    if (threadIdx.x == 0) {
        const double n = (double)r.nx * (double)r.ny * (double)r.nz;
        G<double> *o = (G<double> *)r.records + (size_t)step * DREC;
        o[0] = r.step0 + (double)step;
        o[1] = (r.step0 + (double)step) * r.dt;  // one rounding: the same for any split into calls
        o[2] = 0.5 * res[0] / n;
        o[3] = 0.5 * res[2] / n;
        o[4] = sqrt(res[1] / n);
        o[5] = sqrt(res[0] / n);
        o[6] = sqrt(res[7]);
        o[7] = res[3] / n;
        o[8] = res[4] / n;
        o[9] = res[5] / n;
        o[10] = res[6] / n;
        o[11] = res[8];
        o[12] = (double)wall_clock64();  // constant-rate device clock: per-step latencies of a run
    }
}

// ------------------------------------------------------------------ seed field
// Counter-based use of SplitMix64 (Steele, Lea, Flood 2014): output i of stream
// (seed, sid) is mix(key + (i+1) * gamma) with key = mix(seed ^ mix(sid)).  The host
// uses the same functions for the forcing draws.
constexpr uint64_t SM_GAMMA = 0x9E3779B97F4A7C15ull;

__host__ __device__ inline uint64_t sm_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm_key(uint64_t seed, uint64_t sid) { return sm_mix(seed ^ sm_mix(sid)); }
__host__ __device__ inline double sm_unif(uint64_t key, uint64_t ctr)
{
    return (double)(sm_mix(key + (ctr + 1) * SM_GAMMA) >> 11) * (1.0 / 9007199254740992.0);
}

template <typename T>
struct SeedArgs {
    T *f[NF];          // the seven fields of the current buffer set
    uint64_t key[3];   // SplitMix64 keys of A_x, A_y, A_z (streams 100 + field index)
    double amp;
    uint64_t n;        // cells
};

// Initial state: ln rho = 0, u = 0, and each component of A Gaussian noise of standard
// deviation amp, cell i (x fastest) taking value i of its stream.  Counters 2p and 2p+1
// give the pair of cells 2p, 2p+1 by the Box-Muller transform, in FP64 and rounded
// once to T.  One thread per pair, grid-stride.
template <typename T>
__global__ void __launch_bounds__(256) k_seed(SeedArgs<T> a)
{
    const uint64_t npair = (a.n + 1) / 2;
    for (uint64_t pi = (uint64_t)blockIdx.x * 256 + threadIdx.x; pi < npair; pi += (uint64_t)gridDim.x * 256) {
        const uint64_t i0 = 2 * pi, i1 = i0 + 1;
        const bool two = i1 < a.n;
        for (int f = 0; f < 4; f++) {
            ((G<T> *)a.f[f])[i0] = T(0);
            if (two) ((G<T> *)a.f[f])[i1] = T(0);
        }
        for (int c = 0; c < 3; c++) {
            const double u1 = sm_unif(a.key[c], i0), u2 = sm_unif(a.key[c], i1);
            const double r = sqrt(-2.0 * log1p(-u1));
            const double z0 = a.amp * (r * cos(2.0 * M_PI * u2));
            const double z1 = a.amp * (r * sin(2.0 * M_PI * u2));
            ((G<T> *)a.f[4 + c])[i0] = (T)z0;
            if (two) ((G<T> *)a.f[4 + c])[i1] = (T)z1;
        }
    }
}

}  // namespace mhd
