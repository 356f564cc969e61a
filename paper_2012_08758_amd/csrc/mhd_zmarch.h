// z-marching substep kernel with register queues ("zm").
//
// A work-group owns a 32 x 8 column tile of one run and walks a z-segment of it one
// plane per step.  Each step brings one plane of each of the seven fields into LDS
// (the tile plus a 3-cell x/y halo, x wrapped while copying) by direct-to-LDS loads,
// two steps ahead of use, together with the s-2 state and the forcing phase of the
// plane being finished.  The z direction never goes through LDS:
//   * every thread keeps its own column's last six planes of its fields in registers
//     (the newest plane is the seventh), so the z first and second derivatives at the
//     plane three behind the newest come from registers;
//   * the mixed x-z and y-z derivatives (sixth-order diagonal stencils) are sums over
//     planes z +- s of x- (or y-) differences taken inside one plane, so each plane's
//     differences are pushed, with their weights, into accumulators of the six output
//     planes they reach (the +s part into plane z' - s, the -s part into z' + s);
//   * the parts of a cell's right-hand side that only need its own plane (x/y
//     derivatives and their products) are formed when the plane arrives and either
//     added to the same pending accumulators or held three steps until the z parts
//     are known.
// Output (the RK3 update of the plane three behind the newest) then needs only
// registers, so one plane of each field in LDS suffices.
//
// Threads 0..255 ("flow") carry ln rho and u of one column each, threads 256..511
// ("field") carry A of the same columns; at each output plane they swap u and J x B
// through LDS.  Register queues rotate with period six: the step loop is unrolled by
// six so that every queue slot is a compile-time index.
//
// Needs nx % 32 == 0, ny % 8 == 0 and 16-byte aligned field arrays (checked on the host).
#pragma once
#include "mhd_device.h"

namespace mhd {

template <typename T, int TXV = 32, bool ALLFV = sizeof(T) == 8>
struct ZmCfg {
    static constexpr int TX = TXV, TY = 8, NC = TX * TY;  // columns of a tile
    static constexpr int NT = 2 * NC;                      // flow + field threads
    static constexpr int NW = NT / 64;                     // waves
    static constexpr int EPL = 16 / (int)sizeof(T);        // values per 16-byte copy
    static constexpr int XW = TX + 8, YW = TY + 6;         // plane box (x from x0-4)
    static constexpr int PLE = XW * YW;                    // values per field plane
    static constexpr int PV = PLE / EPL;                   // copies per field plane
    // one step's planes: ln rho and u (read by flow threads) and A (field threads) land
    // in separate regions, whole wave-copies each
    static constexpr int NIF = (4 * PV + 63) / 64, NIA = (3 * PV + 63) / 64;
    // ALLF (FP64, and the kernels with the diagnostics, see Zm::C): the flow threads
    // issue every copy of a step, the field threads none, so that the field waves (the
    // longer path to the exchange barrier) start their output at once while the copies
    // still leave at the top of the step (512^3: FP64 diagnostics substep 5.10 -> 4.98
    // ms, step 16.5 -> 16.3 ms; FP32 diagnostics substep 3.80 -> 3.46 ms).  FP32
    // substeps 2 and 3 measured 5-9 % slower with it: there every wave issues, the
    // field waves after their stores (Zm::LATE).
    static constexpr bool ALLF = ALLFV;
    static constexpr int NWI = ALLF ? NW / 2 : NW, NTI = 64 * NWI;  // waves, threads that issue copies
    static constexpr int NLP = (NIF + NIA + NWI - 1) / NWI;  // plane copies per issuing thread per step
    static constexpr int FREG = NIF * 64 * EPL, AREG = NIA * 64 * EPL;  // values per slot
    static constexpr int SV = NF * NC / EPL;               // copies of the s-2 state per step
    static constexpr int NLS = (SV + 1 + NTI - 1) / NTI;   // ... plus the forcing z slot
    static constexpr int SREG = NLS * NTI * EPL;
    static constexpr int D = 3;                            // slots: planes in flight + the one in use
    static constexpr int FLOW = 0;                         // D flow regions
    static constexpr int FIELD = FLOW + D * FREG;          // D field regions
    static constexpr int S2 = FIELD + D * AREG;            // D s-2 regions (+ forcing z slot)
    // FP32: the exchange of a step is consumed one step later (two slots, by step
    // parity), so that a step holds one barrier; FP64 keeps a barrier of its own for it
    // (512^3 substeps, FP32: 10.3 -> 9.7 ms per step; FP64 with the deferral: 5.9 ->
    // 6.2 ms for substep 2, so not there)
    static constexpr bool DEFER = sizeof(T) == 4;
    static constexpr int NXJ = DEFER ? 2 : 1;
    static constexpr int XJ = S2 + D * SREG;               // exchange: rho^-1 J x B + f [NXJ][3][NC]
    static constexpr int FH = XJ + NXJ * 3 * NC;           // forcing head and the tile's x, y phase slots
    static constexpr int NFH = FHEAD / EPL + TX + TY;
    static constexpr int NFHC = (NFH + 63) / 64;           // wave-copies of the forcing slots
    static constexpr int LDS = FH + NFHC * 64 * EPL;
    static_assert(PLE % EPL == 0 && XW % EPL == 0, "plane rows hold whole vectors");
    static_assert(NFHC <= 2, "forcing slots: at most two copies");
    static_assert(NC % 64 == 0, "flow and field threads fill whole waves");
    // every LDS read of a thread is an immediate offset (< 64 KiB) from one base
    static_assert((D * FREG + 6 * XW) * (int)sizeof(T) < 65536 && (D * AREG + 6 * XW) * (int)sizeof(T) < 65536 &&
                      (D * SREG) * (int)sizeof(T) < 65536,
                  "regions within 16-bit LDS offsets");
};

// LDS pointers keep their address space through the asm barriers below (a generic
// pointer there would turn every LDS read into a flat load)
template <typename T>
using LP = __attribute__((address_space(3))) T;

// LDS reads of the stencils.  FP64 values are read one by one (ds_read_b64 at a 16-bit
// immediate offset from the step's base): left to itself the compiler merges pairs into
// ds_read2_b64, whose 8-bit offsets need a fresh base VGPR (one v_add per pair) across
// fields and rows, 23-29 extra VALU operations per plane; the volatile reads keep them
// apart (512^3 substep 2: 6.27 -> 5.77 ms).  FP32 keeps the merged reads: its kernels
// issue four waves per SIMD and are VALU-bound, and there the doubled LDS issue cost more
// than the adds (3.17 -> 3.21 ms).
template <class PT>
__device__ __forceinline__ auto ldv(const PT *p)
{
    if constexpr (sizeof(*p) == 8)
        return *(const volatile PT *)p;
    else
        return *p;
}

// One field's plane box in LDS, addressed relative to this thread's column (offsets
// -CO .. CO, CO = 3 rows + 3 columns).  FP32 reads go through two opaque bases, the box
// origin for negative offsets and the column for the others, so that every pair the
// compiler merges into ds_read2_b32 (two 8-bit dword offsets from one base) finds its
// base among these two: without them it adds a fresh base per pair (about 25 extra
// integer operations per plane, 4 % of the substep's VALU work).  FP64 reads stay one
// by one at 16-bit offsets from the step's single base.
template <typename T, int CO>
struct Box {
    const LP<T> *lo, *hi;
    __device__ __forceinline__ explicit Box(const LP<T> *col) : lo(col - CO), hi(col)
    {
        if constexpr (sizeof(T) == 4) asm volatile("" : "+v"(lo), "+v"(hi));
    }
    __device__ __forceinline__ T operator[](int o) const { return o < 0 ? ldv(lo + (o + CO)) : ldv(hi + o); }
};

// Wait until at most n vector-memory operations of this wave are outstanding (n is
// wave-uniform; the immediate of s_waitcnt is picked by a switch; any n above 31 waits
// for all), then for the LDS, then for the work-group.
__device__ __forceinline__ void zm_wait(int n)
{
    __builtin_amdgcn_sched_barrier(0);
    switch (n) {
#define ZM_W(c) \
    case c: wait_vmcnt<c>(); break;
        ZM_W(1) ZM_W(2) ZM_W(3) ZM_W(4) ZM_W(5) ZM_W(6) ZM_W(7) ZM_W(8)
        ZM_W(9) ZM_W(10) ZM_W(11) ZM_W(12) ZM_W(13) ZM_W(14) ZM_W(15) ZM_W(16)
        ZM_W(17) ZM_W(18) ZM_W(19) ZM_W(20) ZM_W(21) ZM_W(22) ZM_W(23) ZM_W(24)
        ZM_W(25) ZM_W(26) ZM_W(27) ZM_W(28) ZM_W(29) ZM_W(30) ZM_W(31)
#undef ZM_W
    default: wait_vmcnt<0>(); break;
    }
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// Sums of the three symmetric pairs along one direction: p_s = f(+s) + f(-s) and the
// differences d_s = f(+s) - f(-s), s = 1..3, at stride st from s[0].
template <typename T>
struct Pairs {
    T c, p[3], d[3];
    template <class B>
    __device__ __forceinline__ void load(const B &s, int st)
    {
        c = s[0];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const T a = s[(k + 1) * st], b = s[-(k + 1) * st];
            p[k] = a + b;
            d[k] = a - b;
        }
    }
    __device__ __forceinline__ T d1(T ih) const { return ih * (T(W1_1) * d[0] + T(W1_2) * d[1] + T(W1_3) * d[2]); }
    // with the weights already divided by the spacing (one multiply fewer)
    __device__ __forceinline__ T d1w(const T (&w)[3]) const { return w[0] * d[0] + w[1] * d[1] + w[2] * d[2]; }
    __device__ __forceinline__ T d2w(const T (&w)[4]) const { return w[0] * c + w[1] * p[0] + w[2] * p[1] + w[3] * p[2]; }
    __device__ __forceinline__ T d2(T ih2) const
    {
        return ih2 * (T(W2_0) * c + T(W2_1) * p[0] + T(W2_2) * p[1] + T(W2_3) * p[2]);
    }
    __device__ __forceinline__ T d6() const { return T(-20) * c + T(15) * p[0] + T(-6) * p[1] + p[2]; }
};

// acc + d_x d_y from the two diagonals through s[0] (rows of stride sy); w = the
// diagonal weights divided by 4 h_x h_y (times the role's factor)
template <typename T, class B>
__device__ __forceinline__ T zm_dxy(T acc, const B &s, int sy, const T (&w)[3])
{
    const int p = 1 + sy, q = 1 - sy;
#pragma unroll
    for (int k = 1; k <= 3; k++) acc = fma(w[k - 1], (s[k * p] + s[-k * p]) - (s[k * q] + s[-k * q]), acc);
    return acc;
}

// in-plane stencil weights divided by the spacings, read once and pinned in scalar
// registers; the mixed-derivative weights are those of the thread's role (the flow
// role's carry the nu / 3 of the viscous term)
template <typename T>
struct ZmWts {
    T w1x[3], w1y[3], w2x[4], w2y[4], wm[3], qx[3], qy[3];
    __device__ __forceinline__ void load(const Coef<T> &c, int role)
    {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            w1x[k] = c.w1[0][k];
            w1y[k] = c.w1[1][k];
            wm[k] = c.wm[role][k];
            qx[k] = c.wq[role][0][k];
            qy[k] = c.wq[role][1][k];
            asm volatile("" : "+s"(w1x[k]), "+s"(w1y[k]), "+s"(wm[k]), "+s"(qx[k]), "+s"(qy[k]));
        }
#pragma unroll
        for (int k = 0; k < 4; k++) {
            w2x[k] = c.w2[0][k];
            w2y[k] = c.w2[1][k];
            asm volatile("" : "+s"(w2x[k]), "+s"(w2y[k]));
        }
    }
};

// z derivatives at the output plane from a register queue: q[(j + i) % 6] holds the
// plane z' - 6 + i' ... see the callers; here v[0..6] = planes zo-3 .. zo+3.
template <typename T>
struct ZCol {
    T v[7];
    __device__ __forceinline__ T d1(T ih) const
    {
        return ih * (T(W1_1) * (v[4] - v[2]) + T(W1_2) * (v[5] - v[1]) + T(W1_3) * (v[6] - v[0]));
    }
    __device__ __forceinline__ T d2(T ih2) const
    {
        return ih2 * (T(W2_0) * v[3] + T(W2_1) * (v[4] + v[2]) + T(W2_2) * (v[5] + v[1]) + T(W2_3) * (v[6] + v[0]));
    }
    __device__ __forceinline__ double d1d(double ih) const
    {
        return ih * (W1_1 * ((double)v[4] - (double)v[2]) + W1_2 * ((double)v[5] - (double)v[1]) +
                     W1_3 * ((double)v[6] - (double)v[0]));
    }
    __device__ __forceinline__ T d6() const
    {
        return T(-20) * v[3] + T(15) * (v[4] + v[2]) + T(-6) * (v[5] + v[1]) + (v[6] + v[0]);
    }
};

// queue slot of the plane `back` steps behind the newest (0 = newest, held apart)
template <int J, int BACK>
struct QS {
    static constexpr int v = ((J - BACK) % 6 + 6) % 6;
};

// the seven planes zo-3 .. zo+3 of one queue (newest plane in `now`)
template <typename T, int J>
__device__ __forceinline__ ZCol<T> zcol(const T (&q)[6], T now)
{
    ZCol<T> z;
    z.v[0] = q[QS<J, 6>::v];
    z.v[1] = q[QS<J, 5>::v];
    z.v[2] = q[QS<J, 4>::v];
    z.v[3] = q[QS<J, 3>::v];
    z.v[4] = q[QS<J, 2>::v];
    z.v[5] = q[QS<J, 1>::v];
    z.v[6] = now;
    return z;
}

// pending-accumulator slot of the output plane z' + off (z' = the newest plane)
template <int J, int OFF>
struct PS {
    static constexpr int v = ((J + 3 + OFF) % 6 + 6) % 6;
};

// Push the mixed-derivative contributions q_s (s = 1..3) of the newest plane z': + into
// the output plane z' - s, - into z' + s.  The s = 3 '+' part completes the current
// output plane and is added before it is finished; the s = 3 '-' part starts the
// accumulator of plane z' + 3, which takes over the slot the output just released, so
// it is subtracted there; the caller cleared that slot after the output.
// q_s = w_s d_s: one fused multiply-add per target plane.
template <typename T, int J>
__device__ __forceinline__ void push3(T (&acc)[6], const T (&d)[3], const T (&w)[3])
{
    acc[PS<J, -1>::v] = fma(w[0], d[0], acc[PS<J, -1>::v]);
    acc[PS<J, 1>::v] = fma(-w[0], d[0], acc[PS<J, 1>::v]);
    acc[PS<J, -2>::v] = fma(w[1], d[1], acc[PS<J, -2>::v]);
    acc[PS<J, 2>::v] = fma(-w[1], d[1], acc[PS<J, 2>::v]);
    acc[PS<J, 3>::v] = fma(-w[2], d[2], acc[PS<J, 3>::v]);
}

template <typename T, int SUB, bool DIAG, bool STORE, bool UPW, int TXV>
struct Zm {
    using C = ZmCfg<T, TXV, sizeof(T) == 8 || DIAG>;
    static constexpr int NLS_E = STORE ? (SUB == 0 ? 1 : C::NLS) : 0;  // s-2 / forcing copies per step
    static constexpr int NL = C::NLP + NLS_E;                         // copies per step per thread
    static constexpr int NSF = STORE ? 4 : 0, NSA = STORE ? 3 : 0;     // stores per output (flow, field)
    static constexpr int FZ = SUB == 0 ? 0 : C::SV * C::EPL;  // forcing z slot within an s-2 region
    static_assert(NL + 2 * NSF <= 31, "the waits of a step cover at most 31 operations");
    // copies a thread of the role issues per step
    template <int ROLE>
    __host__ __device__ static constexpr int nl()
    {
        return (C::ALLF && ROLE == 1) ? 0 : NL;
    }
    // A field thread issues its copies of a step after its output stores (below) in the
    // FP32 kernels without ALLF: with all waves issuing at once the last in line (the
    // field waves) fell about a quarter of the step behind (512^3 substep 2: 3.22 ->
    // 2.66 ms).  FP64 measured faster with the early issue.
    static constexpr bool LATE = sizeof(T) == 4 && !C::ALLF;
    // stores of a thread at step j (output plane j - 6; a flow thread with the deferred
    // exchange stores ln rho alone at its first output step and u of the previous plane
    // with every later one)
    template <int ROLE>
    __host__ __device__ static constexpr int stores(int j)
    {
        if (j < 6) return 0;
        if (ROLE == 0) return (C::DEFER && j == 6) ? (STORE ? 1 : 0) : NSF;
        return NSA;
    }
    // operations a thread issues after the copies of plane k, up to the wait of step k:
    // in a step a thread issues copies then stores (a field thread with LATE: stores
    // then copies); plane k's copies are issued at step k - 2 (planes 0 and 1 before the
    // loop)
    template <int ROLE>
    __host__ __device__ static constexpr int after(int k, int K)
    {
        const int next = k + 1 < K ? nl<ROLE>() : 0;
        if (ROLE == 1 && LATE) return next + stores<1>(k - 1);
        return stores<ROLE>(k - 2) + next + stores<ROLE>(k - 1);
    }
    // Replays a thread's operations in issue order for every step count K up to KMAX and
    // checks that after() is, at each step k, the number issued after plane k's copies
    // and before the wait (checked at compile time below).
    template <int ROLE>
    __host__ __device__ static constexpr bool after_exact(int KMAX)
    {
        constexpr bool late = ROLE == 1 && LATE;
        for (int K = 1; K <= KMAX; K++) {
            constexpr int n = nl<ROLE>();
            int end[64] = {}, issued = 0;  // end[p]: operations issued up to plane p's copies
            end[0] = issued += n;
            if (K > 1) end[1] = issued += n;
            for (int k = 0; k < K; k++) {
                if (issued - end[k] != after<ROLE>(k, K)) return false;
                if (!late && k + 2 < K) end[k + 2] = issued += n;
                issued += stores<ROLE>(k);
                if (late && k + 2 < K) end[k + 2] = issued += n;
            }
        }
        return true;
    }
    static_assert(after_exact<0>(40) && after_exact<1>(40), "vmcnt accounting of a step");
};

// substep constants of the update and the imposed field, read once and pinned in
// scalar registers
template <typename T>
struct ZmK {
    T bdt, brho, bext[3];
    ZmWts<T> w;
    __device__ __forceinline__ void load(const Coef<T> &c, int sub, int role)
    {
        w.load(c, role);
        bdt = c.bdt[sub];
        brho = c.brho[sub];
#pragma unroll
        for (int a = 0; a < 3; a++) bext[a] = c.bext[a];
        asm volatile("" : "+s"(bdt), "+s"(brho), "+s"(bext[0]), "+s"(bext[1]), "+s"(bext[2]));
    }
};

// Register state of one thread.  A flow thread and a field thread of a column keep
// the same layout (so that the kernel needs registers for one of them, not both):
//   q:   last six planes of the thread's fields (ln rho, u_x, u_y, u_z / A_x, A_y, A_z),
//        slot = step mod 6;
//   acc: pending right-hand sides of u (flow) / current density (field) of the six
//        output planes still open, slot = output step mod 6;
//   del: per plane (slot = step mod 3) what the plane's output still needs when its z
//        parts exist:
//        flow  g_x, g_y, d_x u_z, d_y u_z, div_xy u, R_lnrho part;
//        field d_y A_z, -d_x A_z, d_x A_y - d_y A_x, eta (D2x + D2y) A_m, and the flow
//              values ln rho, u_x, u_y, u_z at the column (for rho^-1 J x B, u x B and the
//              diagnostics, which the field thread of a column takes on).
template <typename T>
struct ZmState {
    T q[4][6];
    T acc[3][6];
    T del[10][3];
    T fpr, fpi;       // field: forcing exp(i (k_x x + k_y y)) at the column
    T pend[3];        // flow, deferred exchange: the last output plane's new u, still without
                      // dt beta rho^-1 J x B + f
    double dg[9];     // diagnostics in the order of the per-tile partials: |B|^2, |u|^2, rho |u|^2,
                      // ln rho, B_x, B_y, B_z, max |u|^2, non-finite cells; a flow thread sums the
                      // u and ln rho terms, a field thread the B terms and the non-finite count
                      // (it holds all seven values of its cell)
    double bd[3][3];  // diagnostics of FP32 runs, field: the B parts of del in FP64
};

// first derivative in FP64 of FP32 values in LDS (diagnostics of FP32 runs)
template <class B>
__device__ __forceinline__ double zm_d1d(const B &s, int st, double ih)
{
    return ih * (W1_1 * ((double)s[st] - (double)s[-st]) + W1_2 * ((double)s[2 * st] - (double)s[-2 * st]) +
                 W1_3 * ((double)s[3 * st] - (double)s[-3 * st]));
}


// One step of the march: wait for the newest plane z' (step k), request the plane two
// steps ahead, finish the output plane z' - 3 (k >= 6), then fold plane z' into the
// register queues and pending accumulators.  J = k mod 6 fixes every queue slot;
// Complete a flow thread's pending output plane: add dt beta (rho^-1 J x B + f), which
// the field thread of the column left in exchange slot xp, and store u.
template <typename T, int NC>
__device__ __forceinline__ void zm_flush(const T (&pend)[3], const LP<T> *xp, const RunDesc<T> &r, int out_set,
                                         uint64_t zb, uint32_t gcb, T bdt)
{
#pragma unroll
    for (int m = 0; m < 3; m++) *(G<T> *)((G<char> *)r.buf[out_set][1 + m] + zb + gcb) = pend[m] + bdt * xp[m * NC];
}

// ROLE 0 is a flow thread, 1 a field thread.
template <typename T, int SUB, bool DIAG, bool STORE, bool UPW, int TXV, int ROLE, int J, class KR, class ISSUE>
__device__ __forceinline__ void zm_body(int k, int K, T *lds, ZmState<T> &S, const KR &Kr, const ZmK<T> &Zk,
                                        const DCoef &dc, const RunDesc<T> &r, LP<T> *&pb0, LP<T> *&sb0, LP<T> *&xb0, LP<T> *&cf0, int col,
                                        uint32_t gcb, uint64_t plane_b, int zs, int out_set, T (&fa)[3], T (&fb)[3],
                                        bool &fon, ISSUE &issue)
{
    using Z = Zm<T, SUB, DIAG, STORE, UPW, TXV>;
    using C = typename Z::C;
    constexpr int NC = C::NC, PLE = C::PLE, XW = C::XW;
    constexpr int JD = J % 3;                       // delayed-set slot of plane z'
    constexpr int PO = PS<J, -3>::v;                // pending slot of the output plane (= J)
    constexpr int PN = PS<J, 0>::v;                 // pending slot of plane z' itself
    if (k >= K) return;
    zm_wait(Z::template after<ROLE>(k, K));
    // the copies of plane k + 2, into the slot plane k - 1 left (see Zm::LATE)
    constexpr bool LATE = ROLE == 1 && Z::LATE, ISSUES = !(C::ALLF && ROLE == 1);
    if (ISSUES && !LATE && k + 2 < K) issue(k + 2, (J + 2) % 3);
    // this thread's planes (pb0 points 3 rows and 3 columns before its column in slot 0
    // of its role's region), s-2 values and exchange slots; the asm keeps the compiler
    // from hoisting addresses derived from them out of the step loop
    asm volatile("" : "+v"(pb0), "+v"(sb0), "+v"(xb0), "+v"(cf0), "+v"(gcb));
    constexpr int CO = 3 * XW + 3;
    const LP<T> *P = pb0 + JD * (ROLE == 0 ? C::FREG : C::AREG) + CO;  // P[f * PLE] = field f of the role at the column
    const LP<T> *S2 = sb0 + JD * C::SREG;                               // S2[f * NC] = s-2 value of field f
    const bool out = k >= 6;
    const int zo = zs + k - 6;

    if constexpr (STORE) {
        if (k == 0) {  // forcing head and this column's x/y phase product (arrived with plane 0)
            constexpr int HV = FHEAD / C::EPL;
            const T *H = lds + C::FH;
            fon = H[6] != T(0);
#pragma unroll
            for (int a = 0; a < 3; a++) { fa[a] = H[a]; fb[a] = H[3 + a]; }
            const int cx = col % C::TX, cy = col / C::TX;
            const T *ex = H + (HV + cx) * C::EPL, *ey = H + (HV + C::TX + cy) * C::EPL;
            S.fpr = ex[0] * ey[0] - ex[1] * ey[1];
            S.fpi = ex[0] * ey[1] + ex[1] * ey[0];
        }
    }

    // ---------------------------------------------------------------- output plane
    // the newest plane's centre values and the s = 3 differences that complete it
    T now[4];
    // the role's fields in this step's slot (flow: ln rho, u_x, u_y, u_z; field: A)
    using Bx = Box<T, CO>;
    const Bx F0(P), F1(P + PLE), F2(P + 2 * PLE), F3(P + (ROLE == 0 ? 3 : 2) * PLE);
    if constexpr (ROLE == 0) {
        const Bx &X = F1, &Y = F2, &W = F3;
        now[0] = F0[0];
        now[1] = X[0];
        now[2] = Y[0];
        now[3] = W[0];
        if constexpr (STORE) {
            const T k3x = Zk.w.qx[2], k3y = Zk.w.qy[2];
            S.acc[0][PO] = fma(k3x, W[3] - W[-3], S.acc[0][PO]);
            S.acc[1][PO] = fma(k3y, W[3 * XW] - W[-3 * XW], S.acc[1][PO]);
            S.acc[2][PO] = fma(k3y, Y[3 * XW] - Y[-3 * XW], fma(k3x, X[3] - X[-3], S.acc[2][PO]));
        }
    } else {
        const Bx &AX = F0, &AY = F1, &AZ = F2;
        now[0] = AX[0];
        now[1] = AY[0];
        now[2] = AZ[0];
        now[3] = T(0);
        if constexpr (STORE) {
            const T k3x = Zk.w.qx[2], k3y = Zk.w.qy[2];
            S.acc[0][PO] = fma(k3x, AZ[3] - AZ[-3], S.acc[0][PO]);
            S.acc[1][PO] = fma(k3y, AZ[3 * XW] - AZ[-3 * XW], S.acc[1][PO]);
            S.acc[2][PO] = fma(k3y, AY[3 * XW] - AY[-3 * XW], fma(k3x, AX[3] - AX[-3], S.acc[2][PO]));
        }
    }

    // The field thread of a column forms rho^-1 J x B + f (it holds ln rho and u of the
    // output plane, see del) and hands it to the flow thread through LDS.  Deferred
    // (C::DEFER): in the slot of this step's parity, and the flow thread completes that
    // plane's u one step later, after the barrier that opens the next step; otherwise
    // behind a barrier of this step.
    LP<T> *XJ = xb0 + (C::DEFER ? (J & 1) * 3 * NC : 0);  // XJ[m * NC]: component m at the column
    if (out) {
        const T ihz = Kr.ih1[2], ih2z = Kr.ih2[2];
        if constexpr (ROLE == 0) {
            const ZCol<T> L = zcol<T, J>(S.q[0], now[0]), X = zcol<T, J>(S.q[1], now[1]);
            const ZCol<T> Y = zcol<T, J>(S.q[2], now[2]), W = zcol<T, J>(S.q[3], now[3]);
            if constexpr (DIAG) {
                const double lz = (double)L.v[3], dx = (double)X.v[3], dy = (double)Y.v[3], dz = (double)W.v[3];
                const double u2 = dx * dx + dy * dy + dz * dz;
                S.dg[1] += u2;
                S.dg[2] += exp(lz) * u2;
                S.dg[3] += lz;
                S.dg[7] = fmax(S.dg[7], u2);
            }
            if constexpr (STORE) {
                const T l0 = L.v[3], ux = X.v[3], uy = Y.v[3], uz = W.v[3];
                const T gz = L.d1(ihz), dzx = X.d1(ihz), dzy = Y.d1(ihz), dzz = W.d1(ihz);
                const T gx = S.del[0][JD], gy = S.del[1][JD], dxz = S.del[2][JD], dyz = S.del[3][JD];
                const T divxy = S.del[4][JD], pl = S.del[5][JD];
                const T nu = Kr.nu, n23 = Kr.nu2_3;
                T R[4];
                R[0] = pl - uz * gz - dzz;
                if constexpr (UPW) R[0] += Kr.upw[2] * fabs(uz) * L.d6();
                R[1] = S.acc[0][PO] + nu * X.d2(ih2z) - uz * dzx + nu * (dzx * gz + dxz * gz) - n23 * dzz * gx;
                R[2] = S.acc[1][PO] + nu * Y.d2(ih2z) - uz * dzy + nu * (dzy * gz + dyz * gz) - n23 * dzz * gy;
                R[3] = S.acc[2][PO] + (nu + Kr.nu3) * W.d2(ih2z) - uz * dzz +
                       nu * (T(2) * dzz * gz + dzx * gx + dzy * gy) - n23 * (divxy + dzz) * gz - Kr.cs2 * gz;
                const T bdt = Zk.bdt, brho = Zk.brho;
                if constexpr (C::DEFER) {
                    if (k >= 7)  // the previous step's output plane, with its exchange
                        zm_flush<T, NC>(S.pend, xb0 + ((J + 1) & 1) * 3 * NC, r, out_set, (uint64_t)(zo - 1) * plane_b,
                                        gcb, bdt);
                } else {
                    lds_barrier();  // rho^-1 J x B + f of the column is in XJ
                    R[1] += XJ[0];
                    R[2] += XJ[NC];
                    R[3] += XJ[2 * NC];
                }
                const T v[4] = {l0, ux, uy, uz};
                T o[4];
#pragma unroll
                for (int f = 0; f < 4; f++) {
                    if constexpr (SUB == 0) {
                        o[f] = v[f] + bdt * R[f];
                    } else {
                        const T old = S2[f * NC];
                        o[f] = v[f] + brho * (v[f] - old) + bdt * R[f];
                    }
                }
                const uint64_t zb = (uint64_t)zo * plane_b;
#pragma unroll
                for (int f = 0; f < 4; f++) {
                    if (C::DEFER && f > 0) S.pend[f - 1] = o[f];
                    else *(G<T> *)((G<char> *)r.buf[out_set][f] + zb + gcb) = o[f];
                }
            }
        } else {
            const ZCol<T> AX = zcol<T, J>(S.q[0], now[0]), AY = zcol<T, J>(S.q[1], now[1]);
            const ZCol<T> AZ = zcol<T, J>(S.q[2], now[2]);
            const T l0 = S.del[6][JD], ux = S.del[7][JD], uy = S.del[8][JD], uz = S.del[9][JD];
            const T dzax = AX.d1(ihz), dzay = AY.d1(ihz);
            const T bx = Zk.bext[0] + S.del[0][JD] - dzay, by = Zk.bext[1] + dzax + S.del[1][JD];
            const T bz = Zk.bext[2] + S.del[2][JD];
            if constexpr (STORE) {
                const T jx = S.acc[0][PO] - AX.d2(ih2z);
                const T jy = S.acc[1][PO] - AY.d2(ih2z);
                const T jz = S.acc[2][PO];
                const T rinv = exp(-l0);
                T f[3] = {T(0), T(0), T(0)};
                if (fon) {
                    const T *Ez = lds + C::S2 + JD * C::SREG + Z::FZ;
                    const T cr = S.fpr * Ez[0] - S.fpi * Ez[1], ci = S.fpr * Ez[1] + S.fpi * Ez[0];
#pragma unroll
                    for (int a = 0; a < 3; a++) f[a] = fa[a] * cr + fb[a] * ci;
                }
                XJ[0] = rinv * (jy * bz - jz * by) + f[0];
                XJ[NC] = rinv * (jz * bx - jx * bz) + f[1];
                XJ[2 * NC] = rinv * (jx * by - jy * bx) + f[2];
                const T eta = Kr.eta;
                T R[3];
                R[0] = S.del[3][JD] + eta * AX.d2(ih2z) + (uy * bz - uz * by);
                R[1] = S.del[4][JD] + eta * AY.d2(ih2z) + (uz * bx - ux * bz);
                R[2] = S.del[5][JD] + eta * AZ.d2(ih2z) + (ux * by - uy * bx);
                const T bdt = Zk.bdt, brho = Zk.brho;
                const uint64_t zb = (uint64_t)zo * plane_b;
#pragma unroll
                for (int m = 0; m < 3; m++) {
                    const T vv = m == 0 ? AX.v[3] : (m == 1 ? AY.v[3] : AZ.v[3]);
                    T o;
                    if constexpr (SUB == 0) {
                        o = vv + bdt * R[m];
                    } else {
                        const T old = S2[(4 + m) * NC];
                        o = vv + brho * (vv - old) + bdt * R[m];
                    }
                    *(G<T> *)((G<char> *)r.buf[out_set][4 + m] + zb + gcb) = o;
                }
            }
            if constexpr (DIAG) {
                double Bx, By, Bz;
                if constexpr (sizeof(T) == 8) {
                    Bx = (double)bx;
                    By = (double)by;
                    Bz = (double)bz;
                } else {
                    Bx = dc.bext[0] + S.bd[0][JD] - AY.d1d(dc.ih1[2]);
                    By = dc.bext[1] + AX.d1d(dc.ih1[2]) + S.bd[1][JD];
                    Bz = dc.bext[2] + S.bd[2][JD];
                }
                S.dg[0] += Bx * Bx + By * By + Bz * Bz;
                S.dg[4] += Bx;
                S.dg[5] += By;
                S.dg[6] += Bz;
                const bool ok = finite_v(l0) && finite_v(ux) && finite_v(uy) && finite_v(uz) && finite_v(AX.v[3]) &&
                                finite_v(AY.v[3]) && finite_v(AZ.v[3]);
                S.dg[8] += ok ? 0.0 : 1.0;
            }
            if constexpr (STORE && !C::DEFER) lds_barrier();  // XJ written
        }
    }

    if (ISSUES && LATE && k + 2 < K) issue(k + 2, (J + 2) % 3);

    // ---------------------------------------------------------------- fold in plane z'
    // The output plane's slots are free now: they start the accumulators of plane z' + 3.
    if constexpr (STORE) {
#pragma unroll
        for (int m = 0; m < 3; m++) S.acc[m][PO] = T(0);
    }
    // Field by field, so that few values are live at once: each field's x/y pairs give
    // its in-plane derivatives, which go straight into the accumulators, and its x- or
    // y-differences, pushed as mixed x-z / y-z derivatives into the planes z' +- s.
    if constexpr (ROLE == 0) {
        const Bx &L0 = F0, &X = F1, &Y = F2, &W = F3;
        if constexpr (STORE) {
            const T nu = Kr.nu, nu3 = Kr.nu3, n23 = Kr.nu2_3;
            const T ux = now[1], uy = now[2];
            T gx, gy, pl;
            {
                Pairs<T> lx, ly;
                lx.load(L0, 1);
                ly.load(L0, XW);
                gx = lx.d1w(Zk.w.w1x);
                gy = ly.d1w(Zk.w.w1y);
                pl = -(ux * gx + uy * gy);
                if constexpr (UPW) pl += Kr.upw[0] * fabs(ux) * lx.d6() + Kr.upw[1] * fabs(uy) * ly.d6();
            }
            // u_x: R_x (viscous, advection, strain), R_y (grad div), R_z (mixed push)
            T dxx, dyx;
            {
                Pairs<T> a, b;
                a.load(X, 1);
                b.load(X, XW);
                dxx = a.d1w(Zk.w.w1x);
                dyx = b.d1w(Zk.w.w1y);
                const T d2xx = a.d2w(Zk.w.w2x), d2yx = b.d2w(Zk.w.w2y);
                S.acc[0][PN] += nu * (d2xx + d2yx) + nu3 * d2xx - (ux * dxx + uy * dyx) + nu * (T(2) * dxx * gx + dyx * gy) -
                                Kr.cs2 * gx;
                S.acc[1][PN] = zm_dxy(S.acc[1][PN], X, XW, Zk.w.wm);
                push3<T, J>(S.acc[2], a.d, Zk.w.qx);
            }
            // u_y
            T dyy;
            {
                Pairs<T> a, b;
                a.load(Y, 1);
                b.load(Y, XW);
                const T dxy = a.d1w(Zk.w.w1x);
                dyy = b.d1w(Zk.w.w1y);
                const T d2xy = a.d2w(Zk.w.w2x), d2yy = b.d2w(Zk.w.w2y);
                S.acc[1][PN] += nu * (d2xy + d2yy) + nu3 * d2yy - (ux * dxy + uy * dyy) + nu * (dxy * gx + T(2) * dyy * gy) +
                                nu * dyx * gx - Kr.cs2 * gy;
                S.acc[0][PN] = zm_dxy(S.acc[0][PN] + nu * dxy * gy, Y, XW, Zk.w.wm);
                push3<T, J>(S.acc[2], b.d, Zk.w.qy);
            }
            const T divxy = dxx + dyy;
            S.acc[0][PN] -= n23 * divxy * gx;
            S.acc[1][PN] -= n23 * divxy * gy;
            pl -= divxy;
            // u_z
            {
                Pairs<T> a, b;
                a.load(W, 1);
                b.load(W, XW);
                const T dxz = a.d1w(Zk.w.w1x), dyz = b.d1w(Zk.w.w1y);
                S.acc[2][PN] += nu * (a.d2w(Zk.w.w2x) + b.d2w(Zk.w.w2y)) - (ux * dxz + uy * dyz) + nu * (dxz * gx + dyz * gy);
                push3<T, J>(S.acc[0], a.d, Zk.w.qx);
                push3<T, J>(S.acc[1], b.d, Zk.w.qy);
                S.del[2][JD] = dxz;
                S.del[3][JD] = dyz;
            }
            S.del[0][JD] = gx;
            S.del[1][JD] = gy;
            S.del[4][JD] = divxy;
            S.del[5][JD] = pl;
        }
#pragma unroll
        for (int f = 0; f < 4; f++) S.q[f][J] = now[f];
    } else {
        const Bx &AX = F0, &AY = F1, &AZ = F2;
        if constexpr (STORE) {
            const T eta = Kr.eta;
            T dyax;
            {  // A_x: j_x -= D2y A_x, j_y += D_xy A_x, j_z += D_xz A_x (push), B_z -= d_y A_x
                Pairs<T> a, b;
                a.load(AX, 1);
                b.load(AX, XW);
                const T d2x = a.d2w(Zk.w.w2x), d2y = b.d2w(Zk.w.w2y);
                dyax = b.d1w(Zk.w.w1y);
                S.acc[0][PN] -= d2y;
                S.acc[1][PN] = zm_dxy(S.acc[1][PN], AX, XW, Zk.w.wm);
                S.del[3][JD] = eta * (d2x + d2y);
                push3<T, J>(S.acc[2], a.d, Zk.w.qx);
            }
            {  // A_y: j_y -= D2x A_y, j_x += D_xy A_y, j_z += D_yz A_y (push), B_z += d_x A_y
                Pairs<T> a, b;
                a.load(AY, 1);
                b.load(AY, XW);
                const T d2x = a.d2w(Zk.w.w2x), d2y = b.d2w(Zk.w.w2y);
                S.del[2][JD] = a.d1w(Zk.w.w1x) - dyax;
                S.acc[1][PN] -= d2x;
                S.acc[0][PN] = zm_dxy(S.acc[0][PN], AY, XW, Zk.w.wm);
                S.del[4][JD] = eta * (d2x + d2y);
                push3<T, J>(S.acc[2], b.d, Zk.w.qy);
            }
            {  // A_z: j_z -= D2x A_z + D2y A_z, j_x += D_xz A_z, j_y += D_yz A_z (pushes), B_x, B_y
                Pairs<T> a, b;
                a.load(AZ, 1);
                b.load(AZ, XW);
                const T d2x = a.d2w(Zk.w.w2x), d2y = b.d2w(Zk.w.w2y);
                S.acc[2][PN] -= d2x + d2y;
                S.del[0][JD] = b.d1w(Zk.w.w1y);
                S.del[1][JD] = -a.d1w(Zk.w.w1x);
                S.del[5][JD] = eta * (d2x + d2y);
                push3<T, J>(S.acc[0], a.d, Zk.w.qx);
                push3<T, J>(S.acc[1], b.d, Zk.w.qy);
            }
        } else {
            // diagnostics only: the B parts of this plane
            Pairs<T> ay, bx_, cx_, cy_;
            ay.load(AX, XW);
            bx_.load(AY, 1);
            cx_.load(AZ, 1);
            cy_.load(AZ, XW);
            S.del[0][JD] = cy_.d1w(Zk.w.w1y);
            S.del[1][JD] = -cx_.d1w(Zk.w.w1x);
            S.del[2][JD] = bx_.d1w(Zk.w.w1x) - ay.d1w(Zk.w.w1y);
        }
        {  // ln rho and u of plane z' at the column, from the flow region
            const LP<T> *F = cf0 + JD * C::FREG;
            S.del[6][JD] = F[0];
            S.del[7][JD] = F[PLE];
            S.del[8][JD] = F[2 * PLE];
            S.del[9][JD] = F[3 * PLE];
        }
        if constexpr (DIAG && sizeof(T) == 4) {
            S.bd[0][JD] = zm_d1d(AZ, XW, dc.ih1[1]);
            S.bd[1][JD] = -zm_d1d(AZ, 1, dc.ih1[0]);
            S.bd[2][JD] = zm_d1d(AY, 1, dc.ih1[0]) - zm_d1d(AX, XW, dc.ih1[1]);
        }
#pragma unroll
        for (int m = 0; m < 3; m++) S.q[m][J] = now[m];
    }
}

template <typename T, int SUB, bool DIAG, bool STORE, int WPE, bool UPW = false, int TXV = 32>
__global__ void __launch_bounds__((ZmCfg<T, TXV>::NT), WPE)
k_zm(const RunDesc<T> *__restrict__ runs, const TileEnt *__restrict__ tiles, int step)
{
    using Z = Zm<T, SUB, DIAG, STORE, UPW, TXV>;
    using C = typename Z::C;
    constexpr int NT = C::NT, NC = C::NC, EPL = C::EPL, XW = C::XW, PLE = C::PLE;
    static_assert(!(DIAG && SUB != 0), "diagnostics are taken in substep 0 only");
    __shared__ __align__(16) T lds[C::LDS];

    const TileEnt te = tiles[blockIdx.x];
    const RunDesc<T> &r = runs[te.run];
    const int nx = r.nx, ny = r.ny, nz = r.nz;
    const int x0 = te.xy & 0xffff, y0 = te.xy >> 16, zs = te.z0, x0s = x0 + r.xs;
    const int len = min(r.seg, nz - zs);
    const int K = len + 6;  // steps: planes zs-3 .. zs+len+2
    const int par = (r.parity0 + step) & 1;
    const int in_set = (SUB == 1) ? (par ^ 1) : par;
    const int out_set = (SUB == 1) ? par : (par ^ 1);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const bool flow = wave < NC / 64;
    const int col = tid & (NC - 1);
    const int cx = col % C::TX, cy = col / C::TX;
    const uint64_t plane_b = (uint64_t)nx * (uint64_t)ny * sizeof(T);

    // Plane copies: wave-copy t = j * NWI + (issuing) wave (wave-uniform) brings 64 vectors
    // of the flow planes (t < NIF) or of the field planes (t >= NIF); every lane's source
    // is one field's row segment, the plane is added per step.
    const int wi = wave & (C::NWI - 1), ti = tid & (C::NTI - 1);  // index among the issuing waves, threads
    const G<char> *pp[C::NLP];
    int pdst[C::NLP];  // destination offset within a slot's regions (values; wave-uniform)
#pragma unroll
    for (int j = 0; j < C::NLP; j++) {
        const int t = j * C::NWI + wi;
        int f, v;
        if (t < C::NIF) {
            v = min(t * 64 + lane, 4 * C::PV - 1);
            f = v / C::PV;
            pdst[j] = C::FLOW + t * 64 * EPL;
        } else {
            const int ta = min(t - C::NIF, C::NIA - 1);  // spare copies repeat the last one
            v = min(ta * 64 + lane, 3 * C::PV - 1);
            f = 4 + v / C::PV;
                        pdst[j] = C::FIELD + ta * 64 * EPL;
        }
        const int e = (v - (f < 4 ? f : f - 4) * C::PV) * EPL;
        const int bx = e % XW, by = e / XW;
        const int gx = wrapi(x0s - 4 + bx, nx), gy = wrapi(y0 - 3 + by, ny);
        pp[j] = (const G<char> *)r.buf[in_set][f] + ((uint64_t)gx + (uint64_t)nx * gy) * sizeof(T);
    }
    // s-2 copies and the forcing z slot (SUB 0: every lane brings the forcing slot)
    const G<char> *sp[Z::NLS_E > 0 ? Z::NLS_E : 1];
    bool spf[Z::NLS_E > 0 ? Z::NLS_E : 1];
    const G<T> *fs = (const G<T> *)r.forcing + (size_t)step * (size_t)r.fstride;
    const G<T> *fz = fs + FHEAD + EPL * nx + EPL * ny;  // z phase table
#pragma unroll
    for (int j = 0; j < Z::NLS_E; j++) {
        int q = j * C::NTI + ti;
        spf[j] = SUB == 0 || q == C::SV;
        if (q >= C::SV) q = C::SV - 1;
        const int f = q / (NC / EPL), c = (q - f * (NC / EPL)) * EPL;
        const int x = c % C::TX, y = c / C::TX;
        const int gx = (x0s + x) % nx;
        sp[j] = (const G<char> *)r.buf[out_set][f] + ((uint64_t)gx + (uint64_t)nx * (y0 + y)) * sizeof(T);
    }
    // this thread's column: its byte offset in a plane (a plane holds fewer than 2^29
    // cells, since a run has fewer than 2^32 and nz >= 8), so that the stores take a
    // scalar base (field + plane) and this one 32-bit offset
    const uint32_t gcb = (uint32_t)(((uint64_t)((x0s + cx) % nx) + (uint64_t)nx * (uint64_t)(y0 + cy)) * sizeof(T));
    LP<T> *const lb = (LP<T> *)lds;
    LP<T> *pb0 = lb + (flow ? C::FLOW : C::FIELD) + (cy + 3) * XW + cx + 4 - (3 * XW + 3);
    LP<T> *sb0 = lb + C::S2 + col;
    LP<T> *xb0 = lb + C::XJ + col;
    LP<T> *cf0 = lb + C::FLOW + (cy + 3) * XW + cx + 4;

    KRegsFor<T, UPW> Kr;
    Kr.load(r.c);
    ZmK<T> Zk;
    Zk.load(r.c, SUB, flow ? 0 : 1);
    const DCoef &dc = r.dc;

    auto issue = [&](int k, int d) {
        int zp = zs - 3 + k;
        zp += zp < 0 ? nz : 0;
        zp -= zp >= nz ? nz : 0;
        const int zo = k >= 6 ? zs + k - 6 : zs;
        // the plane offsets in scalar registers: one 64-bit add per copy
        uint64_t zoff = (uint64_t)zp * plane_b, zob = (uint64_t)zo * plane_b;
        asm volatile("" : "+s"(zoff), "+s"(zob));
#pragma unroll
        for (int j = 0; j < C::NLP; j++) {
            const int dd = pdst[j] + d * (pdst[j] >= C::FIELD ? C::AREG : C::FREG);
            __builtin_amdgcn_global_load_lds((gconst_void_t *)(pp[j] + zoff), (lds_void_t *)(lds + dd), 16, 0, 0);
        }
        const G<char> *fzp = (const G<char> *)(fz + EPL * zo);
#pragma unroll
        for (int j = 0; j < Z::NLS_E; j++) {
            const G<char> *src = spf[j] ? fzp : sp[j] + zob;
            __builtin_amdgcn_global_load_lds((gconst_void_t *)src,
                                             (lds_void_t *)(lds + C::S2 + d * C::SREG + (j * C::NTI + wi * 64) * EPL), 16,
                                             0, 0);
        }
    };

    // forcing head and the tile's x/y phase slots (every wave writes the same values)
    if constexpr (STORE) {
        constexpr int HV = FHEAD / EPL;
        const G<T> *Ex = fs + FHEAD, *Ey = Ex + EPL * nx;
#pragma unroll
        for (int h = 0; h < C::NFHC; h++) {
            const G<T> *p = fs;
            int j = h * 64 + lane;
            if (j < HV) p = fs + j * EPL;
            else if ((j -= HV) < C::TX) p = Ex + EPL * ((x0s + j) % nx);
            else if ((j -= C::TX) < C::TY) p = Ey + EPL * (y0 + j);
            __builtin_amdgcn_global_load_lds((gconst_void_t *)p, (lds_void_t *)(lds + C::FH + h * 64 * EPL), 16, 0, 0);
        }
    }
    if (!C::ALLF || flow) {
        issue(0, 0);
        if (K > 1) issue(1, 1);
    }

    // flow and field threads run separate copies of the step loop (the same waits and
    // barriers in the same order), so that each keeps only its own state in registers
    ZmState<T> S;
#pragma unroll
    for (int i = 0; i < 6; i++) {
#pragma unroll
        for (int m = 0; m < 3; m++) S.acc[m][i] = T(0);
    }
#pragma unroll
    for (int i = 0; i < 9; i++) S.dg[i] = 0.0;
    S.fpr = T(1);
    S.fpi = T(0);
    T fa[3] = {T(0), T(0), T(0)}, fb[3] = {T(0), T(0), T(0)};
    bool fon = false;
    const int nit = (K + 5) / 6;
#define ZM_STEPS(ROLE)                                                                                               \
    for (int it = 0; it < nit; it++) {                                                                               \
        zm_body<T, SUB, DIAG, STORE, UPW, TXV, ROLE, 0>(it * 6 + 0, K, lds, S, Kr, Zk, dc, r, pb0, sb0, xb0, cf0, col, gcb, plane_b, zs,  \
                                                  out_set, fa, fb, fon, issue);                                       \
        zm_body<T, SUB, DIAG, STORE, UPW, TXV, ROLE, 1>(it * 6 + 1, K, lds, S, Kr, Zk, dc, r, pb0, sb0, xb0, cf0, col, gcb, plane_b, zs,  \
                                                  out_set, fa, fb, fon, issue);                                       \
        zm_body<T, SUB, DIAG, STORE, UPW, TXV, ROLE, 2>(it * 6 + 2, K, lds, S, Kr, Zk, dc, r, pb0, sb0, xb0, cf0, col, gcb, plane_b, zs,  \
                                                  out_set, fa, fb, fon, issue);                                       \
        zm_body<T, SUB, DIAG, STORE, UPW, TXV, ROLE, 3>(it * 6 + 3, K, lds, S, Kr, Zk, dc, r, pb0, sb0, xb0, cf0, col, gcb, plane_b, zs,  \
                                                  out_set, fa, fb, fon, issue);                                       \
        zm_body<T, SUB, DIAG, STORE, UPW, TXV, ROLE, 4>(it * 6 + 4, K, lds, S, Kr, Zk, dc, r, pb0, sb0, xb0, cf0, col, gcb, plane_b, zs,  \
                                                  out_set, fa, fb, fon, issue);                                       \
        zm_body<T, SUB, DIAG, STORE, UPW, TXV, ROLE, 5>(it * 6 + 5, K, lds, S, Kr, Zk, dc, r, pb0, sb0, xb0, cf0, col, gcb, plane_b, zs,  \
                                                  out_set, fa, fb, fon, issue);                                       \
    }
    if (flow) {
        ZM_STEPS(0)
    } else {
        ZM_STEPS(1)
    }
#undef ZM_STEPS
    if constexpr (STORE && C::DEFER) {  // the last output plane's u takes the last step's exchange
        lds_barrier();
        if (flow)
            zm_flush<T, NC>(S.pend, xb0 + ((K - 1) & 1) * 3 * NC, r, out_set, (uint64_t)(zs + K - 7) * plane_b, gcb,
                            Zk.bdt);
    }

    if constexpr (DIAG) {
        // per-tile partials: lane sums -> wave (DPP) -> fixed-order sum over waves
        double acc[9];  // each thread left zero the sums of the other role
#pragma unroll
        for (int q = 0; q < 9; q++) acc[q] = S.dg[q];
#pragma unroll
        for (int q = 0; q < 9; q++) acc[q] = (q == 7) ? wave_reduce<true>(acc[q]) : wave_reduce<false>(acc[q]);
        double *red = reinterpret_cast<double *>(lds + C::XJ);
        lds_barrier();
        if (lane == 63) {
#pragma unroll
            for (int q = 0; q < 9; q++) red[wave * 9 + q] = acc[q];
        }
        lds_barrier();
        if (tid < 9) {
            double sum = red[tid];
            for (int w = 1; w < NT / 64; w++) sum = (tid == 7) ? fmax(sum, red[w * 9 + tid]) : sum + red[w * 9 + tid];
            ((G<double> *)r.partials)[(size_t)te.tir * DIAGW + tid] = sum;
        }
    }
}

}  // namespace mhd
