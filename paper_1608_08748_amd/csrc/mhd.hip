// HIP implementation of one operator-split step of ideal MHD with H/H2
// chemistry on a uniform periodic grid (Kulikov, Chernykh & Protasov,
// arXiv:1608.08748), for AMD MI355X (gfx950).  C ABI: include/mhdchem.h.
//
// Stage names: NONADV is the paper's "eulerian" stage (Sec. 2.4, 2.5: pressure,
// Lorentz force, p dV work, face-field update); ADV is its "lagrangian" stage
// (Sec. 2.6: advection).  Readings of ambiguous passages are the same as the
// ones listed in the design notes (dq = qR - qL, Step-4 blend weights, the
// projector form of the face state, the pressure-gated dual-energy sync, ...).
//
// Data layout in HBM: structure of arrays, one array of n cells per field,
// x fastest.  The state is split into three groups that are updated by
// different stages, each with three Runge-Kutta slots:
//   H = (rho, h2)            updated by ADV and the tail
//   M = (mx, my, mz, E, e)   updated by NONADV, ADV and the tail
//   B = (bx, by, bz)         updated by NONADV (face-centred, lower faces)
// so no stage copies a field it does not change.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>

#include "mhdchem.h"

namespace {

constexpr int NTH = 256;           // threads per block for cell-parallel kernels
constexpr int NF = 10;             // conserved fields
constexpr int NFACE = 7;           // per-face outputs
enum { RHO = 0, MX, MY, MZ, EN, EI, BX, BY, BZ, H2 };

// ---------------------------------------------------------------- geometry

struct Geo {
    int nx, ny, nz;
    int nxy;
    int n;          // nx * ny * nz
};

__device__ __forceinline__ int wrapc(int x, int n)
{
    if (x < 0) x += n;
    if (x >= n) x -= n;
    if ((unsigned)x >= (unsigned)n) {   // only for boxes thinner than the stencil
        x %= n;
        if (x < 0) x += n;
    }
    return x;
}

// cell index of the neighbour at offset s along direction D
template <int D>
__device__ __forceinline__ int nbr(const Geo& g, int c, int i, int j, int k, int s)
{
    if (D == 0) return c - i + wrapc(i + s, g.nx);
    if (D == 1) return c + (wrapc(j + s, g.ny) - j) * g.nx;
    return c + (wrapc(k + s, g.nz) - k) * g.nxy;
}

__device__ __forceinline__ void decompose(const Geo& g, int c, int& i, int& j, int& k)
{
    unsigned uc = (unsigned)c;
    unsigned t = uc / (unsigned)g.nx;
    i = (int)(uc - t * (unsigned)g.nx);
    unsigned kk = t / (unsigned)g.ny;
    j = (int)(t - kk * (unsigned)g.ny);
    k = (int)kk;
}

template <typename T> struct Fields { T* f[NF]; };
template <typename T> struct CFields { const T* f[NF]; };

// ---------------------------------------------------------------- local parabola (Sec. 2.1)

template <typename T> struct Par { T qL, qR, dq, q6; };

// Step 1: limited central difference (min of the three candidates, sign of
// the central difference; zero at extrema)
template <typename T>
__device__ __forceinline__ T limited_slope(T qm, T q0, T qp)
{
    T dq = T(0.5) * (qp - qm);
    T a = T(2) * fabs(qp - q0);
    T b = T(2) * fabs(q0 - qm);
    T m = fmin(fmin(fabs(dq), a), b);
    return ((qp - q0) * (q0 - qm) > T(0)) ? copysign(m, dq) : T(0);
}

// Step 1: fourth-order interface value q_{j+1/2} = 1/2 (q_j + q_{j+1}) - 1/6 (dm_{j+1} - dm_j)
template <typename T>
__device__ __forceinline__ T interface_value(T q0, T q1, T dm0, T dm1)
{
    return T(0.5) * (q0 + q1) - T(1.0 / 6.0) * (dm1 - dm0);
}

// margins that decide a saturated Step-4 weight without the division
template <typename T> struct EtaMargin;
template <> struct EtaMargin<double> { static constexpr double lo = 0.05 * (1.0 - 1e-9), hi = 0.1 * (1.0 + 1e-9); };
template <> struct EtaMargin<float> { static constexpr float lo = 0.05f * (1.0f - 1e-5f), hi = 0.1f * (1.0f + 1e-5f); };

// Steps 2-5 for cell j with line values qmm..qpp, Step-1 edge values qL, qR
// and limited slope dm of the cell
template <typename T>
__device__ __forceinline__ Par<T> parabola_finish(T qmm, T qm, T q0, T qp, T qpp, T qL, T qR, T dm)
{
    // Step 2: monotone edge values
    T dq = qR - qL;
    T q6 = T(6) * (q0 - T(0.5) * (qL + qR));
    bool flat = (qL - q0) * (q0 - qR) <= T(0);
    bool overL = dq * q6 > dq * dq;
    bool overR = dq * q6 < -(dq * dq);
    T nL = flat ? q0 : (overL ? T(3) * q0 - T(2) * qR : qL);
    T nR = flat ? q0 : ((!overL && overR) ? T(3) * q0 - T(2) * qL : qR);
    // Step 4: discontinuity detector on second differences (h^2 cancels)
    T qLp = q0 - T(0.25) * dm;
    T qRp = q0 + T(0.25) * dm;
    T Dm = q0 - T(2) * qm + qmm;
    T Dp = qpp - T(2) * qp + q0;
    T aqp = fabs(qp), aqm = fabs(qm);
    T mn = fmin(fmin(aqp, aqm), aqp + aqm);
    bool zero_eta = (fabs(qp - qm) - T(0.01) * mn <= T(0)) || (Dp * Dm > T(0));
    // eta = t / d; the weight w = clamp(20 (eta - 0.05), 0, 1) is exactly 0
    // or 1 outside a band around [0.05, 0.1], decided by products with a
    // relative margin far above rounding; the division runs only inside it
    T t = -(Dp - Dm);
    T d = T(6) * (qp - qm);
    T ts = d < T(0) ? -t : t;
    T ds = fabs(d);
    bool sat_hi = !zero_eta && ts >= EtaMargin<T>::hi * ds;
    bool need = !zero_eta && !sat_hi && !(ts <= EtaMargin<T>::lo * ds);
    T w = sat_hi ? T(1) : T(0);
    if (need) {
        T eta = t / d;
        w = fmin(fmax(T(20) * (eta - T(0.05)), T(0)), T(1));
    }
    T fL = (T(1) - w) * nL + w * qLp;
    T fR = (T(1) - w) * nR + w * qRp;
    // Step 5
    Par<T> p;
    p.qL = fL;
    p.qR = fR;
    p.dq = fR - fL;
    p.q6 = T(6) * (q0 - T(0.5) * (fL + fR));
    return p;
}

// Steps 1-5 for the cell with line values qmm, qm, q0, qp, qpp
template <typename T>
__device__ __forceinline__ Par<T> parabola(T qmm, T qm, T q0, T qp, T qpp)
{
    T dm_m = limited_slope(qmm, qm, q0);
    T dm_0 = limited_slope(qm, q0, qp);
    T dm_p = limited_slope(q0, qp, qpp);
    T qL = interface_value(qm, q0, dm_m, dm_0);
    T qR = interface_value(q0, qp, dm_0, dm_p);
    return parabola_finish(qmm, qm, q0, qp, qpp, qL, qR, dm_0);
}

// parabolas of the two cells on either side of a face from the 6-cell line
// q0..q5 (cells i-3..i+2; left cell i-1, right cell i): the middle slopes and
// the face value q_{i-1/2} are shared, so this is the same arithmetic as two
// separate calls
template <typename T>
__device__ __forceinline__ void parabola_pair(T q0, T q1, T q2, T q3, T q4, T q5, Par<T>& PL, Par<T>& PR)
{
    T d1 = limited_slope(q0, q1, q2);
    T d2 = limited_slope(q1, q2, q3);
    T d3 = limited_slope(q2, q3, q4);
    T d4 = limited_slope(q3, q4, q5);
    T f12 = interface_value(q1, q2, d1, d2);
    T f23 = interface_value(q2, q3, d2, d3);
    T f34 = interface_value(q3, q4, d3, d4);
    PL = parabola_finish(q0, q1, q2, q3, q4, f12, f23, d2);
    PR = parabola_finish(q1, q2, q3, q4, q5, f23, f34, d3);
}

// Sec. 2.4: average over the right part of relative width y (the q(-nu t) formula)
template <typename T>
__device__ __forceinline__ T avg_right(const Par<T>& p, T y)
{
    return p.qR - T(0.5) * y * (p.dq - p.q6 * (T(1) - T(2.0 / 3.0) * y));
}

// Sec. 2.4: average over the left part of relative width y (the q(+nu t) formula)
template <typename T>
__device__ __forceinline__ T avg_left(const Par<T>& p, T y)
{
    return p.qL + T(0.5) * y * (p.dq + p.q6 * (T(1) - T(2.0 / 3.0) * y));
}

template <typename T> struct Eps;
template <> struct Eps<double> { static constexpr double v = 1e-12; };
template <> struct Eps<float> { static constexpr float v = 1e-6f; };

// ---------------------------------------------------------------- kernels

struct StepArgs {
    double dt_val;          // explicit step, or
    const double* dt_dev;   // device-resident CFL step when non-null
    double gamma;
    double h;               // 1 / nx
    double theta;
    double cfl_tol;         // relative slack of the dt <= CFL-bound check
};

__device__ __forceinline__ double step_dt(const StepArgs& a)
{
    return a.dt_dev ? *a.dt_dev : a.dt_val;
}

// primitive state of every cell: rho, vx, vy, vz, Bcx, Bcy, Bcz, p
template <typename T>
__global__ __launch_bounds__(NTH) void k_prim(Geo g, CFields<T> U, T* __restrict__ W, StepArgs a,
                                              uint32_t* flags, const double* dt_cfl)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c == 0 && dt_cfl && !a.dt_dev) {
        if (a.dt_val > *dt_cfl * (1.0 + a.cfl_tol)) atomicOr(flags, 2u);
    }
    if (c >= g.n) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const size_t N = (size_t)g.n;
    T rho = U.f[RHO][c];
    W[0 * N + c] = rho;
    W[1 * N + c] = U.f[MX][c] / rho;
    W[2 * N + c] = U.f[MY][c] / rho;
    W[3 * N + c] = U.f[MZ][c] / rho;
    W[4 * N + c] = T(0.5) * (U.f[BX][c] + U.f[BX][nbr<0>(g, c, i, j, k, 1)]);
    W[5 * N + c] = T(0.5) * (U.f[BY][c] + U.f[BY][nbr<1>(g, c, i, j, k, 1)]);
    W[6 * N + c] = T(0.5) * (U.f[BZ][c] + U.f[BZ][nbr<2>(g, c, i, j, k, 1)]);
    W[7 * N + c] = T(a.gamma - 1.0) * U.f[EI][c];
}

// What one side of a face needs from a cell's parabolas (6 variables): the
// edge value facing the face (qR of the left cell, qL of the right cell), dq
// and q6.
template <typename T> struct Side { T e[6], dq[6], q6[6]; };

template <typename T>
__device__ __forceinline__ void side_left(const Par<T>& P, Side<T>& S, int v)
{
    S.e[v] = P.qR;
    S.dq[v] = P.dq;
    S.q6[v] = P.q6;
}

template <typename T>
__device__ __forceinline__ void side_right(const Par<T>& P, Side<T>& S, int v)
{
    S.e[v] = P.qL;
    S.dq[v] = P.dq;
    S.q6[v] = P.q6;
}

// NONADV face state (Sec. 2.4) of one face and the fluxes and edge-field
// contributions it produces.  Inputs: cell-centre rho, p, Bt1, Bt2 of the left
// and right cells, the face normal field bn, the two sides' parabolas of
// (vn, vt1, vt2, Bt1, Bt2, p).  Outputs (7): momentum flux (normal, t1, t2),
// energy flux, face normal velocity, E along t1 (B_t2 U_n - B_n U_t2), E along
// t2 (B_n U_t1 - B_t1 U_n).
template <typename T>
__device__ __forceinline__ void face_solve(T rl, T pl, T b1l, T b2l, T rr, T pr, T b1r, T b2r, T bn,
                                           const Side<T>& L, const Side<T>& R, T gm, T ydx, T out[7])
{
    const T eps = Eps<T>::v;
    // face averages (sqrt(rho) weights; cross weights for Bt)
    T sl = sqrt(rl), sr = sqrt(rr);
    T iw = T(1) / (sl + sr);
    T rho = (sl * rl + sr * rr) * iw;
    T p = (sl * pl + sr * pr) * iw;
    T bt1 = (sl * b1r + sr * b1l) * iw;
    T bt2 = (sl * b2r + sr * b2l) * iw;

    // eigen-structure (Sec. 2.3, 2.4, eigenvector appendix)
    T irho = T(1) / rho;
    T c2 = gm * p * irho;
    T ca2 = bn * bn * irho;
    T b2 = (bn * bn + bt1 * bt1 + bt2 * bt2) * irho;
    T s = c2 + b2;
    T disc = fmax(s * s - T(4) * c2 * ca2, T(0));
    T sd = sqrt(disc);
    T cf2 = T(0.5) * (s + sd);
    T cs2 = fmax(T(0.5) * (s - sd), T(0));
    T cc = sqrt(c2), ca = sqrt(ca2), cf = sqrt(cf2), cs = sqrt(cs2);
    const T r2i = T(0.70710678118654752440);
    T den = cf2 - cs2;
    T af = r2i, as = r2i;
    if (den > eps * s) {
        T iden = T(1) / den;
        af = sqrt(fmax(c2 - cs2, T(0)) * iden);
        as = sqrt(fmax(cf2 - c2, T(0)) * iden);
    }
    T by = r2i, bz = r2i;
    T btsq = bt1 * bt1 + bt2 * bt2;
    if (btsq > eps * (bn * bn + btsq + gm * p)) {
        T ibt = T(1) / sqrt(btsq);
        by = bt1 * ibt;
        bz = bt2 * ibt;
    }
    T sg = bn >= T(0) ? T(1) : T(-1);
    T srho = sqrt(rho);

    // parabola averages on the upwind side of each wave: waves +cf, +cs, +ca
    // read the left cell (right part, q(-nu t)), waves -cf, -cs, -ca the right
    // cell (left part, q(+nu t))
    T qf[6], qfm[6], qs[6], qsm[6], qa[6], qam[6];
    T y3[3] = { ydx * cf, ydx * cs, ydx * ca };
    T hy[3], ky[3];
#pragma unroll
    for (int w = 0; w < 3; w++) {
        hy[w] = T(0.5) * y3[w];
        ky[w] = T(1) - T(2.0 / 3.0) * y3[w];
    }
#pragma unroll
    for (int v = 0; v < 6; v++) {
        qf[v] = L.e[v] - hy[0] * (L.dq[v] - L.q6[v] * ky[0]);
        qs[v] = L.e[v] - hy[1] * (L.dq[v] - L.q6[v] * ky[1]);
        qa[v] = L.e[v] - hy[2] * (L.dq[v] - L.q6[v] * ky[2]);
        qfm[v] = R.e[v] + hy[0] * (R.dq[v] + R.q6[v] * ky[0]);
        qsm[v] = R.e[v] + hy[1] * (R.dq[v] + R.q6[v] * ky[1]);
        qam[v] = R.e[v] + hy[2] * (R.dq[v] + R.q6[v] * ky[2]);
    }

    // characteristic amplitudes s_k = l_k . q_up(k)
    T ic2 = T(1) / c2;
    T isc = T(1) / (srho * cc);
    T A = T(0.5) * ic2;                  // 1 / (2 c^2)
    T Bc = T(0.5) * isc;                 // 1 / (2 sqrt(rho) c)
    T Cc = A * irho;                     // 1 / (2 rho c^2)
    T Dc = r2i / srho;                   // 1 / sqrt(2 rho)
    T afcf = af * cf, ascs = as * cs;
    auto vtb = [&](const T* q) { return by * q[1] + bz * q[2]; };
    auto btb = [&](const T* q) { return by * q[3] + bz * q[4]; };
    auto vtp = [&](const T* q) { return -bz * q[1] + by * q[2]; };
    auto btp = [&](const T* q) { return -bz * q[3] + by * q[4]; };
    T s0 = (afcf * qf[0] - ascs * sg * vtb(qf)) * A + as * btb(qf) * Bc + af * qf[5] * Cc;
    T s1 = (-afcf * qfm[0] + ascs * sg * vtb(qfm)) * A + as * btb(qfm) * Bc + af * qfm[5] * Cc;
    T s2 = (ascs * qs[0] + afcf * sg * vtb(qs)) * A - af * btb(qs) * Bc + as * qs[5] * Cc;
    T s3 = (-ascs * qsm[0] - afcf * sg * vtb(qsm)) * A - af * btb(qsm) * Bc + as * qsm[5] * Cc;
    T s4 = sg * r2i * vtp(qa) - btp(qa) * Dc;
    T s5 = sg * r2i * vtp(qam) + btp(qam) * Dc;

    // face state q = sum_k r_k s_k
    T fdm = s0 - s1, fsm = s0 + s1, sdm = s2 - s3, ssm = s2 + s3, adm = s4 - s5, asm_ = s4 + s5;
    T src = srho * cc;
    T sr2 = r2i * srho;
    T gp = gm * p;
    T Vn = afcf * fdm + ascs * sdm;
    T Vt1 = sg * by * (-ascs * fdm + afcf * sdm) - bz * sg * r2i * asm_;
    T Vt2 = sg * bz * (-ascs * fdm + afcf * sdm) + by * sg * r2i * asm_;
    T Bt1 = by * src * (as * fsm - af * ssm) + sr2 * bz * adm;
    T Bt2 = bz * src * (as * fsm - af * ssm) - sr2 * by * adm;
    T P = gp * (af * fsm + as * ssm);

    // fluxes of the non-advective equations and edge-field contributions
    T Pst = P + T(0.5) * (bn * bn + Bt1 * Bt1 + Bt2 * Bt2);
    T BV = bn * Vn + Bt1 * Vt1 + Bt2 * Vt2;
    out[0] = Pst - bn * bn;
    out[1] = -(bn * Bt1);
    out[2] = -(bn * Bt2);
    out[3] = Pst * Vn - bn * BV;
    out[4] = Vn;
    out[5] = Bt2 * Vn - bn * Vt2;
    out[6] = bn * Vt1 - Bt1 * Vn;
}

// primitive-array slots of the six parabola variables for faces along D:
// (vn, vt1, vt2, Bt1, Bt2, p) in the W layout rho, vx, vy, vz, Bcx, Bcy, Bcz, p
template <int D> struct Vars {
    static constexpr int T1 = (D + 1) % 3, T2 = (D + 2) % 3;
    static constexpr int f[6] = { 1 + D, 1 + T1, 1 + T2, 4 + T1, 4 + T2, 7 };
};

template <typename T>
__device__ __forceinline__ void store_face(T* __restrict__ F, size_t N, int c, const T out[7])
{
#pragma unroll
    for (int q = 0; q < 7; q++) F[q * N + c] = out[q];
}

// NONADV faces along D, one face per thread, both adjacent parabolas computed
// by the thread (general fallback for any box)
template <typename T, int D>
__global__ __launch_bounds__(NTH) void k_nonadv_face(Geo g, const T* __restrict__ W, const T* __restrict__ bface,
                                                     T* __restrict__ F, StepArgs a)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    using V = Vars<D>;
    int i, j, k;
    decompose(g, c, i, j, k);
    const size_t N = (size_t)g.n;
    int idx[6];
#pragma unroll
    for (int m = 0; m < 6; m++) idx[m] = nbr<D>(g, c, i, j, k, m - 3);
    Side<T> L, R;
#pragma unroll
    for (int v = 0; v < 6; v++) {
        const T* q = W + (size_t)V::f[v] * N;
        Par<T> PL, PR;
        parabola_pair(q[idx[0]], q[idx[1]], q[idx[2]], q[idx[3]], q[idx[4]], q[idx[5]], PL, PR);
        side_left(PL, L, v);
        side_right(PR, R, v);
    }
    T out[7];
    face_solve(W[idx[2]], W[7 * N + idx[2]], W[(size_t)V::f[3] * N + idx[2]], W[(size_t)V::f[4] * N + idx[2]],
               W[idx[3]], W[7 * N + idx[3]], W[(size_t)V::f[3] * N + idx[3]], W[(size_t)V::f[4] * N + idx[3]],
               bface[c], L, R, T(a.gamma), T(a.theta * (step_dt(a) / a.h)), out);
    store_face(F, N, c, out);
}

// NONADV faces along x with whole x rows per block: each thread computes the
// parabolas of its own cell once; the left neighbour's side comes from LDS
// (periodic wrap inside the row), so no parabola is computed twice.
template <typename T, int MAXT>
__global__ __launch_bounds__(MAXT) void k_nonadv_xrows(Geo g, const T* __restrict__ W, const T* __restrict__ bface,
                                                       T* __restrict__ F, StepArgs a, int rpb)
{
    extern __shared__ unsigned char smem_raw[];
    T* sm = reinterpret_cast<T*>(smem_raw);
    using V = Vars<0>;
    const size_t N = (size_t)g.n;
    const int nx = g.nx;
    int tid = threadIdx.x;
    int r = tid / nx;
    int i = tid - r * nx;
    int row = blockIdx.x * rpb + r;
    bool act = r < rpb && row < g.ny * g.nz;
    int rowbase = row * nx;
    Side<T> R;
    if (act) {
        int im2 = wrapc(i - 2, nx), im1 = wrapc(i - 1, nx), ip1 = wrapc(i + 1, nx), ip2 = wrapc(i + 2, nx);
        T* mine = sm + (size_t)(r * nx + i) * 18;
#pragma unroll
        for (int v = 0; v < 6; v++) {
            const T* q = W + (size_t)V::f[v] * N + rowbase;
            Par<T> P = parabola(q[im2], q[im1], q[i], q[ip1], q[ip2]);
            side_right(P, R, v);
            mine[3 * v + 0] = P.qR;
            mine[3 * v + 1] = P.dq;
            mine[3 * v + 2] = P.q6;
        }
    }
    __syncthreads();
    if (!act) return;
    int il = i == 0 ? nx - 1 : i - 1;
    const T* left = sm + (size_t)(r * nx + il) * 18;
    Side<T> L;
#pragma unroll
    for (int v = 0; v < 6; v++) {
        L.e[v] = left[3 * v + 0];
        L.dq[v] = left[3 * v + 1];
        L.q6[v] = left[3 * v + 2];
    }
    int c = rowbase + i, cl = rowbase + il;
    T out[7];
    face_solve(W[cl], W[7 * N + cl], W[(size_t)V::f[3] * N + cl], W[(size_t)V::f[4] * N + cl],
               W[c], W[7 * N + c], W[(size_t)V::f[3] * N + c], W[(size_t)V::f[4] * N + c],
               bface[c], L, R, T(a.gamma), T(a.theta * (step_dt(a) / a.h)), out);
    store_face(F, N, c, out);
}

// NONADV faces along D = y or z: each thread marches along one grid line over
// a segment of `seg` faces with a sliding 5-cell window in registers, so each
// cell's parabolas are computed once per segment (seg + 1 per seg faces);
// threads are consecutive in x, so every load is coalesced.
template <typename T, int D>
__global__ __launch_bounds__(NTH) void k_nonadv_march(Geo g, const T* __restrict__ W, const T* __restrict__ bface,
                                                      T* __restrict__ F, StepArgs a, int seg)
{
    using V = Vars<D>;
    const size_t N = (size_t)g.n;
    const int nd = D == 1 ? g.ny : g.nz;
    const int no = D == 1 ? g.nz : g.ny;
    const int nseg = (nd + seg - 1) / seg;
    int t = blockIdx.x * NTH + threadIdx.x;
    int i = t % g.nx;
    int rest = t / g.nx;
    int o = rest % no;
    int sgi = rest / no;
    if (sgi >= nseg) return;
    const int base = D == 1 ? i + g.nxy * o : i + g.nx * o;
    const int stride = D == 1 ? g.nx : g.nxy;
    const int x0 = sgi * seg;
    const int x1 = min(x0 + seg, nd);
    const T gm = T(a.gamma);
    const T ydx = T(a.theta * (step_dt(a) / a.h));

    // window: w[v][m] = variable v of cell x-2+m; v = 0..5 parabola variables, 6 = rho
    T w[7][5];
#pragma unroll
    for (int m = 0; m < 5; m++) {
        int cc = base + wrapc(x0 - 3 + m, nd) * stride;
#pragma unroll
        for (int v = 0; v < 6; v++) w[v][m] = W[(size_t)V::f[v] * N + cc];
        w[6][m] = W[cc];
    }
    // parabolas of cell x0 - 1 (the left side of the first face)
    Side<T> L;
#pragma unroll
    for (int v = 0; v < 6; v++) side_left(parabola(w[v][0], w[v][1], w[v][2], w[v][3], w[v][4]), L, v);

    for (int x = x0; x < x1; x++) {
        int cn = base + wrapc(x + 2, nd) * stride;
#pragma unroll
        for (int v = 0; v < 7; v++) {
#pragma unroll
            for (int m = 0; m < 4; m++) w[v][m] = w[v][m + 1];
            w[v][4] = W[(size_t)(v < 6 ? V::f[v] : 0) * N + cn];
        }
        Side<T> R, Ln;
#pragma unroll
        for (int v = 0; v < 6; v++) {
            Par<T> P = parabola(w[v][0], w[v][1], w[v][2], w[v][3], w[v][4]);
            side_right(P, R, v);
            side_left(P, Ln, v);
        }
        int c = base + x * stride;
        T out[7];
        // left cell x-1 is window slot 1, right cell x is slot 2
        face_solve(w[6][1], w[5][1], w[3][1], w[4][1], w[6][2], w[5][2], w[3][2], w[4][2], bface[c], L, R, gm,
                   ydx, out);
        store_face(F, N, c, out);
        L = Ln;
    }
}

struct RK { double a, b; };

// NONADV update: flux differences, p dV work, face-field update from edge
// fields (Sec. 2.5), Runge-Kutta combination (Sec. 2.2).  debug_inc != 0
// writes tau R(U) instead of the combination.
template <typename T>
__global__ __launch_bounds__(NTH) void k_nonadv_update(Geo g, CFields<T> U, CFields<T> S, Fields<T> O,
                                                       const T* __restrict__ Fx, const T* __restrict__ Fy,
                                                       const T* __restrict__ Fz, StepArgs a, RK rk, int debug_inc)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const size_t N = (size_t)g.n;
    const T dtdx = T(step_dt(a) / a.h);
    int xp = nbr<0>(g, c, i, j, k, 1), xm = nbr<0>(g, c, i, j, k, -1);
    int yp = nbr<1>(g, c, i, j, k, 1), ym = nbr<1>(g, c, i, j, k, -1);
    int zp = nbr<2>(g, c, i, j, k, 1), zm = nbr<2>(g, c, i, j, k, -1);
    const T* Fd[3] = { Fx, Fy, Fz };
    int up[3] = { xp, yp, zp };
    T dF[3][5];
#pragma unroll
    for (int d = 0; d < 3; d++)
#pragma unroll
        for (int v = 0; v < 5; v++) dF[d][v] = Fd[d][v * N + up[d]] - Fd[d][v * N + c];
    T inc[NF];
    // momentum component a takes slot (a - d) mod 3 from direction d
    inc[MX] = -dtdx * ((dF[0][0] + dF[1][2]) + dF[2][1]);
    inc[MY] = -dtdx * ((dF[0][1] + dF[1][0]) + dF[2][2]);
    inc[MZ] = -dtdx * ((dF[0][2] + dF[1][1]) + dF[2][0]);
    inc[EN] = -dtdx * ((dF[0][3] + dF[1][3]) + dF[2][3]);
    T divv = (dF[0][4] + dF[1][4]) + dF[2][4];
    inc[EI] = -T(a.gamma - 1.0) * U.f[EI][c] * dtdx * divv;

    // edge fields (electric-field appendix): Ex at (i, j-1/2, k-1/2) from
    // z faces at j-1, j and y faces at k, k-1; Ey at (i-1/2, j, k-1/2) from
    // z faces at i-1, i and x faces at k-1, k; Ez at (i-1/2, j-1/2, k) from
    // x faces at j-1, j and y faces at i-1, i.
    const T* ezx = Fz + 5 * N;   // z faces, E along x
    const T* ezy = Fz + 6 * N;   // z faces, E along y
    const T* eyz = Fy + 5 * N;   // y faces, E along z
    const T* eyx = Fy + 6 * N;   // y faces, E along x
    const T* exy = Fx + 5 * N;   // x faces, E along y
    const T* exz = Fx + 6 * N;   // x faces, E along z
    auto Ex = [&](int cc, int cym, int czm) { return T(0.25) * (((ezx[cym] + ezx[cc]) + eyx[cc]) + eyx[czm]); };
    auto Ey = [&](int cc, int cxm, int czm) { return T(0.25) * (((ezy[cxm] + ezy[cc]) + exy[czm]) + exy[cc]); };
    auto Ez = [&](int cc, int cym, int cxm) { return T(0.25) * (((exz[cym] + exz[cc]) + eyz[cxm]) + eyz[cc]); };
    // neighbours of the shifted cells
    int ip, jp, kp;
    // Ex at c, c+y, c+z
    T Ex_c = Ex(c, ym, zm);
    decompose(g, yp, ip, jp, kp);
    T Ex_yp = Ex(yp, c, nbr<2>(g, yp, ip, jp, kp, -1));
    decompose(g, zp, ip, jp, kp);
    T Ex_zp = Ex(zp, nbr<1>(g, zp, ip, jp, kp, -1), c);
    // Ey at c, c+x, c+z
    T Ey_c = Ey(c, xm, zm);
    decompose(g, xp, ip, jp, kp);
    T Ey_xp = Ey(xp, c, nbr<2>(g, xp, ip, jp, kp, -1));
    decompose(g, zp, ip, jp, kp);
    T Ey_zp = Ey(zp, nbr<0>(g, zp, ip, jp, kp, -1), c);
    // Ez at c, c+x, c+y
    T Ez_c = Ez(c, ym, xm);
    decompose(g, xp, ip, jp, kp);
    T Ez_xp = Ez(xp, nbr<1>(g, xp, ip, jp, kp, -1), c);
    decompose(g, yp, ip, jp, kp);
    T Ez_yp = Ez(yp, c, nbr<0>(g, yp, ip, jp, kp, -1));
    inc[BX] = -dtdx * (Ez_yp - Ez_c) + dtdx * (Ey_zp - Ey_c);
    inc[BY] = -dtdx * (Ex_zp - Ex_c) + dtdx * (Ez_xp - Ez_c);
    inc[BZ] = -dtdx * (Ey_xp - Ey_c) + dtdx * (Ex_yp - Ex_c);

    const int upd[8] = { MX, MY, MZ, EN, EI, BX, BY, BZ };
    if (debug_inc) {
#pragma unroll
        for (int q = 0; q < 8; q++) O.f[upd[q]][c] = inc[upd[q]];
        O.f[RHO][c] = T(0);
        O.f[H2][c] = T(0);
        return;
    }
    const T ra = T(rk.a), rb = T(rk.b);
#pragma unroll
    for (int q = 0; q < 8; q++) {
        int f = upd[q];
        T u = U.f[f][c];
        O.f[f][c] = (u + ra * (S.f[f][c] - u)) + rb * inc[f];
    }
}

// ADV fluxes at the lower face of every cell along D (Sec. 2.6): outputs, 7 x N,
// in the order rho, mx, my, mz, E, e, h2.
template <typename T, int D>
__global__ __launch_bounds__(NTH) void k_adv_face(Geo g, CFields<T> U, T* __restrict__ F, StepArgs a)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const size_t N = (size_t)g.n;
    const T ydx = T(a.theta * (step_dt(a) / a.h));
    int idx[6];
#pragma unroll
    for (int m = 0; m < 6; m++) idx[m] = nbr<D>(g, c, i, j, k, m - 3);
    T rl = U.f[RHO][idx[2]], rr = U.f[RHO][c];
    T vl = U.f[MX + D][idx[2]] / rl;
    T vr = U.f[MX + D][c] / rr;
    T sl = sqrt(rl), sr = sqrt(rr);
    T vf = (sl * vl + sr * vr) / (sl + sr);
    bool upw = vf >= T(0);
    T y = upw ? ydx * vf : ydx * (-vf);
    const int fld[7] = { RHO, MX, MY, MZ, EN, EI, H2 };
#pragma unroll
    for (int q = 0; q < 7; q++) {
        const T* u = U.f[fld[q]];
        int o = upw ? 0 : 1;
        T q0 = u[idx[o]], q1 = u[idx[o + 1]], q2 = u[idx[o + 2]], q3 = u[idx[o + 3]], q4 = u[idx[o + 4]];
        Par<T> P = parabola(q0, q1, q2, q3, q4);
        T qup = upw ? avg_right(P, y) : avg_left(P, y);
        F[q * N + c] = vf * qup;
    }
}

template <typename T>
__global__ __launch_bounds__(NTH) void k_adv_update(Geo g, CFields<T> U, CFields<T> S, Fields<T> O,
                                                    const T* __restrict__ Fx, const T* __restrict__ Fy,
                                                    const T* __restrict__ Fz, StepArgs a, RK rk, int debug_inc)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const size_t N = (size_t)g.n;
    const T dtdx = T(step_dt(a) / a.h);
    int xp = nbr<0>(g, c, i, j, k, 1), yp = nbr<1>(g, c, i, j, k, 1), zp = nbr<2>(g, c, i, j, k, 1);
    const int fld[7] = { RHO, MX, MY, MZ, EN, EI, H2 };
    const T ra = T(rk.a), rb = T(rk.b);
#pragma unroll
    for (int q = 0; q < 7; q++) {
        T dx = Fx[q * N + xp] - Fx[q * N + c];
        T dy = Fy[q * N + yp] - Fy[q * N + c];
        T dz = Fz[q * N + zp] - Fz[q * N + c];
        T inc = -dtdx * ((dx + dy) + dz);
        int f = fld[q];
        if (debug_inc) {
            O.f[f][c] = inc;
        } else {
            T u = U.f[f][c];
            O.f[f][c] = (u + ra * (S.f[f][c] - u)) + rb * inc;
        }
    }
    if (debug_inc) {
        O.f[BX][c] = T(0);
        O.f[BY][c] = T(0);
        O.f[BZ][c] = T(0);
    }
}

// ---------------------------------------------------------------- FP64 per-cell physics

struct ChemArgs {
    int on;
    double n_unit, T_unit, t_unit;
};

// Sec. 2.7 with the appendix rates of reactions 1-4 (optically thin k4)
__device__ double chem_h2(const ChemArgs& ch, double gamma, double rho, double e, double h2, double dt)
{
    double p = (gamma - 1.0) * e;
    double xh2 = h2 / rho;
    double mu = 1.0 / (1.0 - 0.5 * xh2);
    double T = ch.T_unit * mu * p / rho;
    double nH = ch.n_unit * (rho - h2);
    double nH2 = ch.n_unit * h2 / 2.0;
    double n = nH + nH2;
    double t2 = T / 100.0;
    double st2 = sqrt(t2);
    double k1b = 3e-17 * st2 / (1.0 + 0.4 * st2 + 0.2 * t2 + 0.08 * t2 * t2);
    double k2 = (T > 7390.0) ? 6.11e-14 * exp(-2.93e4 / T) : 2.67e-15 * exp(-(6750.0 / T) * (6750.0 / T));
    double k3 = (T > 7291.0) ? 5.22e-14 * exp(-3.22e4 / T)
                             : 3.17e-15 * exp(-(4060.0 / T) - (7500.0 / T) * (7500.0 / T));
    double k4 = 3.3 * 1.7e-11;
    double C = k1b * n * nH;
    double Dd = k2 * nH + k3 * nH2 + k4;
    double ts = dt * ch.t_unit;
    double nn = nH2 + ts * (C - Dd * nH2) / (1.0 + ts * Dd);
    double nmax = ch.n_unit * rho / 2.0;
    nn = nn > nmax ? nmax : nn;
    nn = nn < 0.0 ? 0.0 : nn;
    return 2.0 * nn / ch.n_unit;
}

// Sec. 2.3: the speed sum of the CFL rule for one cell (FP64)
__device__ double cell_speed(double gamma, double rho, double mx, double my, double mz, double e, double bx,
                             double by, double bz)
{
    double vx = mx / rho, vy = my / rho, vz = mz / rho;
    double v = sqrt(vx * vx + vy * vy + vz * vz);
    double p = (gamma - 1.0) * e;
    double c2 = gamma * p / rho;
    double ca2 = bx * bx / rho;
    double b2 = (bx * bx + by * by + bz * bz) / rho;
    double s = c2 + b2;
    double disc = s * s - 4.0 * c2 * ca2;
    disc = disc < 0.0 ? 0.0 : disc;
    double sd = sqrt(disc);
    double cf2 = 0.5 * (s + sd);
    double cs2 = 0.5 * (s - sd);
    cs2 = cs2 < 0.0 ? 0.0 : cs2;
    return v + sqrt(b2) + sqrt(c2) + sqrt(ca2) + sqrt(cs2) + sqrt(cf2);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        double o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void block_max_store(double v, double* out)
{
    __shared__ double red[NTH / 64];
    v = wave_max(v);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < NTH / 64; w++) m = red[w] > m ? red[w] : m;
        out[blockIdx.x] = m;
    }
}

// Tail of the step (after ADV): H2 clamp to [0, rho], chemistry, dual-energy
// sync (Sec. 2.8, pressure-gated), validity flag, per-block CFL speed maximum.
// mode: 1 = full tail, 0 = speed only (state unchanged).
template <typename T>
__global__ __launch_bounds__(NTH) void k_tail(Geo g, Fields<T> U, StepArgs a, ChemArgs ch, int mode,
                                              double* __restrict__ part, uint32_t* flags)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    double spd = 0.0;
    if (c < g.n) {
        int i, j, k;
        decompose(g, c, i, j, k);
        double rho = (double)U.f[RHO][c];
        double mx = (double)U.f[MX][c], my = (double)U.f[MY][c], mz = (double)U.f[MZ][c];
        double E = (double)U.f[EN][c];
        double e = (double)U.f[EI][c];
        double bx = 0.5 * ((double)U.f[BX][c] + (double)U.f[BX][nbr<0>(g, c, i, j, k, 1)]);
        double by = 0.5 * ((double)U.f[BY][c] + (double)U.f[BY][nbr<1>(g, c, i, j, k, 1)]);
        double bz = 0.5 * ((double)U.f[BZ][c] + (double)U.f[BZ][nbr<2>(g, c, i, j, k, 1)]);
        if (mode == 1) {
            double h2 = (double)U.f[H2][c];
            h2 = h2 > rho ? rho : h2;
            h2 = h2 < 0.0 ? 0.0 : h2;
            if (ch.on) h2 = chem_h2(ch, a.gamma, rho, e, h2, step_dt(a));
            double K = 0.5 * (mx * mx + my * my + mz * mz) / rho;
            double M = 0.5 * (bx * bx + by * by + bz * bz);
            double ei = E - K - M;
            if (ei >= 1e-3 * E && (a.gamma - 1.0) * ei > M) e = ei;
            U.f[H2][c] = (T)h2;
            U.f[EI][c] = (T)e;
            e = (double)(T)e;
        }
        bool ok = rho > 0.0 && e > 0.0 && isfinite(rho) && isfinite(e) && isfinite(E) && isfinite(mx) &&
                  isfinite(my) && isfinite(mz) && isfinite(bx) && isfinite(by) && isfinite(bz);
        if (!ok) atomicOr(flags, 1u);
        spd = ok ? cell_speed(a.gamma, rho, mx, my, mz, e, bx, by, bz) : 0.0;
    }
    block_max_store(spd, part);
}

// dt = cfl h / max speed over the per-block maxima (max is exact, so the
// result equals the minimum over cells of cfl h / speed)
__global__ __launch_bounds__(1024) void k_reduce_dt(const double* __restrict__ part, int nparts, double cflh,
                                                    double* __restrict__ dt)
{
    __shared__ double red[16];
    double m = 0.0;
    for (int t = threadIdx.x; t < nparts; t += 1024) m = part[t] > m ? part[t] : m;
    m = wave_max(m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = red[0];
        for (int w = 1; w < 16; w++) r = red[w] > r ? red[w] : r;
        *dt = r > 0.0 ? cflh / r : 0.0;
    }
}

// FP64 totals: per-block fixed-order sums of the 10 fields
template <typename T>
__global__ __launch_bounds__(NTH) void k_totals_partial(Geo g, CFields<T> U, double* __restrict__ part)
{
    __shared__ double red[NF][NTH / 64];
    int c = blockIdx.x * NTH + threadIdx.x;
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int f = 0; f < NF; f++) {
        double v = c < g.n ? (double)U.f[f][c] : 0.0;
        v = wave_sum(v);
        if (lane == 0) red[f][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < NF) {
        double s = 0.0;
        for (int w = 0; w < NTH / 64; w++) s += red[threadIdx.x][w];
        part[(size_t)blockIdx.x * NF + threadIdx.x] = s;
    }
}

__global__ __launch_bounds__(1024) void k_totals_final(const double* __restrict__ part, int nparts,
                                                       double* __restrict__ out)
{
    __shared__ double red[NF][16];
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int f = 0; f < NF; f++) {
        double s = 0.0;
        for (int t = threadIdx.x; t < nparts; t += 1024) s += part[(size_t)t * NF + f];
        s = wave_sum(s);
        if (lane == 0) red[f][wv] = s;
    }
    __syncthreads();
    if (threadIdx.x < NF) {
        double s = 0.0;
        for (int w = 0; w < 16; w++) s += red[threadIdx.x][w];
        out[threadIdx.x] = s;
    }
}

// primitive (host order rho, vx, vy, vz, p, bx_f, by_f, bz_f, x_h2) -> conserved
template <typename T>
__global__ __launch_bounds__(NTH) void k_init(Geo g, const double* __restrict__ Wp, Fields<T> U, double gamma)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    int i, j, k;
    decompose(g, c, i, j, k);
    const size_t N = (size_t)g.n;
    double rho = Wp[c];
    double vx = Wp[N + c], vy = Wp[2 * N + c], vz = Wp[3 * N + c];
    double p = Wp[4 * N + c];
    double bxf = Wp[5 * N + c], byf = Wp[6 * N + c], bzf = Wp[7 * N + c];
    double bx = 0.5 * (bxf + Wp[5 * N + nbr<0>(g, c, i, j, k, 1)]);
    double by = 0.5 * (byf + Wp[6 * N + nbr<1>(g, c, i, j, k, 1)]);
    double bz = 0.5 * (bzf + Wp[7 * N + nbr<2>(g, c, i, j, k, 1)]);
    double e = p / (gamma - 1.0);
    U.f[RHO][c] = (T)rho;
    U.f[MX][c] = (T)(rho * vx);
    U.f[MY][c] = (T)(rho * vy);
    U.f[MZ][c] = (T)(rho * vz);
    U.f[EI][c] = (T)e;
    U.f[EN][c] = (T)(e + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bx * bx + by * by + bz * bz));
    U.f[BX][c] = (T)bxf;
    U.f[BY][c] = (T)byf;
    U.f[BZ][c] = (T)bzf;
    U.f[H2][c] = (T)(Wp[8 * N + c] * rho);
}

template <typename T>
__global__ __launch_bounds__(NTH) void k_from_f64(Geo g, const double* __restrict__ src, Fields<T> U)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    const size_t N = (size_t)g.n;
#pragma unroll
    for (int f = 0; f < NF; f++) U.f[f][c] = (T)src[f * N + c];
}

template <typename T>
__global__ __launch_bounds__(NTH) void k_to_f64(Geo g, CFields<T> U, double* __restrict__ dst)
{
    int c = blockIdx.x * NTH + threadIdx.x;
    if (c >= g.n) return;
    const size_t N = (size_t)g.n;
#pragma unroll
    for (int f = 0; f < NF; f++) dst[f * N + c] = (double)U.f[f][c];
}

__global__ void k_clear_flags(uint32_t* flags)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *flags = 0u;
}

}  // namespace

// ---------------------------------------------------------------- host runtime

struct mhd_box {
    mhd_params p;
    Geo g;
    hipStream_t s;
    int prec;          // MHD_FP64 / MHD_FP32_MIXED
    size_t esz;        // bytes per stored value
    int nblocks;
    char* slot[3];     // three Runge-Kutta copies of the 10 fields
    char* W;           // primitives, 8 x N
    char* F[3];        // per-direction face outputs, 7 x N each
    double* part;      // per-block partials: NF x nblocks
    uint32_t* flags;
    double* dt_dev;
    double* tot_dev;
    int cur[3];        // current slot of the groups H, M, B
    // per-launch event timing (mhd_set_timing)
    int timing;
    int nev;                    // event pairs recorded in the current step
    hipEvent_t ev[2 * 64];
    int evcls[64];
    int ev_ready;
    double tms[MHD_NKCLASS];
    int64_t tcnt[MHD_NKCLASS];
};

namespace {

enum { GH = 0, GM = 1, GB = 2 };
int group_of(int f)
{
    if (f == RHO || f == H2) return GH;
    if (f >= BX && f <= BZ) return GB;
    return GM;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t slot, W, F, part, misc, total;
};

bool valid_params(const mhd_params* p)
{
    if (!p) return false;
    for (int d = 0; d < 3; d++)
        if (p->n[d] < 1) return false;
    double n = (double)p->n[0] * p->n[1] * p->n[2];
    if (n >= 2147483647.0) return false;
    if (!(p->gamma > 1.0) || !std::isfinite(p->gamma)) return false;
    if (!(p->cfl > 0.0) || !std::isfinite(p->cfl)) return false;
    if (!(p->theta >= 0.0) || !std::isfinite(p->theta)) return false;
    if (p->precision != MHD_FP64 && p->precision != MHD_FP32_MIXED) return false;
    if (p->chemistry != 0 && p->chemistry != 1) return false;
    if (p->chemistry && !(p->n_unit_cm3 > 0.0 && p->T_unit_K > 0.0 && p->t_unit_s > 0.0)) return false;
    return true;
}

Layout layout_of(const mhd_params* p)
{
    Layout L;
    size_t N = (size_t)p->n[0] * p->n[1] * p->n[2];
    size_t esz = p->precision == MHD_FP64 ? 8 : 4;
    size_t nb = (N + NTH - 1) / NTH;
    L.slot = align256(NF * N * esz);
    L.W = align256(8 * N * esz);
    size_t fbytes = align256(NFACE * N * esz);
    // the face scratch doubles as host staging (9 or 10 FP64 fields)
    size_t stage = align256(10 * N * 8);
    L.F = 3 * fbytes > stage ? 3 * fbytes : stage;
    L.part = align256(nb * NF * sizeof(double));
    L.misc = 256 + 256 + 256;
    L.total = 3 * L.slot + L.W + L.F + L.part + L.misc;
    return L;
}

template <typename T>
Fields<T> view(mhd_box* b, int sH, int sM, int sB)
{
    Fields<T> v;
    size_t N = (size_t)b->g.n;
    for (int f = 0; f < NF; f++) {
        int grp = group_of(f);
        int s = grp == GH ? sH : (grp == GM ? sM : sB);
        v.f[f] = reinterpret_cast<T*>(b->slot[s]) + f * N;
    }
    return v;
}

template <typename T>
CFields<T> cview(const Fields<T>& v)
{
    CFields<T> c;
    for (int f = 0; f < NF; f++) c.f[f] = v.f[f];
    return c;
}

int launch_status() { return hipGetLastError() == hipSuccess ? MHD_OK : MHD_EDEVICE; }

StepArgs step_args(mhd_box* b, double dt, bool dev)
{
    StepArgs a;
    a.dt_val = dt;
    a.dt_dev = dev ? b->dt_dev : nullptr;
    a.gamma = b->p.gamma;
    a.h = 1.0 / (double)b->p.n[0];
    a.theta = b->p.theta;
    // the bound is computed from the stored state: FP32 storage moves it by ~1e-7
    a.cfl_tol = b->prec == MHD_FP64 ? 1e-12 : 1e-4;
    return a;
}

ChemArgs chem_args(mhd_box* b)
{
    ChemArgs c;
    c.on = b->p.chemistry;
    c.n_unit = b->p.n_unit_cm3;
    c.T_unit = b->p.T_unit_K;
    c.t_unit = b->p.t_unit_s;
    return c;
}

const RK rk_coef[3] = { { 0.0, 1.0 }, { 0.75, 0.25 }, { 1.0 / 3.0, 2.0 / 3.0 } };

struct Slots { int h, m, b; };

// event pair around one launch of class cls (no-op unless timing is on)
struct KTimer {
    mhd_box* b;
    int slot;
    KTimer(mhd_box* box, int cls) : b(box), slot(-1)
    {
        if (b->timing && b->nev < 64) {
            slot = b->nev++;
            b->evcls[slot] = cls;
            hipEventRecord(b->ev[2 * slot], b->s);
        }
    }
    ~KTimer()
    {
        if (slot >= 0) hipEventRecord(b->ev[2 * slot + 1], b->s);
    }
};

int timing_collect(mhd_box* b)
{
    if (!b->timing || b->nev == 0) return MHD_OK;
    if (hipEventSynchronize(b->ev[2 * (b->nev - 1) + 1]) != hipSuccess) return MHD_EDEVICE;
    for (int i = 0; i < b->nev; i++) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b->ev[2 * i], b->ev[2 * i + 1]) != hipSuccess) return MHD_EDEVICE;
        b->tms[b->evcls[i]] += ms;
        b->tcnt[b->evcls[i]] += 1;
    }
    b->nev = 0;
    return MHD_OK;
}

// x faces: whole rows per block when a row fits one block, else one face per thread
template <typename T>
void launch_nonadv_x(mhd_box* b, const T* W, const T* bx, T* F, const StepArgs& a)
{
    const int nx = b->g.nx;
    const int maxt = sizeof(T) == 8 ? 512 : 1024;
    if (nx <= maxt) {
        int rpb = nx >= 256 ? 1 : 256 / nx;
        int threads = rpb * nx;
        int rows = b->g.ny * b->g.nz;
        int blocks = (rows + rpb - 1) / rpb;
        size_t shm = (size_t)threads * 18 * sizeof(T);   // at most 72 KiB
        if (threads <= 256) {
            k_nonadv_xrows<T, 256><<<blocks, threads, shm, b->s>>>(b->g, W, bx, F, a, rpb);
        } else if (threads <= 512) {
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nonadv_xrows<T, 512>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            k_nonadv_xrows<T, 512><<<blocks, threads, shm, b->s>>>(b->g, W, bx, F, a, rpb);
        } else {
            hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nonadv_xrows<T, 1024>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
            k_nonadv_xrows<T, 1024><<<blocks, threads, shm, b->s>>>(b->g, W, bx, F, a, rpb);
        }
    } else {
        k_nonadv_face<T, 0><<<b->nblocks, NTH, 0, b->s>>>(b->g, W, bx, F, a);
    }
}

constexpr int MARCH_SEG = 32;

template <typename T, int D>
void launch_nonadv_march(mhd_box* b, const T* W, const T* bf, T* F, const StepArgs& a)
{
    const int nd = D == 1 ? b->g.ny : b->g.nz;
    const int no = D == 1 ? b->g.nz : b->g.ny;
    int seg = nd < MARCH_SEG ? nd : MARCH_SEG;
    long long threads = (long long)b->g.nx * no * ((nd + seg - 1) / seg);
    int blocks = (int)((threads + NTH - 1) / NTH);
    k_nonadv_march<T, D><<<blocks, NTH, 0, b->s>>>(b->g, W, bf, F, a, seg);
}

template <typename T>
int nonadv_substage(mhd_box* b, Slots sin, Slots sS, Slots sout, const StepArgs& a, RK rk, int dbg, bool first)
{
    dim3 grid(b->nblocks), blk(NTH);
    Fields<T> in = view<T>(b, sin.h, sin.m, sin.b);
    Fields<T> S = view<T>(b, sS.h, sS.m, sS.b);
    Fields<T> out = view<T>(b, sout.h, sout.m, sout.b);
    T* W = reinterpret_cast<T*>(b->W);
    T* F0 = reinterpret_cast<T*>(b->F[0]);
    T* F1 = reinterpret_cast<T*>(b->F[1]);
    T* F2 = reinterpret_cast<T*>(b->F[2]);
    {
        KTimer t(b, MHD_K_PRIM);
        k_prim<T><<<grid, blk, 0, b->s>>>(b->g, cview(in), W, a, b->flags, first ? b->dt_dev : nullptr);
    }
    {
        KTimer t(b, MHD_K_NONADV_FACE);
        launch_nonadv_x<T>(b, W, in.f[BX], F0, a);
    }
    {
        KTimer t(b, MHD_K_NONADV_FACE);
        launch_nonadv_march<T, 1>(b, W, in.f[BY], F1, a);
    }
    {
        KTimer t(b, MHD_K_NONADV_FACE);
        launch_nonadv_march<T, 2>(b, W, in.f[BZ], F2, a);
    }
    {
        KTimer t(b, MHD_K_NONADV_UPDATE);
        k_nonadv_update<T><<<grid, blk, 0, b->s>>>(b->g, cview(in), cview(S), out, F0, F1, F2, a, rk, dbg);
    }
    return launch_status();
}

template <typename T>
int adv_substage(mhd_box* b, Slots sin, Slots sS, Slots sout, const StepArgs& a, RK rk, int dbg)
{
    dim3 grid(b->nblocks), blk(NTH);
    Fields<T> in = view<T>(b, sin.h, sin.m, sin.b);
    Fields<T> S = view<T>(b, sS.h, sS.m, sS.b);
    Fields<T> out = view<T>(b, sout.h, sout.m, sout.b);
    T* F0 = reinterpret_cast<T*>(b->F[0]);
    T* F1 = reinterpret_cast<T*>(b->F[1]);
    T* F2 = reinterpret_cast<T*>(b->F[2]);
    {
        KTimer t(b, MHD_K_ADV_FACE);
        k_adv_face<T, 0><<<grid, blk, 0, b->s>>>(b->g, cview(in), F0, a);
    }
    {
        KTimer t(b, MHD_K_ADV_FACE);
        k_adv_face<T, 1><<<grid, blk, 0, b->s>>>(b->g, cview(in), F1, a);
    }
    {
        KTimer t(b, MHD_K_ADV_FACE);
        k_adv_face<T, 2><<<grid, blk, 0, b->s>>>(b->g, cview(in), F2, a);
    }
    {
        KTimer t(b, MHD_K_ADV_UPDATE);
        k_adv_update<T><<<grid, blk, 0, b->s>>>(b->g, cview(in), cview(S), out, F0, F1, F2, a, rk, dbg);
    }
    return launch_status();
}

// NONADV stage: the M and B groups each rotate through their three slots
// (stage start S, then A, B, A); H is read from its current slot.
template <typename T>
int nonadv_stage(mhd_box* b, const StepArgs& a, bool first)
{
    int h = b->cur[GH], Sm = b->cur[GM], Sb = b->cur[GB];
    Slots S0 = { h, Sm, Sb };
    Slots A = { h, (Sm + 1) % 3, (Sb + 1) % 3 };
    Slots B2 = { h, (Sm + 2) % 3, (Sb + 2) % 3 };
    int st;
    if ((st = nonadv_substage<T>(b, S0, S0, A, a, rk_coef[0], 0, first))) return st;
    if ((st = nonadv_substage<T>(b, A, S0, B2, a, rk_coef[1], 0, false))) return st;
    if ((st = nonadv_substage<T>(b, B2, S0, A, a, rk_coef[2], 0, false))) return st;
    b->cur[GM] = A.m;
    b->cur[GB] = A.b;
    return MHD_OK;
}

// ADV stage: the H and M groups rotate; B is read from its current slot
template <typename T>
int adv_stage(mhd_box* b, const StepArgs& a)
{
    int Sh = b->cur[GH], Sm = b->cur[GM], bb = b->cur[GB];
    Slots S0 = { Sh, Sm, bb };
    Slots A = { (Sh + 1) % 3, (Sm + 1) % 3, bb };
    Slots B2 = { (Sh + 2) % 3, (Sm + 2) % 3, bb };
    int st;
    if ((st = adv_substage<T>(b, S0, S0, A, a, rk_coef[0], 0))) return st;
    if ((st = adv_substage<T>(b, A, S0, B2, a, rk_coef[1], 0))) return st;
    if ((st = adv_substage<T>(b, B2, S0, A, a, rk_coef[2], 0))) return st;
    b->cur[GH] = A.h;
    b->cur[GM] = A.m;
    return MHD_OK;
}

template <typename T>
int tail(mhd_box* b, const StepArgs& a, int mode)
{
    Fields<T> u = view<T>(b, b->cur[GH], b->cur[GM], b->cur[GB]);
    {
        KTimer t(b, MHD_K_TAIL);
        k_tail<T><<<b->nblocks, NTH, 0, b->s>>>(b->g, u, a, chem_args(b), mode, b->part, b->flags);
    }
    double cflh = b->p.cfl * (1.0 / (double)b->p.n[0]);
    {
        KTimer t(b, MHD_K_REDUCE);
        k_reduce_dt<<<1, 1024, 0, b->s>>>(b->part, b->nblocks, cflh, b->dt_dev);
    }
    return launch_status();
}

template <typename T>
int full_step(mhd_box* b, double dt, bool dev)
{
    StepArgs a = step_args(b, dt, dev);
    int st;
    if ((st = nonadv_stage<T>(b, a, true))) return st;
    if ((st = adv_stage<T>(b, a))) return st;
    if ((st = tail<T>(b, a, 1))) return st;
    return timing_collect(b);
}

int sync_and_flags(mhd_box* b)
{
    uint32_t fl = 0;
    if (hipMemcpyAsync(&fl, b->flags, sizeof(fl), hipMemcpyDeviceToHost, b->s) != hipSuccess) return MHD_EDEVICE;
    if (hipStreamSynchronize(b->s) != hipSuccess) return MHD_EDEVICE;
    if (fl & 1u) return MHD_ENONPHYS;
    if (fl & 2u) return MHD_ECFL;
    return MHD_OK;
}

template <typename T>
int load_f64(mhd_box* b, const double* host, bool prim)
{
    size_t N = (size_t)b->g.n;
    double* stage = reinterpret_cast<double*>(b->F[0]);
    size_t nf = prim ? 9 : 10;
    if (hipMemcpyAsync(stage, host, nf * N * sizeof(double), hipMemcpyHostToDevice, b->s) != hipSuccess)
        return MHD_EDEVICE;
    b->cur[GH] = b->cur[GM] = b->cur[GB] = 0;
    Fields<T> u = view<T>(b, 0, 0, 0);
    if (prim)
        k_init<T><<<b->nblocks, NTH, 0, b->s>>>(b->g, stage, u, b->p.gamma);
    else
        k_from_f64<T><<<b->nblocks, NTH, 0, b->s>>>(b->g, stage, u);
    k_clear_flags<<<1, 64, 0, b->s>>>(b->flags);
    StepArgs a = step_args(b, 0.0, false);
    int st = tail<T>(b, a, 0);
    if (st) return st;
    if (hipStreamSynchronize(b->s) != hipSuccess) return MHD_EDEVICE;
    return MHD_OK;
}

template <typename T>
int get_f64(mhd_box* b, double* host)
{
    size_t N = (size_t)b->g.n;
    double* stage = reinterpret_cast<double*>(b->F[0]);
    Fields<T> u = view<T>(b, b->cur[GH], b->cur[GM], b->cur[GB]);
    k_to_f64<T><<<b->nblocks, NTH, 0, b->s>>>(b->g, cview(u), stage);
    if (launch_status()) return MHD_EDEVICE;
    if (hipMemcpyAsync(host, stage, NF * N * sizeof(double), hipMemcpyDeviceToHost, b->s) != hipSuccess)
        return MHD_EDEVICE;
    return sync_and_flags(b);
}

template <typename T>
int totals(mhd_box* b, double* out)
{
    Fields<T> u = view<T>(b, b->cur[GH], b->cur[GM], b->cur[GB]);
    k_totals_partial<T><<<b->nblocks, NTH, 0, b->s>>>(b->g, cview(u), b->part);
    k_totals_final<<<1, 1024, 0, b->s>>>(b->part, b->nblocks, b->tot_dev);
    if (launch_status()) return MHD_EDEVICE;
    if (hipMemcpyAsync(out, b->tot_dev, NF * sizeof(double), hipMemcpyDeviceToHost, b->s) != hipSuccess)
        return MHD_EDEVICE;
    return sync_and_flags(b);
}

template <typename T>
int debug_stage(mhd_box* b, int stage, double dt)
{
    StepArgs a = step_args(b, dt, false);
    switch (stage) {
    case MHD_STAGE_NONADV: return nonadv_stage<T>(b, a, false);
    case MHD_STAGE_ADV: return adv_stage<T>(b, a);
    case MHD_STAGE_TAIL: return tail<T>(b, a, 1);
    case MHD_STAGE_NONADV_RHS:
    case MHD_STAGE_ADV_RHS: {
        // tau R(U) of one substage into all ten fields of a free slot; needs
        // the three groups in one slot (true right after mhd_set_state)
        int S = b->cur[GM];
        if (b->cur[GH] != S || b->cur[GB] != S) return MHD_EINVAL;
        int O = (S + 1) % 3;
        Slots s0 = { S, S, S }, so = { O, O, O };
        int st = stage == MHD_STAGE_NONADV_RHS ? nonadv_substage<T>(b, s0, s0, so, a, rk_coef[0], 1, false)
                                               : adv_substage<T>(b, s0, s0, so, a, rk_coef[0], 1);
        if (st) return st;
        b->cur[GH] = b->cur[GM] = b->cur[GB] = O;
        return MHD_OK;
    }
    default: return MHD_EINVAL;
    }
}

}  // namespace

// ---------------------------------------------------------------- C ABI

extern "C" {

size_t mhd_workspace_bytes(const mhd_params* p)
{
    if (!valid_params(p)) return 0;
    return layout_of(p).total;
}

int mhd_create(const mhd_params* p, mhd_box** out)
{
    if (!out) return MHD_EINVAL;
    *out = nullptr;
    if (!valid_params(p)) return MHD_EINVAL;
    Layout L = layout_of(p);
    if (!p->workspace || p->workspace_bytes < L.total) return MHD_ENOMEM;
    if (((uintptr_t)p->workspace) & 255) return MHD_EINVAL;
    mhd_box* b = new (std::nothrow) mhd_box;
    if (!b) return MHD_ENOMEM;
    b->p = *p;
    b->g.nx = p->n[0];
    b->g.ny = p->n[1];
    b->g.nz = p->n[2];
    b->g.nxy = p->n[0] * p->n[1];
    b->g.n = p->n[0] * p->n[1] * p->n[2];
    b->s = reinterpret_cast<hipStream_t>(p->stream);
    b->prec = p->precision;
    b->esz = p->precision == MHD_FP64 ? 8 : 4;
    b->nblocks = (b->g.n + NTH - 1) / NTH;
    char* w = reinterpret_cast<char*>(p->workspace);
    for (int s = 0; s < 3; s++) {
        b->slot[s] = w;
        w += L.slot;
    }
    b->W = w;
    w += L.W;
    size_t fbytes = align256(NFACE * (size_t)b->g.n * b->esz);
    for (int d = 0; d < 3; d++) b->F[d] = w + d * fbytes;
    w += L.F;
    b->part = reinterpret_cast<double*>(w);
    w += L.part;
    b->flags = reinterpret_cast<uint32_t*>(w);
    b->dt_dev = reinterpret_cast<double*>(w + 256);
    b->tot_dev = reinterpret_cast<double*>(w + 512);
    b->cur[0] = b->cur[1] = b->cur[2] = 0;
    b->timing = 0;
    b->nev = 0;
    b->ev_ready = 0;
    for (int c = 0; c < MHD_NKCLASS; c++) {
        b->tms[c] = 0.0;
        b->tcnt[c] = 0;
    }
    *out = b;
    return MHD_OK;
}

int mhd_set_timing(mhd_box* b, int enable)
{
    if (!b) return MHD_EINVAL;
    if (enable && !b->ev_ready) {
        for (int i = 0; i < 2 * 64; i++)
            if (hipEventCreate(&b->ev[i]) != hipSuccess) return MHD_EDEVICE;
        b->ev_ready = 1;
    }
    b->timing = enable ? 1 : 0;
    b->nev = 0;
    for (int c = 0; c < MHD_NKCLASS; c++) {
        b->tms[c] = 0.0;
        b->tcnt[c] = 0;
    }
    return MHD_OK;
}

int mhd_get_timing(mhd_box* b, double* ms, int64_t* counts)
{
    if (!b || !ms || !counts) return MHD_EINVAL;
    int st = timing_collect(b);
    if (st) return st;
    for (int c = 0; c < MHD_NKCLASS; c++) {
        ms[c] = b->tms[c];
        counts[c] = b->tcnt[c];
    }
    return MHD_OK;
}

int mhd_init_state(mhd_box* b, const double* prim)
{
    if (!b || !prim) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? load_f64<double>(b, prim, true) : load_f64<float>(b, prim, true);
}

int mhd_set_state(mhd_box* b, const double* cons)
{
    if (!b || !cons) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? load_f64<double>(b, cons, false) : load_f64<float>(b, cons, false);
}

int mhd_get_state(mhd_box* b, double* cons_out)
{
    if (!b || !cons_out) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? get_f64<double>(b, cons_out) : get_f64<float>(b, cons_out);
}

int mhd_cfl_dt(mhd_box* b, double* dt_out)
{
    if (!b || !dt_out) return MHD_EINVAL;
    if (hipMemcpyAsync(dt_out, b->dt_dev, sizeof(double), hipMemcpyDeviceToHost, b->s) != hipSuccess)
        return MHD_EDEVICE;
    return sync_and_flags(b);
}

int mhd_step(mhd_box* b, double dt)
{
    if (!b || !std::isfinite(dt) || !(dt > 0.0)) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? full_step<double>(b, dt, false) : full_step<float>(b, dt, false);
}

int mhd_step_cfl(mhd_box* b)
{
    if (!b) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? full_step<double>(b, 0.0, true) : full_step<float>(b, 0.0, true);
}

int mhd_conserved_totals(mhd_box* b, double out[10])
{
    if (!b || !out) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? totals<double>(b, out) : totals<float>(b, out);
}

int mhd_debug_stage(mhd_box* b, int stage, double dt)
{
    if (!b) return MHD_EINVAL;
    if (stage != MHD_STAGE_TAIL && (!std::isfinite(dt) || !(dt > 0.0))) return MHD_EINVAL;
    if (stage == MHD_STAGE_TAIL && (!std::isfinite(dt) || dt < 0.0)) return MHD_EINVAL;
    return b->prec == MHD_FP64 ? debug_stage<double>(b, stage, dt) : debug_stage<float>(b, stage, dt);
}

int mhd_destroy(mhd_box* b)
{
    if (b && b->ev_ready)
        for (int i = 0; i < 2 * 64; i++) hipEventDestroy(b->ev[i]);
    delete b;
    return MHD_OK;
}

const char* mhd_strerror(int status)
{
    switch (status) {
    case MHD_OK: return "ok";
    case MHD_EINVAL: return "invalid argument";
    case MHD_ENOMEM: return "workspace missing or too small";
    case MHD_EDEVICE: return "HIP runtime error";
    case MHD_ECFL: return "time step above the CFL bound";
    case MHD_ENONPHYS: return "non-finite or non-positive density or internal energy";
    default: return "unknown status";
    }
}

}  // extern "C"
