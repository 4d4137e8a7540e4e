// Device-side arithmetic of the step: grid indexing, the local parabola
// (Sec. 2.1), the NONADV face Riemann solve (Sec. 2.4 and the eigenvector
// appendix), FP64 chemistry (Sec. 2.7, rate appendix), the CFL speed sum
// (Sec. 2.3) and wavefront reductions.  Included by mhd.hip only.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mhd {

constexpr int NTH = 256;           // threads per block for cell-parallel kernels
constexpr int NF = 11;             // conserved fields (the last, H+, used by the ionisation network)
constexpr int NFACE = 7;           // per-face outputs
enum { RHO = 0, MX, MY, MZ, EN, EI, BX, BY, BZ, H2, HP };

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

// ---------------------------------------------------------------- roots and reciprocals

// Square root, reciprocal square root and reciprocal used by the face solvers.
// FP64: the hardware estimate refined by Newton-Raphson steps, which converge
// quadratically, so the result lands within about one ulp of the correctly
// rounded value at a third of the instruction count of the library forms.
// Arguments are positive and normal (densities, pressures, squared speeds);
// root_nr(0) = 0.  FP32: the single hardware instruction (about one ulp).
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double h = 0.5 * x;
    double y = __builtin_amdgcn_rsq(x);
    double t = h * y;
    double e = fma(-t, y, 0.5);
    y = fma(y, e, y);
    t = h * y;
    e = fma(-t, y, 0.5);
    return fma(y, e, y);
}
// coupled iteration on sqrt(x) and 1/(2 sqrt(x)), then one correction of the
// root from its exact residual x - g^2
__device__ __forceinline__ double root_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}
__device__ __forceinline__ double rcp_nr(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rsqrt_nr(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float root_nr(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float rcp_nr(float b) { return __builtin_amdgcn_rcpf(b); }

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
    // q0 -/+ dm / 4 with one rounding each: dm / 2 is exact, and the fused
    // product (dm / 2) / 2 is the exact dm / 4 (inline constants only)
    const T hdm = T(0.5) * dm;
    T qLp = fma(T(-0.5), hdm, q0);
    T qRp = fma(T(0.5), hdm, q0);
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
        T eta = t * rcp_nr(d);
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
// (vn, vt1, vt2, Bt1, Bt2, p), the adiabatic index gm, or with ion the two
// cells' gamma_eff.  Outputs (7): momentum flux (normal, t1, t2),
// energy flux, face normal velocity, E along t1 (B_t2 U_n - B_n U_t2), E along
// t2 (B_n U_t1 - B_t1 U_n).
template <typename T>
__device__ __forceinline__ void face_solve(T rl, T pl, T b1l, T b2l, T rr, T pr, T b1r, T b2r, T bn,
                                           const Side<T>& L, const Side<T>& R, T gm, T gml, T gmr, bool ion, T ydx,
                                           T sl, T sr, T out[7])
{
    const T eps = Eps<T>::v;
    // face averages (sqrt(rho) weights, sl = root_nr(rl) and sr = root_nr(rr)
    // formed once per cell by the caller; cross weights for Bt); with the
    // ionisation network the adiabatic index is the cells' gamma_eff averaged
    // with the weights of p
    T iw = rcp_nr(sl + sr);
    T rho = (sl * rl + sr * rr) * iw;
    T p = (sl * pl + sr * pr) * iw;
    if (ion) gm = (sl * gml + sr * gmr) * iw;
    T bt1 = (sl * b1r + sr * b1l) * iw;
    T bt2 = (sl * b2r + sr * b2l) * iw;

    // eigen-structure (Sec. 2.3, 2.4, eigenvector appendix); every root and
    // reciprocal of rho and gamma p derives from their two reciprocal roots
    T rs = rsqrt_nr(rho);                // 1 / sqrt(rho)
    T irho = rs * rs;
    T srho = rho * rs;
    T gp = gm * p;
    T rg = rsqrt_nr(gp);                 // 1 / sqrt(gamma p) = 1 / (sqrt(rho) c)
    T c2 = gp * irho;
    T ca2 = bn * bn * irho;
    T b2 = (bn * bn + bt1 * bt1 + bt2 * bt2) * irho;
    T s = c2 + b2;
    T disc = fmax(s * s - T(4) * c2 * ca2, T(0));
    T sd = root_nr(disc);
    T cf2 = T(0.5) * (s + sd);
    T cs2 = fmax(T(0.5) * (s - sd), T(0));
    T cc = (gp * rg) * rs, ca = fabs(bn) * rs, cf = root_nr(cf2), cs = root_nr(cs2);
    const T r2i = T(0.70710678118654752440);
    T den = cf2 - cs2;
    T af = r2i, as = r2i;
    if (den > eps * s) {
        T iden = rcp_nr(den);
        af = root_nr(fmax(c2 - cs2, T(0)) * iden);
        as = root_nr(fmax(cf2 - c2, T(0)) * iden);
    }
    T by = r2i, bz = r2i;
    T btsq = bt1 * bt1 + bt2 * bt2;
    if (btsq > eps * (bn * bn + btsq + gm * p)) {
        T ibt = rsqrt_nr(btsq);
        by = bt1 * ibt;
        bz = bt2 * ibt;
    }
    T sg = bn >= T(0) ? T(1) : T(-1);

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
    T A = T(0.5) * (rho * (rg * rg));    // 1 / (2 c^2)
    T Bc = T(0.5) * rg;                  // 1 / (2 sqrt(rho) c)
    T Cc = T(0.5) * (rg * rg);           // 1 / (2 rho c^2)
    T Dc = r2i * rs;                     // 1 / sqrt(2 rho)
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
    T src = gp * rg;                     // sqrt(rho) c = sqrt(gamma p)
    T sr2 = r2i * srho;
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

// ---------------------------------------------------------------- FP64 per-cell physics

struct ChemArgs {
    int on;     // chemistry stage
    int cool;   // heating/cooling stage
    int ion;    // ionisation network (reactions 5-8, H+ field, gamma_eff)
    double n_unit, T_unit, t_unit;
};

// Sec. 4.3: effective adiabatic index (5 n_H + 5 n_e + 7 n_H2) / (3 n_H +
// 3 n_e + 5 n_H2) of a cell with the ionisation network (n_e = n_H+), the
// constant gamma without it
__device__ __forceinline__ double gamma_cell(int ion, double gamma, double rho, double h2, double hp)
{
    if (!ion) return gamma;
    double nH = rho - h2 - hp, nH2 = 0.5 * h2, ne = hp;
    return (5.0 * nH + 5.0 * ne + 7.0 * nH2) / (3.0 * nH + 3.0 * ne + 5.0 * nH2);
}

// rates of reactions 5-8 (appendix): cosmic-ray ionisation per H atom (s^-1),
// collisional ionisation (a polynomial in ln of T in eV), radiative and grain
// recombination (cm^3 s^-1, log = log10)
__device__ __forceinline__ double rate_k6(double T)
{
    const double l = log(T * 8.617333262e-5);
    const double c[9] = { -32.7, 13.5, -5.7, 1.5, -0.3, 3.4e-2, -2.6e-3, 1.1e-4, -2.1e-6 };
    double s = 0.0, lp = 1.0;
#pragma unroll
    for (int i = 0; i < 9; i++) {
        s += c[i] * lp;
        lp *= l;
    }
    return exp(s);
}

__device__ __forceinline__ double rate_k7(double T)
{
    double x = log10(T);
    double num = -10.78 + 4.68 * x - 0.87 * x * x + 0.08 * x * x * x - 3.87e-3 * x * x * x * x;
    double den = 1.0 - 0.38 * x + 0.06 * x * x - 5.1e-3 * x * x * x + 2.4e-4 * x * x * x * x;
    return pow(10.0, num / den);
}

__device__ __forceinline__ double rate_k8(double T)
{
    double inner = 1.0 + 5.087e2 * pow(T, 1.586e-2) * pow(10.0, -1.8892 - 4.4e-5 * log10(T));
    return 12.25e-14 / (1.0 + 8.074e-6 * pow(10.0, 2.756) * inner);
}

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

// Sec. 2 stage 5 and Sec. 2.8 with the appendix heating and cooling of
// reactions 1-4 (erg cm^-3 s^-1, x = log10(T / 1e4)): H2 formation heating
// 7.2e-12 erg per formed molecule (formation rate of reaction 1) thermalised
// by the fraction 1 / (1 + n_cr / n), n_cr = 10^(4 - 0.416 x - 0.327 x^2);
// photodissociation heating 6.4e-13 erg per event; the two cooling terms
// n_H2 L_H / (1 + L_H / L_L) of reactions 2 and 3.  In reaction 3's low-density
// limit k_H = k_H2 = 6.29e-15 * 1.38 f(T) / f(4500), f = sqrt(T) a exp(-a),
// a = 1 + 1 / (k_B T) with k_B T in eV, evaluated in logarithms.  Returns
// Gamma - Lambda.
__device__ double heat_cool(const ChemArgs& ch, double gamma, double rho, double e, double h2)
{
    const double kb_ev = 8.617333262e-5;
    double p = (gamma - 1.0) * e;
    double mu = 1.0 / (1.0 - 0.5 * (h2 / rho));
    double T = ch.T_unit * mu * p / rho;
    double nH = ch.n_unit * (rho - h2);
    double nH2 = ch.n_unit * h2 / 2.0;
    double n = nH + nH2;
    double x = log10(T / 1e4);
    double t2 = T / 100.0;
    double st2 = sqrt(t2);
    double k1b = 3e-17 * st2 / (1.0 + 0.4 * st2 + 0.2 * t2 + 0.08 * t2 * t2);
    double ncr = pow(10.0, 4.0 - 0.416 * x - 0.327 * x * x);
    double g1 = 7.2e-12 * (k1b * n * nH) / (1.0 + ncr / n);
    double g4 = 6.4e-13 * (3.3 * 1.7e-11) * nH2;
    double lh2 = (T > 1087.0) ? 3.9e-19 * exp(-6118.0 / T) : pow(10.0, -19.24 + 0.474 * x - 1.247 * x * x);
    double fl2 = (T > 4031.0) ? 1.38e-22 * exp(-9243.0 / T) : pow(10.0, -22.9 - 0.553 * x - 1.148 * x * x);
    double ll2 = (pow(nH2, 0.77) + 1.2 * pow(nH, 0.77)) * fl2;
    double l2 = nH2 * lh2 / (1.0 + lh2 / ll2);
    double a = 1.0 + 1.0 / (kb_ev * T);
    const double a45 = 1.0 + 1.0 / (kb_ev * 4500.0);
    double lnf = 0.5 * log(T) + log(a) - a;
    double lnf45 = 0.5 * log(4500.0) + log(a45) - a45;
    double ln_ll3 = log(8.18e-13) + log(n) + log(6.29e-15 * 1.38) + lnf - lnf45;
    double ln_lh3 = log(1.1e-13) - 6744.0 / T;
    double l3 = nH2 * exp(ln_lh3) / (1.0 + exp(ln_lh3 - ln_ll3));
    return (g1 + g4) - (l2 + l3);
}

// explicit Euler step of the internal energy over dt with Gamma - Lambda
// frozen; energy unit n_unit k_B T_unit; cooling stops at the internal energy
// of 10 K, or at e where the cell is already colder
__device__ double cooled_e(const ChemArgs& ch, double gamma, double rho, double e, double h2, double dt)
{
    const double kb = 1.380649e-16, t_floor = 10.0;
    double eu = ch.n_unit * kb * ch.T_unit;
    double de = dt * ch.t_unit * heat_cool(ch, gamma, rho, e, h2) / eu;
    double mu = 1.0 / (1.0 - 0.5 * (h2 / rho));
    double efloor = rho * t_floor / (ch.T_unit * mu * (gamma - 1.0));
    double lo = e < efloor ? e : efloor;
    double en = e + de;
    return en < lo ? lo : en;
}

// Sec. 2.7 with reactions 1-8 (ionisation network): semi-implicit updates of
// n_H2 and n_H+ = n_e from the state at the start of the step, n_H = n_u (rho
// - h2 - hp); H2 clamped to [0, n_u (rho - hp) / 2], then H+ to [0, n_u (rho -
// h2')]; temperature from gamma_eff and the mean mass 1 / (1 - x_H2/2 + x_H+)
__device__ void chem_ion(const ChemArgs& ch, double rho, double e, double h2, double hp, double dt, double& h2_out,
                         double& hp_out)
{
    double gam = gamma_cell(1, 0.0, rho, h2, hp);
    double p = (gam - 1.0) * e;
    double mu = 1.0 / (1.0 - 0.5 * (h2 / rho) + hp / rho);
    double T = ch.T_unit * mu * p / rho;
    double nH = ch.n_unit * (rho - h2 - hp);
    double nH2 = ch.n_unit * h2 / 2.0;
    double ne = ch.n_unit * hp;
    double n = nH + nH2 + ne;
    double ts = dt * ch.t_unit;
    double t2 = T / 100.0;
    double st2 = sqrt(t2);
    double k1b = 3e-17 * st2 / (1.0 + 0.4 * st2 + 0.2 * t2 + 0.08 * t2 * t2);
    double k2 = (T > 7390.0) ? 6.11e-14 * exp(-2.93e4 / T) : 2.67e-15 * exp(-(6750.0 / T) * (6750.0 / T));
    double k3 = (T > 7291.0) ? 5.22e-14 * exp(-3.22e4 / T)
                             : 3.17e-15 * exp(-(4060.0 / T) - (7500.0 / T) * (7500.0 / T));
    double k4 = 3.3 * 1.7e-11;
    double C = k1b * n * nH;
    double Dd = k2 * nH + k3 * nH2 + k4;
    double m2 = nH2 + ts * (C - Dd * nH2) / (1.0 + ts * Dd);
    double m2max = ch.n_unit * (rho - hp) / 2.0;
    m2 = m2 > m2max ? m2max : m2;
    m2 = m2 < 0.0 ? 0.0 : m2;
    double Ci = 6e-18 * nH + rate_k6(T) * nH * ne;
    double Di = (rate_k7(T) + rate_k8(T)) * ne;
    double mi = ne + ts * (Ci - Di * ne) / (1.0 + ts * Di);
    double h2n = 2.0 * m2 / ch.n_unit;
    double mimax = ch.n_unit * (rho - h2n);
    mi = mi > mimax ? mimax : mi;
    mi = mi < 0.0 ? 0.0 : mi;
    h2_out = h2n;
    hp_out = mi / ch.n_unit;
}

// heating/cooling with the ionisation network: the terms of reactions 1-4
// with gamma_eff, the ion mean mass and n = n_H + n_H2 + n_H+, plus cosmic-ray
// heating 1.92e-28 n and collisional-ionisation cooling 2.18e-11 erg k6 n_H n_e
__device__ double heat_cool_ion(const ChemArgs& ch, double rho, double e, double h2, double hp)
{
    const double kb_ev = 8.617333262e-5;
    double gam = gamma_cell(1, 0.0, rho, h2, hp);
    double p = (gam - 1.0) * e;
    double mu = 1.0 / (1.0 - 0.5 * (h2 / rho) + hp / rho);
    double T = ch.T_unit * mu * p / rho;
    double nH = ch.n_unit * (rho - h2 - hp);
    double nH2 = ch.n_unit * h2 / 2.0;
    double ne = ch.n_unit * hp;
    double n = nH + nH2 + ne;
    double x = log10(T / 1e4);
    double t2 = T / 100.0;
    double st2 = sqrt(t2);
    double k1b = 3e-17 * st2 / (1.0 + 0.4 * st2 + 0.2 * t2 + 0.08 * t2 * t2);
    double ncr = pow(10.0, 4.0 - 0.416 * x - 0.327 * x * x);
    double g1 = 7.2e-12 * (k1b * n * nH) / (1.0 + ncr / n);
    double g4 = 6.4e-13 * (3.3 * 1.7e-11) * nH2;
    double lh2 = (T > 1087.0) ? 3.9e-19 * exp(-6118.0 / T) : pow(10.0, -19.24 + 0.474 * x - 1.247 * x * x);
    double fl2 = (T > 4031.0) ? 1.38e-22 * exp(-9243.0 / T) : pow(10.0, -22.9 - 0.553 * x - 1.148 * x * x);
    double ll2 = (pow(nH2, 0.77) + 1.2 * pow(nH, 0.77)) * fl2;
    double l2 = nH2 * lh2 / (1.0 + lh2 / ll2);
    double a = 1.0 + 1.0 / (kb_ev * T);
    const double a45 = 1.0 + 1.0 / (kb_ev * 4500.0);
    double lnf = 0.5 * log(T) + log(a) - a;
    double lnf45 = 0.5 * log(4500.0) + log(a45) - a45;
    double ln_ll3 = log(8.18e-13) + log(n) + log(6.29e-15 * 1.38) + lnf - lnf45;
    double ln_lh3 = log(1.1e-13) - 6744.0 / T;
    double l3 = nH2 * exp(ln_lh3) / (1.0 + exp(ln_lh3 - ln_ll3));
    double g5 = 1.92e-28 * n;
    double l6 = 2.18e-11 * rate_k6(T) * nH * ne;
    return (g1 + g4 + g5) - (l2 + l3 + l6);
}

__device__ double cooled_e_ion(const ChemArgs& ch, double rho, double e, double h2, double hp, double dt)
{
    const double kb = 1.380649e-16, t_floor = 10.0;
    double eu = ch.n_unit * kb * ch.T_unit;
    double de = dt * ch.t_unit * heat_cool_ion(ch, rho, e, h2, hp) / eu;
    double mu = 1.0 / (1.0 - 0.5 * (h2 / rho) + hp / rho);
    double efloor = rho * t_floor / (ch.T_unit * mu * (gamma_cell(1, 0.0, rho, h2, hp) - 1.0));
    double lo = e < efloor ? e : efloor;
    double en = e + de;
    return en < lo ? lo : en;
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

template <int NT = NTH>
__device__ __forceinline__ void block_max_store(double v, double* out, int blk)
{
    __shared__ double red[NT / 64];
    v = wave_max(v);
    int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) red[wv] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < NT / 64; w++) m = red[w] > m ? red[w] : m;
        out[blk] = m;
    }
}


}  // namespace mhd
