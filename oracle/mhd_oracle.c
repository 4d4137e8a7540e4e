/*
 * Plain FP64 CPU oracle for one operator-split step of ideal MHD with H/H2
 * chemistry on a uniform periodic grid (Kulikov, Chernykh & Protasov,
 * "A new code for numerical simulation of MHD astrophysical flows with
 * chemistry", arXiv:1608.08748).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker for the HIP library:
 * only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header, table or helper with the
 * GPU path.  It is written to be read against the paper: scalar loops, one
 * function per step of the method, every intermediate stored, no blocking or
 * fusion.
 *
 * Stage names.  The paper calls the pressure / Lorentz-force / p dV stage the
 * "eulerian" stage (Sec. 2, stage 1; Sec. 2.4) and the advection stage the
 * "lagrangian" stage (Sec. 2, stage 3; Sec. 2.6).  Here they are NONADV and
 * ADV respectively.
 *
 * Readings of passages that are ambiguous or garbled in the paper (each is
 * also listed in the design notes of the repository):
 *   R-dq     Sec. 2.1: dq = qR - qL (the printed qL - qR contradicts the
 *            parabola formula and the overshoot tests).
 *   R-step4w Sec. 2.1 Step 4: q_final = (1-w) q + w q^+ (w -> 1 only at
 *            discontinuities); the printed weights are swapped.
 *   R-step4c Sec. 2.1 Step 4: the "q_{i+1} q_{i-1} > 0" test is read as a
 *            test on the second differences, d2 q_{i+1} d2 q_{i-1} > 0.
 *   R-d2     Sec. 2.1 Step 4: d2 q_j = (q_{j+1} - 2 q_j + q_{j-1}) / (6 h^2);
 *            the h^2 of eta cancels, so eta = -(D_{i+1}-D_{i-1})/(6 (q_{i+1}-q_{i-1}))
 *            with D_j the plain second difference.
 *   R-rk     Sec. 2.2: the three-stage SSP Runge-Kutta formulas, written in
 *            increment form Q_s = Q_{s-1} + a_s (Q_0 - Q_{s-1}) + b_s tau R(Q_{s-1}).
 *   R-theta  Sec. 2.4: the parabola-average width is theta * |lambda| * tau,
 *            theta = 1 being the paper's literal choice; tau is the full step
 *            in every Runge-Kutta substage.
 *   R-avg    Sec. 2.4 face averages: left/right inputs are cell-centre values;
 *            pressure uses the sqrt(rho) weights of the velocity.
 *   R-b      Sec. 2.3: b = |B| / sqrt(rho) (the only reading under which the
 *            printed eigenvectors diagonalise the Jacobian).
 *   R-ab     Sec. 2.4 alpha/beta cases: alpha from the general formula when
 *            cf^2 - cs^2 > eps (c^2 + b^2), else 1/sqrt(2); beta = Bt/|Bt| when
 *            |Bt|^2 > eps (|B|^2 + gamma p), else 1/sqrt(2); sign(0) = +1.
 *   R-bn     Sec. 2.4/2.5: the normal field at a face is the staggered face
 *            value; transverse fields come from cell centres.
 *   R-proj   Appendix (eigenvectors): the face state is the projector sum
 *            q = sum_k r_k (l_k . q_up(k)); the expanded closed forms of the
 *            appendix carry sign/factor typos and are not used.
 *   R-adv    Sec. 2.6: lambda = |v_n| with v_n the sqrt(rho)-weighted face
 *            normal velocity of the current substage.
 *   R-ct     Sec. 2.5: the face-field update is part of the NONADV
 *            Runge-Kutta state; each substage uses its own face states.
 *   R-flux   Sec. 2 eqs. without advective terms: momentum flux
 *            (P* - bn^2, -bn Bt1, -bn Bt2), energy flux P* Vn - bn (B.V),
 *            internal energy source -(gamma-1) e div(V) from face velocities.
 *   R-reg    Sec. 2.8: dual-energy synchronisation only: e = E-K-M where
 *            E-K-M >= 1e-3 E and the pressure (gamma-1)(E-K-M) exceeds the
 *            magnetic pressure M = B^2/2; elsewhere e is kept.  Velocities are
 *            not changed.  The pressure gate is needed for the scheme to stay
 *            stable at low beta: the split moves the magnetic part of E with
 *            the Riemann velocity in NONADV but with the averaged velocity in
 *            ADV, and an unconditional sync feeds that mismatch into the
 *            pressure (it oscillates on the paper's shock tube of Sec. 3.1).
 *   R-chem   Sec. 2.7 + Appendix rates: H/H2 (reactions 1-4); n_H =
 *            n_u (rho - h2), n_H2 = n_u h2 / 2, C = k1 n_H^2 with k1 carrying its
 *            n/n_H factor (evaluated as k1' n n_H), D = k2 n_H + k3 n_H2 + k4,
 *            k4 optically thin; one semi-implicit update per step.
 *   R-units  Code units: n_u H nuclei per cm^3 per unit density, T = T_u mu p / rho
 *            with mu = 1 / (1 - x_H2/2), time unit t_u seconds.
 *   R-cfl    Sec. 2.3: verbatim speed sum v + b + c + c_a + c_s + c_f with
 *            c_a from the x component of the cell-centre field.
 *   R-cool   Sec. 2 stage 5, Sec. 2.8 and the appendix heating/cooling of
 *            reactions 1-4: the stage runs after chemistry and before
 *            regularisation; Gamma - Lambda is evaluated once per cell at the
 *            state entering it and held over tau (explicit Euler); the code
 *            energy density unit is n_u k_B T_u; cooling never takes e below
 *            the internal energy at 10 K (or below e if already colder); E
 *            gets the change e took.  x = log10(T / 1e4).  Gamma1 = 7.2e-12 erg
 *            x (formation rate C of reaction 1) / (1 + n_cr / n) with
 *            n_cr = 10^(4 - 0.416 x - 0.327 x^2) (the printed form drops the
 *            rate and the power of ten).  Lambda2 verbatim.  Lambda3: k_H is
 *            undefined in print and read as k_H = k_H2; f(T) = sqrt(T) a
 *            exp(-a) with a = 1 + 1/(k_B T), k_B T in eV (the printed exp(+a)
 *            grows without bound as T -> 0, unlike an excitation rate, and
 *            gives cooling times of 1e7 s at 700 K).  Gamma4 = 6.4e-13 erg k4
 *            n_H2.  The terms of reactions 5-8 come with the ionisation
 *            network (R-ion).
 *   R-grav   Sec. 2 equations, Sec. 2.4 and Sec. 2.9: Laplace(Phi) = 4 pi G
 *            rho; in harmonic space Phi_hat = -(2/3) pi G h^2 rho_hat /
 *            (1 - prod_d (3 - 2 sin^2(pi m_d / n_d)) / 3) (the printed form
 *            lacks the minus sign and G: it would put potential maxima on
 *            density peaks), the zero mode set to zero (periodic box);
 *            discrete Fourier transform of the periodic grid.  The potential
 *            is that of the current density: the Poisson stage ends one step
 *            and NONADV of the next reads it; rho does not change inside
 *            NONADV.  Sources in every NONADV substage: -rho grad(Phi) on m,
 *            -m . grad(Phi) on E, central differences (2h).  G in code
 *            units is G_cgs n_u m_H t_u^2.
 *   R-ion    Sec. 4.3 + Appendix, reactions 5-8 (optional): H+ mass density
 *            hp advected with the other ADV fields, n_e = n_H+ = n_u hp,
 *            n_H = n_u (rho - h2 - hp), mean mass 1 / (1 - x_H2/2 + x_H+);
 *            gamma_eff = (5 n_H + 5 n_e + 7 n_H2) / (3 n_H + 3 n_e + 5 n_H2) as
 *            printed, per cell in p = (gamma - 1) e, the sound speed, the e
 *            source, CFL and regularisation, the face value the sqrt(rho)-
 *            weighted mean of the two cells'.  k5 = 6e-18 s^-1 per H atom; k6 the
 *            printed polynomial in ln(T in eV); k7 and k8 as printed with log =
 *            log10.  H+: C = k5 n_H + k6 n_H n_e, D = (k7 + k8) n_e, semi-
 *            implicit with n_H, n_e frozen; H2 updated alongside with
 *            n_H excluding the ions; n = n_H + n_H2 + n_H+.
 *
 * Layout: the state is 11 structure-of-arrays fields of nx*ny*nz doubles,
 * x fastest: rho, mx, my, mz, E, e (= rho eps), bx, by, bz, h2 (= rho_H2),
 * hp (= rho_H+, zero and untouched without the ionisation network).
 * bx[i,j,k] is B_x on the face (i-1/2, j, k); by and bz likewise on the lower
 * y and z faces of the cell.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stddef.h>

#define ORC_PI 3.14159265358979323846

enum { F_RHO = 0, F_MX, F_MY, F_MZ, F_E, F_EI, F_BX, F_BY, F_BZ, F_H2, F_HP, NF };

typedef struct {
    int nx, ny, nz;
    double gamma;
    double cfl;
    double theta;
    int chemistry;
    int cooling;     /* subgrid heating/cooling stage (Sec. 2.8) on/off */
    int ionisation;  /* reactions 5-8 with H+ and e-, effective adiabatic index (Sec. 4.3) */
    double grav_G;   /* gravitational constant in code units; 0 = no self-gravity */
    double n_unit;   /* H nuclei per cm^3 per unit code density */
    double T_unit;   /* K: T = T_unit * mu * p / rho            */
    double t_unit;   /* s per code time unit                    */
} orc_params;

/* ------------------------------------------------------------------ */
/* indexing on the periodic grid                                        */
/* ------------------------------------------------------------------ */
static int wrap(int i, int n) { i %= n; return i < 0 ? i + n : i; }

static size_t cell(const orc_params *P, int i, int j, int k)
{
    return (size_t)wrap(i, P->nx) + (size_t)P->nx *
           ((size_t)wrap(j, P->ny) + (size_t)P->ny * (size_t)wrap(k, P->nz));
}

static size_t ncell(const orc_params *P)
{
    return (size_t)P->nx * (size_t)P->ny * (size_t)P->nz;
}

/* ------------------------------------------------------------------ */
/* Sec. 2.1: local parabola on a 5-cell line q[0..4] = q_{i-2..i+2}.    */
/* out = (qL, qR, dq, q6).                                              */
/* ------------------------------------------------------------------ */

/* Step 1: limited central difference delta_m q_j from q_{j-1}, q_j, q_{j+1}. */
static double limited_slope(double qm, double q0, double qp)
{
    double dq = 0.5 * (qp - qm);
    if ((qp - q0) * (q0 - qm) > 0.0) {
        double m = fabs(dq);
        double a = 2.0 * fabs(qp - q0);
        double b = 2.0 * fabs(q0 - qm);
        if (a < m) m = a;
        if (b < m) m = b;
        return dq >= 0.0 ? m : -m;
    }
    return 0.0;
}

/* Step 1: fourth-order interface value q_{j+1/2} = 1/2 (q_j + q_{j+1}) - 1/6 (dm_{j+1} - dm_j). */
static double interface_value(double q0, double q1, double dm0, double dm1)
{
    return 0.5 * (q0 + q1) - (1.0 / 6.0) * (dm1 - dm0);
}

void orc_parabola(const double q[5], double out[4])
{
    const double qmm = q[0], qm = q[1], q0 = q[2], qp = q[3], qpp = q[4];

    /* Step 1 */
    double dm_m = limited_slope(qmm, qm, q0);
    double dm_0 = limited_slope(qm, q0, qp);
    double dm_p = limited_slope(q0, qp, qpp);
    double qL = interface_value(qm, q0, dm_m, dm_0);
    double qR = interface_value(q0, qp, dm_0, dm_p);

    /* Step 2: parabola parameters and monotonicity of the edge values */
    double dq = qR - qL;
    double q6 = 6.0 * (q0 - 0.5 * (qL + qR));
    if ((qL - q0) * (q0 - qR) <= 0.0) {
        qL = q0;
        qR = q0;
    } else if (dq * q6 > dq * dq) {
        qL = 3.0 * q0 - 2.0 * qR;
    } else if (dq * q6 < -(dq * dq)) {
        qR = 3.0 * q0 - 2.0 * qL;
    }

    /* Step 3: parameters from the new edge values (Step 5 recomputes them
     * again after Step 4, so their values here are not used further). */

    /* Step 4: discontinuity detector and blend */
    double qLp = q0 - 0.25 * dm_0;
    double qRp = q0 + 0.25 * dm_0;
    double D_m = q0 - 2.0 * qm + qmm;       /* second difference at i-1 */
    double D_p = qpp - 2.0 * qp + q0;       /* second difference at i+1 */
    double eta = 0.0;
    double aqp = fabs(qp), aqm = fabs(qm);
    double mn = aqp;
    if (aqm < mn) mn = aqm;
    if (aqp + aqm < mn) mn = aqp + aqm;
    /* d2 q_j = D_j / (6 h^2): the h^2 cancels in eta and the sign test is scale free */
    int zero_eta = (fabs(qp - qm) - 0.01 * mn <= 0.0) || (D_p * D_m > 0.0);
    if (!zero_eta)
        eta = -(D_p - D_m) / (6.0 * (qp - qm));
    double w = 20.0 * (eta - 0.05);
    if (w > 1.0) w = 1.0;
    if (w < 0.0) w = 0.0;
    qL = (1.0 - w) * qL + w * qLp;
    qR = (1.0 - w) * qR + w * qRp;

    /* Step 5 */
    dq = qR - qL;
    q6 = 6.0 * (q0 - 0.5 * (qL + qR));

    out[0] = qL;
    out[1] = qR;
    out[2] = dq;
    out[3] = q6;
}

/* Sec. 2.4: average of the parabola over the right part of the cell of
 * relative width y (the paper's q(-nu t)). */
double orc_avg_right(const double par[4], double y)
{
    return par[1] - 0.5 * y * (par[2] - par[3] * (1.0 - (2.0 / 3.0) * y));
}

/* Sec. 2.4: average over the left part of relative width y (q(+nu t)). */
double orc_avg_left(const double par[4], double y)
{
    return par[0] + 0.5 * y * (par[2] + par[3] * (1.0 - (2.0 / 3.0) * y));
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3 / 2.4 / Appendix: eigen-structure of the NONADV Jacobian at a */
/* face for q = (vn, vt1, vt2, Bt1, Bt2, p).                             */
/* R is stored row-major with R[i*6+k] = component i of right vector k.  */
/* L is stored row-major with L[k*6+j] = component j of left vector k.   */
/* ------------------------------------------------------------------ */
void orc_eigen(double rho, double p, double bn, double bt1, double bt2,
               double gamma, double eps, double lam[6], double R[36], double L[36])
{
    double c2 = gamma * p / rho;
    double ca2 = bn * bn / rho;
    double b2 = (bn * bn + bt1 * bt1 + bt2 * bt2) / rho;
    double s = c2 + b2;
    double disc = s * s - 4.0 * c2 * ca2;
    if (disc < 0.0) disc = 0.0;
    double sd = sqrt(disc);
    double cf2 = 0.5 * (s + sd);
    double cs2 = 0.5 * (s - sd);
    if (cs2 < 0.0) cs2 = 0.0;
    double c = sqrt(c2), ca = sqrt(ca2), cf = sqrt(cf2), cs = sqrt(cs2);

    double af, as;
    double den = cf2 - cs2;
    if (den > eps * s) {
        double nf = c2 - cs2, ns = cf2 - c2;
        if (nf < 0.0) nf = 0.0;
        if (ns < 0.0) ns = 0.0;
        af = sqrt(nf / den);
        as = sqrt(ns / den);
    } else {
        af = 1.0 / sqrt(2.0);
        as = 1.0 / sqrt(2.0);
    }
    double by, bz;
    double bt2sq = bt1 * bt1 + bt2 * bt2;
    if (bt2sq > eps * (bn * bn + bt2sq + gamma * p)) {
        double bt = sqrt(bt2sq);
        by = bt1 / bt;
        bz = bt2 / bt;
    } else {
        by = 1.0 / sqrt(2.0);
        bz = 1.0 / sqrt(2.0);
    }
    double sg = bn >= 0.0 ? 1.0 : -1.0;
    double sr = sqrt(rho);
    double gp = gamma * p;
    double r2 = sqrt(2.0);
    double sr2 = sqrt(rho / 2.0);
    double s2r = sqrt(2.0 * rho);

    lam[0] = cf;  lam[1] = -cf;
    lam[2] = cs;  lam[3] = -cs;
    lam[4] = ca;  lam[5] = -ca;

    /* right eigenvectors: columns of R (rows of the printed transpose) */
    double RT[6][6] = {
        {  af * cf, -as * cs * by * sg, -as * cs * bz * sg,  as * sr * c * by,  as * sr * c * bz, af * gp },
        { -af * cf,  as * cs * by * sg,  as * cs * bz * sg,  as * sr * c * by,  as * sr * c * bz, af * gp },
        {  as * cs,  af * cf * by * sg,  af * cf * bz * sg, -af * sr * c * by, -af * sr * c * bz, as * gp },
        { -as * cs, -af * cf * by * sg, -af * cf * bz * sg, -af * sr * c * by, -af * sr * c * bz, as * gp },
        {  0.0, -bz / r2 * sg,  by / r2 * sg,  sr2 * bz, -sr2 * by, 0.0 },
        {  0.0, -bz / r2 * sg,  by / r2 * sg, -sr2 * bz,  sr2 * by, 0.0 },
    };
    double tc2 = 2.0 * c2;
    double src = 2.0 * sr * c;
    double rc2 = 2.0 * rho * c2;
    double Lm[6][6] = {
        {  af * cf / tc2, -as * cs * by / tc2 * sg, -as * cs * bz / tc2 * sg,  as * by / src,  as * bz / src, af / rc2 },
        { -af * cf / tc2,  as * cs * by / tc2 * sg,  as * cs * bz / tc2 * sg,  as * by / src,  as * bz / src, af / rc2 },
        {  as * cs / tc2,  af * cf * by / tc2 * sg,  af * cf * bz / tc2 * sg, -af * by / src, -af * bz / src, as / rc2 },
        { -as * cs / tc2, -af * cf * by / tc2 * sg, -af * cf * bz / tc2 * sg, -af * by / src, -af * bz / src, as / rc2 },
        {  0.0, -bz / r2 * sg,  by / r2 * sg,  bz / s2r, -by / s2r, 0.0 },
        {  0.0, -bz / r2 * sg,  by / r2 * sg, -bz / s2r,  by / s2r, 0.0 },
    };
    for (int i = 0; i < 6; i++)
        for (int k = 0; k < 6; k++) {
            R[i * 6 + k] = RT[k][i];
            L[k * 6 + i] = Lm[k][i];
        }
}

/* ------------------------------------------------------------------ */
/* Sec. 2.4: linearised Riemann problem with parabolic data at one face. */
/* cl, cr: cell-centre (rho, vn, vt1, vt2, Bt1, Bt2, p) of the two cells. */
/* parl, parr: parabolas (4 numbers each) of the 6 variables             */
/* (vn, vt1, vt2, Bt1, Bt2, p) of the left and right cells.               */
/* bn: face normal field.  ydx = theta * tau / h.                        */
/* out: (Vn, Vt1, Vt2, Bt1, Bt2, P) at the face.                          */
/* ------------------------------------------------------------------ */
void orc_riemann_face(const double cl[7], const double cr[7],
                      const double parl[24], const double parr[24],
                      double bn, double gamma, double eps, double ydx, double out[6])
{
    double sl = sqrt(cl[0]), srr = sqrt(cr[0]);
    double w = sl + srr;
    double rho = (sl * cl[0] + srr * cr[0]) / w;
    double p = (sl * cl[6] + srr * cr[6]) / w;
    /* cross-weighted transverse field */
    double bt1 = (sl * cr[4] + srr * cl[4]) / w;
    double bt2 = (sl * cr[5] + srr * cl[5]) / w;

    double lam[6], R[36], L[36];
    orc_eigen(rho, p, bn, bt1, bt2, gamma, eps, lam, R, L);

    double s[6];
    for (int k = 0; k < 6; k++) {
        double qup[6];
        /* waves 1,3,5 (positive speed) read the left cell, 2,4,6 the right cell */
        double nu = fabs(lam[k]);
        double y = ydx * nu;
        for (int j = 0; j < 6; j++)
            qup[j] = (k % 2 == 0) ? orc_avg_right(parl + 4 * j, y)
                                  : orc_avg_left(parr + 4 * j, y);
        double acc = 0.0;
        for (int j = 0; j < 6; j++)
            acc += L[k * 6 + j] * qup[j];
        s[k] = acc;
    }
    for (int i = 0; i < 6; i++) {
        double acc = 0.0;
        for (int k = 0; k < 6; k++)
            acc += R[i * 6 + k] * s[k];
        out[i] = acc;
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 2 (equation of state, field projection of Sec. 2.5)             */
/* ------------------------------------------------------------------ */

/* Sec. 4.3: effective adiabatic index (5 n_H + 5 n_e + 7 n_H2) / (3 n_H + 3 n_e + 5 n_H2)
 * with the ionisation network, the constant gamma without it */
double orc_gamma_cell(const orc_params *P, double rho, double h2, double hp)
{
    if (!P->ionisation) return P->gamma;
    double nH = rho - h2 - hp, nH2 = 0.5 * h2, ne = hp;   /* in units of n_u */
    return (5.0 * nH + 5.0 * ne + 7.0 * nH2) / (3.0 * nH + 3.0 * ne + 5.0 * nH2);
}

/* mean particle mass in m_H: rho / (n_H + n_H2 + n_H+ + n_e) per unit n_u */
static double mean_mass(double rho, double h2, double hp)
{
    return 1.0 / (1.0 - 0.5 * (h2 / rho) + hp / rho);
}

/* primitive state of one cell: rho, vx, vy, vz, Bcx, Bcy, Bcz, p, gamma */
static void cell_primitives(const orc_params *P, const double *U, int i, int j, int k, double w[9])
{
    size_t N = ncell(P);
    size_t c = cell(P, i, j, k);
    double rho = U[F_RHO * N + c];
    w[0] = rho;
    w[1] = U[F_MX * N + c] / rho;
    w[2] = U[F_MY * N + c] / rho;
    w[3] = U[F_MZ * N + c] / rho;
    w[4] = 0.5 * (U[F_BX * N + c] + U[F_BX * N + cell(P, i + 1, j, k)]);
    w[5] = 0.5 * (U[F_BY * N + c] + U[F_BY * N + cell(P, i, j + 1, k)]);
    w[6] = 0.5 * (U[F_BZ * N + c] + U[F_BZ * N + cell(P, i, j, k + 1)]);
    w[8] = orc_gamma_cell(P, rho, U[F_H2 * N + c], U[F_HP * N + c]);
    w[7] = (w[8] - 1.0) * U[F_EI * N + c];
}

/* direction d: normal axis d, transverse t1 = d+1, t2 = d+2 (cyclic) */
static void unit_offset(int d, int o[3]) { o[0] = o[1] = o[2] = 0; o[d] = 1; }

/* ------------------------------------------------------------------ */
/* NONADV right-hand side (Sec. 2.4, 2.5) for one Runge-Kutta substage.  */
/* U: current substage state.  inc: tau * R(U) for mx,my,mz,E,e,bx,by,bz */
/* stored in the field slots of a 10-field array (rho, h2 slots zero).   */
/* ------------------------------------------------------------------ */
void orc_potential(const orc_params *P, const double *rho, double *phi);

static void nonadv_increment(const orc_params *P, const double *U, double dt, double *inc)
{
    const size_t N = ncell(P);
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const double h = 1.0 / (double)nx;
    const double dtdx = dt / h;
    const double ydx = P->theta * dtdx;
    const double gm = P->gamma;
    const double eps = 1e-12;

    double *W = (double *)malloc(sizeof(double) * 9 * N);
    /* face states per direction: Vn, Vt1, Vt2, Bt1, Bt2, P (6 x N per direction) */
    double *FS = (double *)malloc(sizeof(double) * 18 * N);

    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double w[9];
                cell_primitives(P, U, i, j, k, w);
                size_t c = cell(P, i, j, k);
                for (int v = 0; v < 9; v++) W[v * N + c] = w[v];
            }

    for (int d = 0; d < 3; d++) {
        const int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        int o[3];
        unit_offset(d, o);
        const double *bface = U + (size_t)(F_BX + d) * N;
        #pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    /* face between cell c - e_d (left) and c (right) */
                    double line[6][8];    /* cells c-3e_d .. c+2e_d: rho, vn, vt1, vt2, Bt1, Bt2, p, gamma */
                    for (int m = 0; m < 6; m++) {
                        int s = m - 3;
                        size_t cc = cell(P, i + s * o[0], j + s * o[1], k + s * o[2]);
                        line[m][0] = W[0 * N + cc];
                        line[m][1] = W[(1 + d) * N + cc];
                        line[m][2] = W[(1 + t1) * N + cc];
                        line[m][3] = W[(1 + t2) * N + cc];
                        line[m][4] = W[(4 + t1) * N + cc];
                        line[m][5] = W[(4 + t2) * N + cc];
                        line[m][6] = W[7 * N + cc];
                        line[m][7] = W[8 * N + cc];
                    }
                    double parl[24], parr[24];
                    for (int v = 0; v < 6; v++) {
                        double ql[5], qr[5];
                        for (int m = 0; m < 5; m++) {
                            ql[m] = line[m][1 + v];       /* cells c-3 .. c+1 around c-1 */
                            qr[m] = line[m + 1][1 + v];   /* cells c-2 .. c+2 around c   */
                        }
                        orc_parabola(ql, parl + 4 * v);
                        orc_parabola(qr, parr + 4 * v);
                    }
                    size_t c = cell(P, i, j, k);
                    double out[6];
                    /* face adiabatic index: the sqrt(rho)-weighted mean of the two cells' */
                    double gface = gm;
                    if (P->ionisation) {
                        double sl = sqrt(line[2][0]), sr = sqrt(line[3][0]);
                        gface = (sl * line[2][7] + sr * line[3][7]) / (sl + sr);
                    }
                    orc_riemann_face(line[2], line[3], parl, parr, bface[c], gface, eps, ydx, out);
                    for (int v = 0; v < 6; v++) FS[(size_t)(6 * d + v) * N + c] = out[v];
                }
    }

    /* fluxes and EMF contributions per face (Sec. 2 equations without the
     * advective terms; Sec. 2.5 E = B x U with the face states) */
    double *FL = (double *)malloc(sizeof(double) * 15 * N);  /* per dir: Fmn, Fmt1, Fmt2, FE, Vn */
    double *EM = (double *)malloc(sizeof(double) * 6 * N);   /* per dir: E_t1 part, E_t2 part */
    for (int d = 0; d < 3; d++) {
        const double *bface = U + (size_t)(F_BX + d) * N;
        #pragma omp parallel for schedule(static)
        for (size_t c = 0; c < N; c++) {
            double Vn = FS[(size_t)(6 * d + 0) * N + c];
            double Vt1 = FS[(size_t)(6 * d + 1) * N + c];
            double Vt2 = FS[(size_t)(6 * d + 2) * N + c];
            double Bt1 = FS[(size_t)(6 * d + 3) * N + c];
            double Bt2 = FS[(size_t)(6 * d + 4) * N + c];
            double Pg = FS[(size_t)(6 * d + 5) * N + c];
            double bn = bface[c];
            double Pst = Pg + 0.5 * (bn * bn + Bt1 * Bt1 + Bt2 * Bt2);
            double BV = bn * Vn + Bt1 * Vt1 + Bt2 * Vt2;
            FL[(size_t)(5 * d + 0) * N + c] = Pst - bn * bn;
            FL[(size_t)(5 * d + 1) * N + c] = -(bn * Bt1);
            FL[(size_t)(5 * d + 2) * N + c] = -(bn * Bt2);
            FL[(size_t)(5 * d + 3) * N + c] = Pst * Vn - bn * BV;
            FL[(size_t)(5 * d + 4) * N + c] = Vn;
            /* E component along t1: B_t2 U_n - B_n U_t2; along t2: B_n U_t1 - B_t1 U_n */
            EM[(size_t)(2 * d + 0) * N + c] = Bt2 * Vn - bn * Vt2;
            EM[(size_t)(2 * d + 1) * N + c] = bn * Vt1 - Bt1 * Vn;
        }
    }
    /* EMF contribution to component a from the face of direction d:
     * d = x gives (E_y, E_z), d = y gives (E_z, E_x), d = z gives (E_x, E_y). */
#define EMF(d, slot, ii, jj, kk) EM[(size_t)(2 * (d) + (slot)) * N + cell(P, ii, jj, kk)]

    /* edge fields, Appendix (electric field):
     *   Ex at (i, j-1/2, k-1/2): z-faces at j-1 and j, y-faces at k and k-1
     *   Ey at (i-1/2, j, k-1/2): z-faces at i-1 and i, x-faces at k-1 and k
     *   Ez at (i-1/2, j-1/2, k): x-faces at j-1 and j, y-faces at i-1 and i */
    double *Ed = (double *)malloc(sizeof(double) * 3 * N);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cell(P, i, j, k);
                Ed[0 * N + c] = 0.25 * (EMF(2, 0, i, j - 1, k) + EMF(2, 0, i, j, k) +
                                        EMF(1, 1, i, j, k) + EMF(1, 1, i, j, k - 1));
                Ed[1 * N + c] = 0.25 * (EMF(2, 1, i - 1, j, k) + EMF(2, 1, i, j, k) +
                                        EMF(0, 0, i, j, k - 1) + EMF(0, 0, i, j, k));
                Ed[2 * N + c] = 0.25 * (EMF(0, 1, i, j - 1, k) + EMF(0, 1, i, j, k) +
                                        EMF(1, 0, i - 1, j, k) + EMF(1, 0, i, j, k));
            }
#undef EMF

    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cell(P, i, j, k);
                size_t up[3] = { cell(P, i + 1, j, k), cell(P, i, j + 1, k), cell(P, i, j, k + 1) };
                double dF[3][5];
                for (int d = 0; d < 3; d++)
                    for (int v = 0; v < 5; v++)
                        dF[d][v] = FL[(size_t)(5 * d + v) * N + up[d]] - FL[(size_t)(5 * d + v) * N + c];
                /* momentum component a receives, from direction d, the flux slot
                 * 0 if a == d, 1 if a == d+1, 2 if a == d+2 (cyclic) */
                for (int a = 0; a < 3; a++) {
                    double sum = 0.0;
                    for (int d = 0; d < 3; d++) {
                        int slot = (a - d + 3) % 3;
                        sum += dF[d][slot];
                    }
                    inc[(size_t)(F_MX + a) * N + c] = -dtdx * sum;
                }
                inc[F_E * N + c] = -dtdx * (dF[0][3] + dF[1][3] + dF[2][3]);
                double divv = dF[0][4] + dF[1][4] + dF[2][4];
                inc[F_EI * N + c] = -(W[8 * N + c] - 1.0) * U[F_EI * N + c] * dtdx * divv;

                /* Sec. 2.5 face-field update from the edge fields */
                double dEz_y = Ed[2 * N + cell(P, i, j + 1, k)] - Ed[2 * N + c];
                double dEy_z = Ed[1 * N + cell(P, i, j, k + 1)] - Ed[1 * N + c];
                double dEx_z = Ed[0 * N + cell(P, i, j, k + 1)] - Ed[0 * N + c];
                double dEz_x = Ed[2 * N + cell(P, i + 1, j, k)] - Ed[2 * N + c];
                double dEy_x = Ed[1 * N + cell(P, i + 1, j, k)] - Ed[1 * N + c];
                double dEx_y = Ed[0 * N + cell(P, i, j + 1, k)] - Ed[0 * N + c];
                inc[F_BX * N + c] = -dtdx * dEz_y + dtdx * dEy_z;
                inc[F_BY * N + c] = -dtdx * dEx_z + dtdx * dEz_x;
                inc[F_BZ * N + c] = -dtdx * dEy_x + dtdx * dEx_y;
                inc[F_RHO * N + c] = 0.0;
                inc[F_H2 * N + c] = 0.0;
                inc[F_HP * N + c] = 0.0;
            }

    /* Sec. 2 (momentum and energy equations) and Sec. 2.4: self-gravity
     * sources -rho grad(Phi) and -rho v . grad(Phi) with central differences
     * of the potential of the current density (rho is the same in every
     * NONADV substage) */
    if (P->grav_G > 0.0) {
        double *phi = (double *)malloc(sizeof(double) * N);
        orc_potential(P, U + F_RHO * N, phi);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(P, i, j, k);
                    double g[3];
                    g[0] = (phi[cell(P, i + 1, j, k)] - phi[cell(P, i - 1, j, k)]) / (2.0 * h);
                    g[1] = (phi[cell(P, i, j + 1, k)] - phi[cell(P, i, j - 1, k)]) / (2.0 * h);
                    g[2] = (phi[cell(P, i, j, k + 1)] - phi[cell(P, i, j, k - 1)]) / (2.0 * h);
                    double rho = U[F_RHO * N + c];
                    double work = 0.0;
                    for (int a = 0; a < 3; a++) {
                        inc[(size_t)(F_MX + a) * N + c] -= dt * rho * g[a];
                        work += U[(size_t)(F_MX + a) * N + c] * g[a];
                    }
                    inc[F_E * N + c] -= dt * work;
                }
        free(phi);
    }

    free(W);
    free(FS);
    free(FL);
    free(EM);
    free(Ed);
}

/* ------------------------------------------------------------------ */
/* ADV right-hand side (Sec. 2.6): upwind parabola averages of the      */
/* conserved fields rho, mx, my, mz, E, e, h2 with the sqrt(rho)-weighted */
/* face velocity.                                                       */
/* ------------------------------------------------------------------ */
static const int adv_fields[8] = { F_RHO, F_MX, F_MY, F_MZ, F_E, F_EI, F_H2, F_HP };

static void adv_increment(const orc_params *P, const double *U, double dt, double *inc)
{
    const size_t N = ncell(P);
    const int nx = P->nx, ny = P->ny, nz = P->nz;
    const double h = 1.0 / (double)nx;
    const double dtdx = dt / h;
    const double ydx = P->theta * dtdx;

    const int nadv = P->ionisation ? 8 : 7;                   /* H+ is advected with the network */
    double *F = (double *)malloc(sizeof(double) * 24 * N);   /* per dir, per field */

    for (int d = 0; d < 3; d++) {
        int o[3];
        unit_offset(d, o);
        #pragma omp parallel for collapse(2) schedule(static)
        for (int k = 0; k < nz; k++)
            for (int j = 0; j < ny; j++)
                for (int i = 0; i < nx; i++) {
                    size_t c = cell(P, i, j, k);
                    size_t cl = cell(P, i - o[0], j - o[1], k - o[2]);
                    double rl = U[F_RHO * N + cl], rr = U[F_RHO * N + c];
                    double vl = U[(size_t)(F_MX + d) * N + cl] / rl;
                    double vr = U[(size_t)(F_MX + d) * N + c] / rr;
                    double sl = sqrt(rl), sr = sqrt(rr);
                    double vf = (sl * vl + sr * vr) / (sl + sr);
                    for (int f = 0; f < nadv; f++) {
                        const double *q = U + (size_t)adv_fields[f] * N;
                        double flux;
                        if (vf >= 0.0) {
                            double s5[5], par[4];
                            for (int m = 0; m < 5; m++) {
                                int s = m - 3;
                                s5[m] = q[cell(P, i + s * o[0], j + s * o[1], k + s * o[2])];
                            }
                            orc_parabola(s5, par);
                            flux = vf * orc_avg_right(par, ydx * vf);
                        } else {
                            double s5[5], par[4];
                            for (int m = 0; m < 5; m++) {
                                int s = m - 2;
                                s5[m] = q[cell(P, i + s * o[0], j + s * o[1], k + s * o[2])];
                            }
                            orc_parabola(s5, par);
                            flux = vf * orc_avg_left(par, ydx * (-vf));
                        }
                        F[(size_t)(8 * d + f) * N + c] = flux;
                    }
                }
    }

    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t c = cell(P, i, j, k);
                size_t up[3] = { cell(P, i + 1, j, k), cell(P, i, j + 1, k), cell(P, i, j, k + 1) };
                for (int f = 0; f < nadv; f++) {
                    double dx = F[(size_t)(8 * 0 + f) * N + up[0]] - F[(size_t)(8 * 0 + f) * N + c];
                    double dy = F[(size_t)(8 * 1 + f) * N + up[1]] - F[(size_t)(8 * 1 + f) * N + c];
                    double dz = F[(size_t)(8 * 2 + f) * N + up[2]] - F[(size_t)(8 * 2 + f) * N + c];
                    inc[(size_t)adv_fields[f] * N + c] = -dtdx * (dx + dy + dz);
                }
                if (nadv == 7) inc[F_HP * N + c] = 0.0;
                inc[F_BX * N + c] = 0.0;
                inc[F_BY * N + c] = 0.0;
                inc[F_BZ * N + c] = 0.0;
            }
    free(F);
}

/* ------------------------------------------------------------------ */
/* Sec. 2.2: three-stage Runge-Kutta over one split stage.               */
/* ------------------------------------------------------------------ */
typedef void (*rhs_fn)(const orc_params *, const double *, double, double *);

static void rk3_stage(const orc_params *P, double *U, double dt, rhs_fn rhs)
{
    const size_t N = ncell(P);
    const size_t T = NF * N;
    static const double a[3] = { 0.0, 0.75, 1.0 / 3.0 };
    static const double b[3] = { 1.0, 0.25, 2.0 / 3.0 };
    double *U0 = (double *)malloc(sizeof(double) * T);
    double *inc = (double *)malloc(sizeof(double) * T);
    memcpy(U0, U, sizeof(double) * T);
    for (int s = 0; s < 3; s++) {
        rhs(P, U, dt, inc);
        #pragma omp parallel for schedule(static)
        for (size_t t = 0; t < T; t++)
            U[t] = (U[t] + a[s] * (U0[t] - U[t])) + b[s] * inc[t];
    }
    free(U0);
    free(inc);
}

void orc_nonadv_stage(const orc_params *P, double *U, double dt) { rk3_stage(P, U, dt, nonadv_increment); }
void orc_adv_stage(const orc_params *P, double *U, double dt) { rk3_stage(P, U, dt, adv_increment); }

/* single-substage right-hand sides, for unit checks: inc = tau R(U) */
void orc_nonadv_rhs(const orc_params *P, const double *U, double dt, double *inc) { nonadv_increment(P, U, dt, inc); }
void orc_adv_rhs(const orc_params *P, const double *U, double dt, double *inc) { adv_increment(P, U, dt, inc); }

/* ------------------------------------------------------------------ */
/* Sec. 2.7 + Appendix (reaction rates 1-4): H/H2 chemistry of one cell. */
/* Returns the new H2 mass density.  rates_out (optional): k1', k2, k3, */
/* k4, C, D, T.                                                          */
/* ------------------------------------------------------------------ */

/* k1 without its n/n_H factor: C = k1 n_H^2 = k1' n n_H (Appendix, reaction 1) */
double orc_k1_base(double T)
{
    double t2 = T / 100.0;
    return 3e-17 * sqrt(t2) / (1.0 + 0.4 * sqrt(t2) + 0.2 * t2 + 0.08 * t2 * t2);
}

double orc_k2(double T)   /* Appendix, reaction 2 (collisional dissociation by H) */
{
    if (T > 7390.0) return 6.11e-14 * exp(-2.93e4 / T);
    return 2.67e-15 * exp(-(6750.0 / T) * (6750.0 / T));
}

double orc_k3(double T)   /* Appendix, reaction 3 (collisional dissociation by H2) */
{
    if (T > 7291.0) return 5.22e-14 * exp(-3.22e4 / T);
    return 3.17e-15 * exp(-(4060.0 / T) - (7500.0 / T) * (7500.0 / T));
}

double orc_k4(void)       /* Appendix, reaction 4: optically thin, f_shield = f_dust = 1 */
{
    return 3.3 * 1.7e-11;
}

double orc_chem_cell(const orc_params *P, double rho, double e, double h2, double dt, double *rates_out)
{
    double p = (P->gamma - 1.0) * e;
    double xh2 = h2 / rho;
    double mu = 1.0 / (1.0 - 0.5 * xh2);
    double T = P->T_unit * mu * p / rho;
    double nH = P->n_unit * (rho - h2);
    double nH2 = P->n_unit * h2 / 2.0;
    double n = nH + nH2;
    double k1b = orc_k1_base(T), k2 = orc_k2(T), k3 = orc_k3(T), k4 = orc_k4();
    double C = k1b * n * nH;
    double D = k2 * nH + k3 * nH2 + k4;
    double ts = dt * P->t_unit;
    /* Sec. 2.7: n(t+tau) = n + tau (C - D n) / (1 + tau D) */
    double nn = nH2 + ts * (C - D * nH2) / (1.0 + ts * D);
    double nmax = P->n_unit * rho / 2.0;
    if (nn > nmax) nn = nmax;
    if (nn < 0.0) nn = 0.0;
    if (rates_out) {
        rates_out[0] = k1b; rates_out[1] = k2; rates_out[2] = k3; rates_out[3] = k4;
        rates_out[4] = C; rates_out[5] = D; rates_out[6] = T;
    }
    return 2.0 * nn / P->n_unit;
}

/* ------------------------------------------------------------------ */
/* Sec. 2 stage 5 and Sec. 2.8 ("subgrid physics") with the appendix    */
/* heating and cooling functions of reactions 1-4 (erg cm^-3 s^-1).      */
/* ------------------------------------------------------------------ */
#define ORC_KB_ERG 1.380649e-16      /* Boltzmann constant, erg / K  */
#define ORC_KB_EV 8.617333262e-5     /* Boltzmann constant, eV / K   */
#define ORC_T_FLOOR 10.0             /* K: lower bound of the cooling */

/* critical density of the H2 formation heating, 10^(4 - 0.416 x - 0.327 x^2) cm^-3, x = log10(T / 1e4) */
double orc_ncrit(double T)
{
    double x = log10(T / 1e4);
    return pow(10.0, 4.0 - 0.416 * x - 0.327 * x * x);
}

/* reaction 2 cooling: high- and low-density limits L_H, L_L (erg s^-1 per H2) */
double orc_lh2(double T)
{
    double x = log10(T / 1e4);
    if (T > 1087.0) return 3.9e-19 * exp(-6118.0 / T);
    return pow(10.0, -19.24 + 0.474 * x - 1.247 * x * x);
}

double orc_ll2(double T, double nH, double nH2)
{
    double x = log10(T / 1e4);
    double f = (T > 4031.0) ? 1.38e-22 * exp(-9243.0 / T) : pow(10.0, -22.9 - 0.553 * x - 1.148 * x * x);
    return (pow(nH2, 0.77) + 1.2 * pow(nH, 0.77)) * f;
}

/* reaction 3 cooling: log of the low-density limit L_L = 8.18e-13 (n_H k_H + n_H2 k_H2)
 * with k_H = k_H2 = 6.29e-15 * 1.38 * f(T) / f(4500), f(T) = sqrt(T) a exp(-a),
 * a = 1 + 1 / (k_B T) with k_B T in eV (exp(-a): a collisional excitation
 * rate falls with temperature); kept in logarithms because f underflows at
 * low temperature */
static double orc_lnf3(double T)
{
    double a = 1.0 + 1.0 / (ORC_KB_EV * T);
    return 0.5 * log(T) + log(a) - a;
}

double orc_ln_ll3(double T, double n)
{
    return log(8.18e-13) + log(n) + log(6.29e-15 * 1.38) + orc_lnf3(T) - orc_lnf3(4500.0);
}

/* Gamma - Lambda of one cell (erg cm^-3 s^-1) at its current state.
 * terms_out (optional): Gamma1, Gamma4, Lambda2, Lambda3, T. */
double orc_heat_cool(const orc_params *P, double rho, double e, double h2, double *terms_out)
{
    double p = (P->gamma - 1.0) * e;
    double mu = 1.0 / (1.0 - 0.5 * (h2 / rho));
    double T = P->T_unit * mu * p / rho;
    double nH = P->n_unit * (rho - h2);
    double nH2 = P->n_unit * h2 / 2.0;
    double n = nH + nH2;
    /* Gamma1: 7.2e-12 erg per H2 formed, times the formation rate C of
     * reaction 1, times the fraction 1 / (1 + n_cr / n) */
    double g1 = 7.2e-12 * (orc_k1_base(T) * n * nH) / (1.0 + orc_ncrit(T) / n);
    /* Gamma4: 6.4e-13 erg per photodissociation */
    double g4 = 6.4e-13 * orc_k4() * nH2;
    /* Lambda2 = n_H2 L_H / (1 + L_H / L_L) */
    double lh2 = orc_lh2(T);
    double l2 = nH2 * lh2 / (1.0 + lh2 / orc_ll2(T, nH, nH2));
    /* Lambda3 = n_H2 L_H / (1 + L_H / L_L), L_H = 1.1e-13 exp(-6744 / T) */
    double ln_lh3 = log(1.1e-13) - 6744.0 / T;
    double l3 = nH2 * exp(ln_lh3) / (1.0 + exp(ln_lh3 - orc_ln_ll3(T, n)));
    if (terms_out) {
        terms_out[0] = g1; terms_out[1] = g4; terms_out[2] = l2; terms_out[3] = l3; terms_out[4] = T;
    }
    return (g1 + g4) - (l2 + l3);
}

/* With the ionisation network: the cell's adiabatic index and mean mass,
 * n_H = n_u (rho - h2 - hp), n = n_H + n_H2 + n_H+, and the terms of
 * reactions 5 and 6 added: cosmic-ray heating Gamma5 = 1.92e-28 n and
 * collisional-ionisation cooling Lambda6 = 2.18e-11 erg (13.6 eV) x k6 n_H n_e.
 * The printed Lambda7 (column densities and a square root of time) and
 * Lambda8 (no density factor) are left out.  terms_out (optional): Gamma1,
 * Gamma4, Lambda2, Lambda3, T, Gamma5, Lambda6. */
double orc_k6(double T);

double orc_heat_cool_ion(const orc_params *P, double rho, double e, double h2, double hp, double *terms_out)
{
    double gam = orc_gamma_cell(P, rho, h2, hp);
    double p = (gam - 1.0) * e;
    double T = P->T_unit * mean_mass(rho, h2, hp) * p / rho;
    double nH = P->n_unit * (rho - h2 - hp);
    double nH2 = P->n_unit * h2 / 2.0;
    double ne = P->n_unit * hp;
    double n = nH + nH2 + ne;
    double g1 = 7.2e-12 * (orc_k1_base(T) * n * nH) / (1.0 + orc_ncrit(T) / n);
    double g4 = 6.4e-13 * orc_k4() * nH2;
    double lh2 = orc_lh2(T);
    double l2 = nH2 * lh2 / (1.0 + lh2 / orc_ll2(T, nH, nH2));
    double ln_lh3 = log(1.1e-13) - 6744.0 / T;
    double l3 = nH2 * exp(ln_lh3) / (1.0 + exp(ln_lh3 - orc_ln_ll3(T, n)));
    double g5 = 1.92e-28 * n;
    double l6 = 2.18e-11 * orc_k6(T) * nH * ne;
    if (terms_out) {
        terms_out[0] = g1; terms_out[1] = g4; terms_out[2] = l2; terms_out[3] = l3; terms_out[4] = T;
        terms_out[5] = g5; terms_out[6] = l6;
    }
    return (g1 + g4 + g5) - (l2 + l3 + l6);
}

/* Sec. 2.8: explicit Euler step of d(rho eps)/dt = d(rho E)/dt = Gamma - Lambda
 * with the rates frozen over dt.  The code energy density unit is
 * n_u k_B T_u; cooling stops at the internal energy of T_floor (or at the
 * current one if the cell is already colder), and E takes the change that e
 * actually took. */
void orc_cooling(const orc_params *P, double *U, double dt)
{
    const size_t N = ncell(P);
    const double eu = P->n_unit * ORC_KB_ERG * P->T_unit;
    #pragma omp parallel for schedule(static)
    for (size_t c = 0; c < N; c++) {
        double rho = U[F_RHO * N + c], e = U[F_EI * N + c], h2 = U[F_H2 * N + c];
        double de, efloor;
        if (P->ionisation) {
            double hp = U[F_HP * N + c];
            de = dt * P->t_unit * orc_heat_cool_ion(P, rho, e, h2, hp, NULL) / eu;
            efloor = rho * ORC_T_FLOOR / (P->T_unit * mean_mass(rho, h2, hp) * (orc_gamma_cell(P, rho, h2, hp) - 1.0));
        } else {
            de = dt * P->t_unit * orc_heat_cool(P, rho, e, h2, NULL) / eu;
            double mu = 1.0 / (1.0 - 0.5 * (h2 / rho));
            efloor = rho * ORC_T_FLOOR / (P->T_unit * mu * (P->gamma - 1.0));
        }
        double lo = e < efloor ? e : efloor;
        double en = e + de;
        if (en < lo) en = lo;
        U[F_E * N + c] += en - e;
        U[F_EI * N + c] = en;
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 2.9: Poisson equation Laplace(Phi) = 4 pi G rho with the 27-point */
/* stencil, solved in harmonic space.  The discrete Fourier transform is  */
/* written out as plain sums along each axis (no fast algorithm).         */
/* ------------------------------------------------------------------ */

/* in-place DFT of every grid line along axis d: X_m = sum_j x_j exp(sgn 2 pi i j m / n) */
static void dft_axis(const orc_params *P, double *re, double *im, int d, int sgn)
{
    const int dims[3] = { P->nx, P->ny, P->nz };
    const int n = dims[d];
    const size_t stride = d == 0 ? 1 : (d == 1 ? (size_t)P->nx : (size_t)P->nx * P->ny);
    const int o1 = dims[d == 0 ? 1 : 0], o2 = dims[d == 2 ? 1 : 2];
    #pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < o2; b++)
        for (int a = 0; a < o1; a++) {
            int idx[3];
            idx[d] = 0;
            idx[d == 0 ? 1 : 0] = a;
            idx[d == 2 ? 1 : 2] = b;
            size_t base = cell(P, idx[0], idx[1], idx[2]);
            double *xr = (double *)malloc(sizeof(double) * 2 * n);
            double *xi = xr + n;
            for (int j = 0; j < n; j++) {
                xr[j] = re[base + j * stride];
                xi[j] = im[base + j * stride];
            }
            for (int m = 0; m < n; m++) {
                double sr = 0.0, si = 0.0;
                for (int j = 0; j < n; j++) {
                    /* angle from the reduced integer product j m mod n */
                    double t = 2.0 * ORC_PI * (double)(((long)j * m) % n) / (double)n;
                    double c = cos(t), s = sgn * sin(t);
                    sr += xr[j] * c - xi[j] * s;
                    si += xr[j] * s + xi[j] * c;
                }
                re[base + m * stride] = sr;
                im[base + m * stride] = si;
            }
            free(xr);
        }
}

/* eigenvalue factor of the 27-point stencil along one axis: (3 - 2 sin^2(pi m / n)) / 3 */
double orc_stencil_factor(int m, int n)
{
    double s = sin(ORC_PI * (double)m / (double)n);
    return (3.0 - 2.0 * s * s) / 3.0;
}

/* Phi = sum over modes of -(2/3) pi G h^2 rho_hat / (1 - ax ay az), the zero
 * mode (the mean density of the periodic box) set to zero */
void orc_potential(const orc_params *P, const double *rho, double *phi)
{
    const size_t N = ncell(P);
    const double h = 1.0 / (double)P->nx;
    double *re = (double *)malloc(sizeof(double) * N);
    double *im = (double *)calloc(N, sizeof(double));
    memcpy(re, rho, sizeof(double) * N);
    for (int d = 0; d < 3; d++) dft_axis(P, re, im, d, -1);
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = cell(P, i, j, k);
                double g = 0.0;
                if (i != 0 || j != 0 || k != 0) {
                    double a = orc_stencil_factor(i, P->nx) * orc_stencil_factor(j, P->ny) *
                               orc_stencil_factor(k, P->nz);
                    g = -(2.0 / 3.0) * ORC_PI * P->grav_G * h * h / (1.0 - a);
                }
                re[c] *= g;
                im[c] *= g;
            }
    for (int d = 0; d < 3; d++) dft_axis(P, re, im, d, +1);
    for (size_t c = 0; c < N; c++) phi[c] = re[c] / (double)N;
    free(re);
    free(im);
}

/* clamp of the advected H2 density to [0, rho] and, with the ionisation
 * network, of the H+ density to [0, rho - h2] (total hydrogen closure) */
void orc_clamp_h2(const orc_params *P, double *U)
{
    const size_t N = ncell(P);
    for (size_t c = 0; c < N; c++) {
        double r = U[F_RHO * N + c], x = U[F_H2 * N + c];
        if (x > r) x = r;
        if (x < 0.0) x = 0.0;
        U[F_H2 * N + c] = x;
        if (P->ionisation) {
            double y = U[F_HP * N + c];
            if (y > r - x) y = r - x;
            if (y < 0.0) y = 0.0;
            U[F_HP * N + c] = y;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 4.3 + Appendix: reactions 5-8 of the ionisation network.        */
/* ------------------------------------------------------------------ */

/* reaction 5, cosmic-ray ionisation: s^-1 per H atom (the printed n_H2
 * factor is read as a typesetting slip: Gamma5 = 1.92e-28 n is 20 eV per
 * ionisation at this rate per atom) */
double orc_k5(void) { return 6e-18; }

/* reaction 6, collisional ionisation (cm^3 s^-1): exp of the printed
 * polynomial in ln(T) with T in eV */
double orc_k6(double T)
{
    static const double c[9] = { -32.7, 13.5, -5.7, 1.5, -0.3, 3.4e-2, -2.6e-3, 1.1e-4, -2.1e-6 };
    double l = log(T * ORC_KB_EV), s = 0.0, lp = 1.0;
    for (int i = 0; i < 9; i++) {
        s += c[i] * lp;
        lp *= l;
    }
    return exp(s);
}

/* reaction 7, radiative recombination (cm^3 s^-1): 10 to the printed ratio
 * of quartics in x = log10(T) */
double orc_k7(double T)
{
    double x = log10(T);
    double num = -10.78 + 4.68 * x - 0.87 * x * x + 0.08 * x * x * x - 3.87e-3 * x * x * x * x;
    double den = 1.0 - 0.38 * x + 0.06 * x * x - 5.1e-3 * x * x * x + 2.4e-4 * x * x * x * x;
    return pow(10.0, num / den);
}

/* reaction 8, recombination on grains (cm^3 s^-1), as printed with log = log10 */
double orc_k8(double T)
{
    double inner = 1.0 + 5.087e2 * pow(T, 1.586e-2) * pow(10.0, -1.8892 - 4.4e-5 * log10(T));
    return 12.25e-14 / (1.0 + 8.074e-6 * pow(10.0, 2.756) * inner);
}

/* Sec. 2.7 with reactions 1-8: new H2 and H+ mass densities of one cell.
 * n_H = n_u (rho - h2 - hp), n_H2 = n_u h2 / 2, n_e = n_H+ = n_u hp, all
 * frozen at the start of the step; one semi-implicit update per species;
 * H2 is clamped to [0, n_u (rho - hp) / 2], then H+ to [0, n_u (rho - h2')].
 * rates_out (optional): k1', k2, k3, k4, k5, k6, k7, k8, T. */
void orc_chem_cell_ion(const orc_params *P, double rho, double e, double h2, double hp, double dt, double *h2_out,
                       double *hp_out, double *rates_out)
{
    double gam = orc_gamma_cell(P, rho, h2, hp);
    double p = (gam - 1.0) * e;
    double T = P->T_unit * mean_mass(rho, h2, hp) * p / rho;
    double nH = P->n_unit * (rho - h2 - hp);
    double nH2 = P->n_unit * h2 / 2.0;
    double ne = P->n_unit * hp;
    double n = nH + nH2 + ne;
    double ts = dt * P->t_unit;
    double k1b = orc_k1_base(T), k2 = orc_k2(T), k3 = orc_k3(T), k4 = orc_k4();
    double k5 = orc_k5(), k6 = orc_k6(T), k7 = orc_k7(T), k8 = orc_k8(T);
    /* H2 */
    double C = k1b * n * nH;
    double D = k2 * nH + k3 * nH2 + k4;
    double m2 = nH2 + ts * (C - D * nH2) / (1.0 + ts * D);
    double m2max = P->n_unit * (rho - hp) / 2.0;
    if (m2 > m2max) m2 = m2max;
    if (m2 < 0.0) m2 = 0.0;
    /* H+ (= e-) */
    double Ci = k5 * nH + k6 * nH * ne;
    double Di = (k7 + k8) * ne;
    double mi = ne + ts * (Ci - Di * ne) / (1.0 + ts * Di);
    double h2n = 2.0 * m2 / P->n_unit;
    double mimax = P->n_unit * (rho - h2n);
    if (mi > mimax) mi = mimax;
    if (mi < 0.0) mi = 0.0;
    *h2_out = h2n;
    *hp_out = mi / P->n_unit;
    if (rates_out) {
        rates_out[0] = k1b; rates_out[1] = k2; rates_out[2] = k3; rates_out[3] = k4;
        rates_out[4] = k5; rates_out[5] = k6; rates_out[6] = k7; rates_out[7] = k8; rates_out[8] = T;
    }
}

void orc_chemistry(const orc_params *P, double *U, double dt)
{
    const size_t N = ncell(P);
    #pragma omp parallel for schedule(static)
    for (size_t c = 0; c < N; c++) {
        if (P->ionisation) {
            double h2n, hpn;
            orc_chem_cell_ion(P, U[F_RHO * N + c], U[F_EI * N + c], U[F_H2 * N + c], U[F_HP * N + c], dt, &h2n,
                              &hpn, NULL);
            U[F_H2 * N + c] = h2n;
            U[F_HP * N + c] = hpn;
        } else {
            U[F_H2 * N + c] = orc_chem_cell(P, U[F_RHO * N + c], U[F_EI * N + c], U[F_H2 * N + c], dt, NULL);
        }
    }
}

/* ------------------------------------------------------------------ */
/* Sec. 2.8: regularisation (dual-energy synchronisation, pressure-gated). */
/* ------------------------------------------------------------------ */
void orc_regularise(const orc_params *P, double *U)
{
    const size_t N = ncell(P);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = cell(P, i, j, k);
                double rho = U[F_RHO * N + c];
                double mx = U[F_MX * N + c], my = U[F_MY * N + c], mz = U[F_MZ * N + c];
                double bx = 0.5 * (U[F_BX * N + c] + U[F_BX * N + cell(P, i + 1, j, k)]);
                double by = 0.5 * (U[F_BY * N + c] + U[F_BY * N + cell(P, i, j + 1, k)]);
                double bz = 0.5 * (U[F_BZ * N + c] + U[F_BZ * N + cell(P, i, j, k + 1)]);
                double E = U[F_E * N + c];
                double K = 0.5 * (mx * mx + my * my + mz * mz) / rho;
                double M = 0.5 * (bx * bx + by * by + bz * bz);
                double ei = E - K - M;
                double gam = orc_gamma_cell(P, rho, U[F_H2 * N + c], U[F_HP * N + c]);
                if (ei >= 1e-3 * E && (gam - 1.0) * ei > M) U[F_EI * N + c] = ei;
            }
}

/* ------------------------------------------------------------------ */
/* Sec. 2.3: time step from the CFL condition.                          */
/* ------------------------------------------------------------------ */
double orc_cell_speed(const orc_params *P, const double *U, int i, int j, int k)
{
    const size_t N = ncell(P);
    double w[9];
    cell_primitives(P, U, i, j, k, w);
    double rho = w[0];
    double v = sqrt(w[1] * w[1] + w[2] * w[2] + w[3] * w[3]);
    double c2 = w[8] * w[7] / rho;
    double ca2 = w[4] * w[4] / rho;
    double b2 = (w[4] * w[4] + w[5] * w[5] + w[6] * w[6]) / rho;
    double s = c2 + b2;
    double disc = s * s - 4.0 * c2 * ca2;
    if (disc < 0.0) disc = 0.0;
    double sd = sqrt(disc);
    double cf2 = 0.5 * (s + sd);
    double cs2 = 0.5 * (s - sd);
    if (cs2 < 0.0) cs2 = 0.0;
    (void)N;
    return v + sqrt(b2) + sqrt(c2) + sqrt(ca2) + sqrt(cs2) + sqrt(cf2);
}

double orc_cfl_dt(const orc_params *P, const double *U)
{
    const double h = 1.0 / (double)P->nx;
    double best = INFINITY;
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                double t = P->cfl * h / orc_cell_speed(P, U, i, j, k);
                if (t < best) best = t;
            }
    return best;
}

/* ------------------------------------------------------------------ */
/* Sec. 2 list of stages: one operator-split step (no gravity):         */
/* NONADV (with the face-field update inside), ADV, H2 clamp,           */
/* chemistry, heating/cooling (optional), regularisation.               */
/* ------------------------------------------------------------------ */
void orc_step(const orc_params *P, double *U, double dt)
{
    orc_nonadv_stage(P, U, dt);
    orc_adv_stage(P, U, dt);
    orc_clamp_h2(P, U);
    if (P->chemistry) orc_chemistry(P, U, dt);
    if (P->cooling) orc_cooling(P, U, dt);
    orc_regularise(P, U);
}

/* conserved totals in field order rho, mx, my, mz, E, e, bx, by, bz, h2
 * (compensated summation, so the totals themselves carry no O(N eps) drift) */
void orc_totals(const orc_params *P, const double *U, double out[NF])
{
    const size_t N = ncell(P);
    for (int f = 0; f < NF; f++) {
        double s = 0.0, comp = 0.0;
        for (size_t c = 0; c < N; c++) {
            double x = U[(size_t)f * N + c];
            double t = s + x;
            if (fabs(s) >= fabs(x)) comp += (s - t) + x;
            else comp += (x - t) + s;
            s = t;
        }
        out[f] = s + comp;
    }
}

/* primitive -> conserved: prim fields rho, vx, vy, vz, p, bx_f, by_f, bz_f, x_h2, x_hp */
void orc_prim_to_cons(const orc_params *P, const double *W, double *U)
{
    const size_t N = ncell(P);
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = cell(P, i, j, k);
                double rho = W[0 * N + c];
                double vx = W[1 * N + c], vy = W[2 * N + c], vz = W[3 * N + c];
                double p = W[4 * N + c];
                double bx = 0.5 * (W[5 * N + c] + W[5 * N + cell(P, i + 1, j, k)]);
                double by = 0.5 * (W[6 * N + c] + W[6 * N + cell(P, i, j + 1, k)]);
                double bz = 0.5 * (W[7 * N + c] + W[7 * N + cell(P, i, j, k + 1)]);
                double h2 = W[8 * N + c] * rho, hp = W[9 * N + c] * rho;
                double e = p / (orc_gamma_cell(P, rho, h2, hp) - 1.0);
                U[F_RHO * N + c] = rho;
                U[F_MX * N + c] = rho * vx;
                U[F_MY * N + c] = rho * vy;
                U[F_MZ * N + c] = rho * vz;
                U[F_EI * N + c] = e;
                U[F_E * N + c] = e + 0.5 * rho * (vx * vx + vy * vy + vz * vz) + 0.5 * (bx * bx + by * by + bz * bz);
                U[F_BX * N + c] = W[5 * N + c];
                U[F_BY * N + c] = W[6 * N + c];
                U[F_BZ * N + c] = W[7 * N + c];
                U[F_H2 * N + c] = h2;
                U[F_HP * N + c] = hp;
            }
}

/* discrete face-based divergence of B times h, max |.| over cells */
double orc_max_divb(const orc_params *P, const double *U)
{
    const size_t N = ncell(P);
    double m = 0.0;
    for (int k = 0; k < P->nz; k++)
        for (int j = 0; j < P->ny; j++)
            for (int i = 0; i < P->nx; i++) {
                size_t c = cell(P, i, j, k);
                double d = (U[F_BX * N + cell(P, i + 1, j, k)] - U[F_BX * N + c]) +
                           (U[F_BY * N + cell(P, i, j + 1, k)] - U[F_BY * N + c]) +
                           (U[F_BZ * N + cell(P, i, j, k + 1)] - U[F_BZ * N + c]);
                if (fabs(d) > m) m = fabs(d);
            }
    return m;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
