/*
 * Plain FP64 CPU oracle of the axisymmetric Shan–Chen lattice Boltzmann step
 * (Srivastava, Perlekar, ten Thije Boonkkamp, Verma, Toschi, "Axisymmetric
 * Multiphase Lattice Boltzmann Method", arXiv:1310.1871).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the HIP library: every constant and stencil below is written out here from
 * the paper on its own.
 *
 * The code is deliberately slow and literal: every intermediate field of one
 * time step is materialised in its own array, stencils are evaluated point by
 * point, and the boundary rules are applied as the paper states them.  The
 * same source is compiled twice: once with `double` (symbols or_*) and once
 * with `double _Complex` (symbols orc_*, define ORACLE_COMPLEX) for
 * complex-step derivatives.  No operation branches on a field value, so the
 * complex build is the analytic continuation of the real one.
 *
 * Conventions (paper Sec. II.C and II.E):
 *   - nodes z_k = k (k = 0..nz-1, periodic unless ORACLE_FLAG_ZWALLS) and
 *     r_j = j + 1/2 (j = 0..nr-1);
 *     the axis r = 0 lies half-way between row 0 and its mirror row -1, the
 *     outer wall r = nr half-way between row nr-1 and its mirror row nr;
 *   - populations f[i][j][k] (direction, row, column), z fastest;
 *   - the stored state is post-streaming (pre-collision) populations.
 *
 * Readings of points the paper leaves open are marked "Reading:" below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORACLE_COMPLEX
#include <complex.h>
typedef double _Complex num;
#define NUM_EXP cexp
#define API(name) orc_##name
#else
typedef double num;
#define NUM_EXP exp
#define API(name) or_##name
#endif

/* D2Q9 lattice (paper Sec. II.A and appendix, Eq. e_distribution):
 * velocities as (c_z, c_r).  Directions 1..4 are the axial/radial links with
 * c_1 = +z, c_2 = +r, c_3 = -z, c_4 = -r, which is the assignment the
 * mixed-derivative stencils of Sec. II.D require (they step along c_1/c_3 in
 * z and along c_2/c_4 in r).  Directions 5..8 are the diagonals. */
static const int CZ[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CR[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WT[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;  /* c_s^2 */

/* ghost rows kept on each r side of an extended field */
#define NG 6

typedef struct {
    int32_t nz, nr;
    double G, G_im;       /* Shan–Chen coupling (imaginary part: complex build only) */
    double tau, tau_im;   /* BGK relaxation time (imaginary part: complex build only) */
    double psi_rho0;      /* rho_0 of the pseudopotential */
    double gz;            /* body acceleration along +z */
    int32_t wall;         /* 0: no-slip (mid-grid bounce-back), 1: free-slip (mid-grid specular) */
    int32_t axisym;       /* 1: axisymmetric terms on, 0: plain 2D Shan–Chen */
    int32_t flags;        /* ORACLE_FLAG_* bits (see below) */
    int32_t in_row;       /* open boundaries (see below): inlet row or -1 */
    int32_t out_row;      /* outlet row or -1 */
    int32_t pad;
    double rho_in;        /* density imposed at the inlet */
    double rho_out;       /* density imposed at the outlet */
    const double* uz_in;  /* [nz] velocity imposed at the inlet, per column */
    const double* ur_in;
} or_params;

/* Force incorporation.  Default: the Shan–Chen velocity shift the paper's
 * scheme uses (Sec. II.A, Eqs. ueq and uhydro).  ORACLE_FLAG_GUO: the scheme
 * of Guo, Zheng and Shi (Phys. Rev. E 65, 046308, 2002), which the paper
 * compares against in Sec. IV.A and Table I: f^eq at the hydrodynamic
 * velocity u = (j + F/2)/rho and a forcing term
 *   (1 - 1/(2 tau)) W_i [ (c_i - u)/c_s^2 + (c_i . u) c_i / c_s^4 ] . F
 * added in the collision.  The axisymmetric sources h_i and the forces are
 * the same in both cases. */
#define ORACLE_FLAG_GUO 4

/* Derivative terms at the outer wall.  Sec. II.E states only that they vanish
 * at the non-axis boundaries.  Default reading: every field is reflected
 * evenly across the wall and the stencils run unchanged.
 * ORACLE_FLAG_NO_WALL_DERIV: the other reading -- F^{gamma,sym} is zero on
 * rows whose stencils reach across the wall (the 4 rows next to it) and the
 * velocity derivatives of H are zero on the 2 rows next to it. */
#define ORACLE_FLAG_NO_WALL_DERIV 2

/* Closed ends in z.  Sec. II.E imposes no-slip walls by mid-grid
 * bounce-back; with ORACLE_FLAG_ZWALLS the two ends of the z range are such
 * walls (at z = -1/2 and z = nz - 1/2, the two discs of the radial-flow
 * test of Sec. III) instead of a periodic join.  Reading for the fields
 * across them: psi is reflected evenly (for the Shan–Chen sum), and, as
 * Sec. II.E asks at the boundaries other than the axis, the derivative
 * terms are zero wherever their stencils would reach across: F^{gamma,sym}
 * on the 4 columns next to each wall, the velocity derivatives of H on the
 * 2 columns next to each wall. */
#define ORACLE_FLAG_ZWALLS 8

/* Source term position.  Sec. II.C places h_i at the mid-link point
 * (x + c_i/2, t + 1/2) without saying how it is evaluated; the default
 * reading takes the node value h_i(x, t).  ORACLE_FLAG_MIDLINK takes the
 * average of the two ends of the link, (h_i(x) + h_i(x + c_i)) / 2, with
 * h_i(y) = W_i (mass(y) + 3 c_i . H(y)) from the fields at y.  Across the
 * axis y is the mirror node with H_r reversed (H_z and the mass source are
 * even there, H_r odd); across the outer wall the mirror node's values are
 * used as they are (every field is even there).  Periodic z only; with open
 * rows the far end of a link may be an open row's node, whose fields are
 * used as they are. */
#define ORACLE_FLAG_MIDLINK 16

/* Open boundaries (Sec. II.E: a prescribed velocity or pressure is imposed
 * through the equilibrium populations, before streaming).  With
 * in_row >= 0 the post-collision populations of that row are replaced by
 * f^eq(rho_in, uz_in[z], ur_in[z]); with out_row >= 0 those of that row by
 * f^eq(rho_out, u) with u the hydrodynamic velocity of the node one row
 * inside (reading: an open outlet at imposed pressure passes the interior
 * velocity on).  The flow domain is the rows between them; derivative terms
 * are zero on rows whose stencils reach past an open row (F^{gamma,sym}
 * within 3 rows inside it, the velocity derivatives within 1 row inside it,
 * and on every row outside). */

/* order of the intermediate fields written by *_fields() */
enum {
    FLD_RHO, FLD_JZ, FLD_JR, FLD_PSI,
    FLD_FSCZ, FLD_FSCR,
    FLD_DR, FLD_DRR, FLD_D1R, FLD_DZR,
    FLD_FSYMZ, FLD_FSYMR,
    FLD_FZ, FLD_FR,
    FLD_UEQZ, FLD_UEQR, FLD_UZ, FLD_UR,
    FLD_DRUZ, FLD_DZUR, FLD_DRUR,
    FLD_HZ, FLD_HR,
    FLD_COUNT
};
/* after the FLD_COUNT scalar fields, *_fields() writes h[9] and fstar[9] */

static inline int wrap(int k, int n) {
    k %= n;
    return k < 0 ? k + n : k;
}

/* column of the node a (possibly ghost) column takes its value from:
 * periodic, or mirrored about the walls at -1/2 and nz - 1/2 */
static inline int col_of(int k, int n, int zw) {
    if (!zw) return wrap(k, n);
    while (k < 0 || k >= n) k = k < 0 ? -1 - k : 2 * n - 1 - k;
    return k;
}

static inline num get_param_G(const or_params* p) {
#ifdef ORACLE_COMPLEX
    return p->G + I * p->G_im;
#else
    return p->G;
#endif
}

static inline num get_param_tau(const or_params* p) {
#ifdef ORACLE_COMPLEX
    return p->tau + I * p->tau_im;
#else
    return p->tau;
#endif
}

/* index of the lattice direction with velocity (cz, cr) */
static int dir_of(int cz, int cr) {
    for (int i = 0; i < 9; ++i)
        if (CZ[i] == cz && CR[i] == cr) return i;
    abort();
}

/* value of an extended field (rows -NG..nr+NG-1) at column z, row r;
 * zw: z-walls (even mirror) instead of periodic z */
static inline num ext_at(const num* E, int nz, int z, int r, int zw) {
    return E[(size_t)(r + NG) * nz + col_of(z, nz, zw)];
}

/* Ghost extension of a real-row field (Sec. II.E, last sentences).
 * Reading: at the axis the derivative rule is symmetry: the field is
 * mirrored about r = 0 with sign axis_sign (+1 for even fields such as psi
 * and u_z, -1 for u_r).  At the outer wall the derivative terms are made to
 * vanish by an even mirror about r = nr.  z is periodic (no ghost columns). */
static void extend_rows(const num* src, num* E, int nz, int nr, double axis_sign) {
    for (int r = -NG; r < nr + NG; ++r) {
        int rs = r;
        double s = 1.0;
        if (r < 0) {
            rs = -1 - r;
            s = axis_sign;
        } else if (r >= nr) {
            rs = 2 * nr - 1 - r;
        }
        for (int z = 0; z < nz; ++z) E[(size_t)(r + NG) * nz + z] = s * src[(size_t)rs * nz + z];
    }
}

/* Isotropic first derivative on D2Q9 (Sec. II.D, first stencil and its
 * z-analogue): (1/36) sum_{i=1..8} (8 phi(x+c_i) - phi(x+2c_i)) c_i,axis. */
static num d_iso(const num* E, int nz, int z, int r, int along_r, int zw) {
    num s = 0.0;
    for (int i = 1; i < 9; ++i) {
        int c = along_r ? CR[i] : CZ[i];
        if (c == 0) continue;
        num t = 8.0 * ext_at(E, nz, z + CZ[i], r + CR[i], zw) - ext_at(E, nz, z + 2 * CZ[i], r + 2 * CR[i], zw);
        s += t * (double)c;
    }
    return s / 36.0;
}

/* One-dimensional fourth-order first derivative along r (Sec. II.D, last
 * stencil). */
static num d1_r(const num* E, int nz, int z, int r, int zw) {
    return (-ext_at(E, nz, z, r + 2, zw) + 8.0 * ext_at(E, nz, z, r + 1, zw) - 8.0 * ext_at(E, nz, z, r - 1, zw) +
            ext_at(E, nz, z, r - 2, zw)) / 12.0;
}

/* One-dimensional fourth-order first derivative along z of a real-row field
 * (the outer difference of the mixed-derivative stencil, Sec. II.D). */
static num d1_z(const num* F, int nz, int z, int r, int zw) {
    const num* row = F + (size_t)r * nz;
    return (-row[col_of(z + 2, nz, zw)] + 8.0 * row[col_of(z + 1, nz, zw)] - 8.0 * row[col_of(z - 1, nz, zw)] +
            row[col_of(z - 2, nz, zw)]) / 12.0;
}

typedef struct {
    int nz, nr;
    size_t n, next;
    num* fld[FLD_COUNT];
    num* psiE;   /* extended psi */
    num* DrE;    /* isotropic d_r psi on rows -4..nr+3 of an extended array */
    num* uzE;
    num* urE;
    num* h;      /* [9][n] */
    num* fstar;  /* [9][n] */
} workspace;

static int ws_alloc(workspace* w, int nz, int nr) {
    memset(w, 0, sizeof(*w));
    w->nz = nz;
    w->nr = nr;
    w->n = (size_t)nz * nr;
    w->next = (size_t)nz * (nr + 2 * NG);
    for (int k = 0; k < FLD_COUNT; ++k) {
        w->fld[k] = calloc(w->n, sizeof(num));
        if (!w->fld[k]) return -1;
    }
    w->psiE = calloc(w->next, sizeof(num));
    w->DrE = calloc(w->next, sizeof(num));
    w->uzE = calloc(w->next, sizeof(num));
    w->urE = calloc(w->next, sizeof(num));
    w->h = calloc(9 * w->n, sizeof(num));
    w->fstar = calloc(9 * w->n, sizeof(num));
    if (!w->psiE || !w->DrE || !w->uzE || !w->urE || !w->h || !w->fstar) return -1;
    return 0;
}

static void ws_free(workspace* w) {
    for (int k = 0; k < FLD_COUNT; ++k) free(w->fld[k]);
    free(w->psiE);
    free(w->DrE);
    free(w->uzE);
    free(w->urE);
    free(w->h);
    free(w->fstar);
}

/* Equilibrium distribution (appendix, Eq. e_distribution).
 * Reading: the printed form mixes u (linear term) and u^eq (quadratic terms);
 * the lattice Boltzmann equations of Sec. II.A/II.C evaluate f^eq at
 * (rho, u^eq), so one velocity is used throughout. */
static inline num feq(int i, num rho, num uz, num ur) {
    num cu = CZ[i] * uz + CR[i] * ur;
    num uu = uz * uz + ur * ur;
    return WT[i] * rho * (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
}

/* Every intermediate field of one step, from the post-streaming state f. */
static void compute_fields(const or_params* p, const num* f, workspace* w) {
    const int nz = p->nz, nr = p->nr;
    const size_t n = w->n;
    const num G = get_param_G(p);
    const num tau = get_param_tau(p);
    const double rho0 = p->psi_rho0;
    const int zw = (p->flags & ORACLE_FLAG_ZWALLS) != 0;
    num** F = w->fld;

    /* moments (appendix, Eq. hydro_var) and pseudopotential (Sec. II.A) */
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r) {
        for (int z = 0; z < nz; ++z) {
            size_t x = (size_t)r * nz + z;
            num rho = 0.0, jz = 0.0, jr = 0.0;
            for (int i = 0; i < 9; ++i) {
                num fi = f[i * n + x];
                rho += fi;
                jz += CZ[i] * fi;
                jr += CR[i] * fi;
            }
            F[FLD_RHO][x] = rho;
            F[FLD_JZ][x] = jz;
            F[FLD_JR][x] = jr;
            F[FLD_PSI][x] = rho0 * (1.0 - NUM_EXP(-rho / rho0));
        }
    }
    extend_rows(F[FLD_PSI], w->psiE, nz, nr, +1.0);

    /* isotropic d_r psi on the extended rows the second derivative needs */
#pragma omp parallel for schedule(static)
    for (int r = -4; r < nr + 4; ++r)
        for (int z = 0; z < nz; ++z) w->DrE[(size_t)(r + NG) * nz + z] = d_iso(w->psiE, nz, z, r, 1, zw);

#pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r)
        for (int z = 0; z < nz; ++z) {
            size_t x = (size_t)r * nz + z;
            F[FLD_DR][x] = ext_at(w->DrE, nz, z, r, zw);
            /* Reading: the second radial derivative applies the isotropic
             * stencil to the isotropic d_r field; the one-dimensional d_r is
             * used only inside the mixed derivative. */
            F[FLD_DRR][x] = d_iso(w->DrE, nz, z, r, 1, zw);
            F[FLD_D1R][x] = d1_r(w->psiE, nz, z, r, zw);
        }

#pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r)
        for (int z = 0; z < nz; ++z) {
            size_t x = (size_t)r * nz + z;
            F[FLD_DZR][x] = d1_z(F[FLD_D1R], nz, z, r, zw);

            /* Shan–Chen force, first neighbours (Sec. II.A, Eq. scforce) */
            num sz = 0.0, sr = 0.0;
            for (int i = 1; i < 9; ++i) {
                num ps = ext_at(w->psiE, nz, z + CZ[i], r + CR[i], zw);
                sz += WT[i] * ps * (double)CZ[i];
                sr += WT[i] * ps * (double)CR[i];
            }
            num psi = F[FLD_PSI][x];
            F[FLD_FSCZ][x] = -G * psi * sz;
            F[FLD_FSCR][x] = -G * psi * sr;

            /* axisymmetric extra force (Sec. II.D, Eq. scAxisExtra), c_s^4 = 1/9 */
            double rr = r + 0.5;
            num pref = -(G / 2.0) * (CS2 * CS2) * psi;
            const int flat = ((p->flags & ORACLE_FLAG_NO_WALL_DERIV) && r >= nr - 4) ||
                             (zw && (z < 4 || z >= nz - 4)) || (p->in_row >= 0 && r <= p->in_row + 3) ||
                             (p->out_row >= 0 && r >= p->out_row - 3);
            if (p->axisym && !flat) {
                F[FLD_FSYMZ][x] = pref * F[FLD_DZR][x] / rr;
                F[FLD_FSYMR][x] = pref * (F[FLD_DRR][x] / rr - F[FLD_DR][x] / (rr * rr));
            } else {
                F[FLD_FSYMZ][x] = 0.0;
                F[FLD_FSYMR][x] = 0.0;
            }

            /* total force: Shan–Chen + axisymmetric part + body force rho*g
             * along the axis (pipe-flow test, Sec. III) */
            num rho = F[FLD_RHO][x];
            F[FLD_FZ][x] = F[FLD_FSCZ][x] + F[FLD_FSYMZ][x] + rho * p->gz;
            F[FLD_FR][x] = F[FLD_FSCR][x] + F[FLD_FSYMR][x];

            /* equilibrium velocity (Eq. ueq) and hydrodynamic velocity (Eq. uhydro) */
            F[FLD_UZ][x] = (F[FLD_JZ][x] + 0.5 * F[FLD_FZ][x]) / rho;
            F[FLD_UR][x] = (F[FLD_JR][x] + 0.5 * F[FLD_FR][x]) / rho;
            if (p->flags & ORACLE_FLAG_GUO) {
                /* Guo forcing: the equilibrium is taken at the hydrodynamic velocity */
                F[FLD_UEQZ][x] = F[FLD_UZ][x];
                F[FLD_UEQR][x] = F[FLD_UR][x];
            } else {
                F[FLD_UEQZ][x] = (F[FLD_JZ][x] + tau * F[FLD_FZ][x]) / rho;
                F[FLD_UEQR][x] = (F[FLD_JR][x] + tau * F[FLD_FR][x]) / rho;
            }
        }

    /* velocity gradients for the viscous source terms.  Reading: the paper
     * gives stencils only for psi; the same isotropic first-derivative stencil
     * is used for the velocity derivatives, with the symmetry rule at the
     * axis (u_z even, u_r odd) and the even mirror at the wall. */
    extend_rows(F[FLD_UZ], w->uzE, nz, nr, +1.0);
    extend_rows(F[FLD_UR], w->urE, nz, nr, -1.0);

#pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r)
        for (int z = 0; z < nz; ++z) {
            size_t x = (size_t)r * nz + z;
            const int flat_u = ((p->flags & ORACLE_FLAG_NO_WALL_DERIV) && r >= nr - 2) ||
                               (zw && (z < 2 || z >= nz - 2)) || (p->in_row >= 0 && r <= p->in_row + 1) ||
                               (p->out_row >= 0 && r >= p->out_row - 1);
            if (flat_u) {
                F[FLD_DRUZ][x] = 0.0;
                F[FLD_DZUR][x] = 0.0;
                F[FLD_DRUR][x] = 0.0;
            } else {
                F[FLD_DRUZ][x] = d_iso(w->uzE, nz, z, r, 1, zw);
                F[FLD_DZUR][x] = d_iso(w->urE, nz, z, r, 0, zw);
                F[FLD_DRUR][x] = d_iso(w->urE, nz, z, r, 1, zw);
            }

            num rho = F[FLD_RHO][x], uz = F[FLD_UZ][x], ur = F[FLD_UR][x];
            double rr = r + 0.5;
            num hz = 0.0, hr = 0.0, mass = 0.0;
            if (p->axisym) {
                /* Eqs. condition_h and H_terms.  Reading: the c_iz / c_ir
                 * prefactors printed inside H_z, H_r are dropped; with them the
                 * first moment of h_i would vanish, contradicting the moment
                 * conditions derived in the appendix. */
                num mu = rho * CS2 * (tau - 0.5);  /* dynamic viscosity, nu = c_s^2 (tau - 1/2) */
                hz = (mu * (F[FLD_DRUZ][x] + F[FLD_DZUR][x]) - rho * ur * uz) / rr;
                hr = (2.0 * mu * (F[FLD_DRUR][x] - ur / rr) - rho * ur * ur) / rr;
                mass = -rho * ur / rr;
            }
            F[FLD_HZ][x] = hz;
            F[FLD_HR][x] = hr;

            /* source h_i evaluated at the node and current time.  Reading: the
             * paper places h_i at the mid-link, mid-step point without giving
             * its discretisation; the explicit node value is used (the
             * mid-link average is the ORACLE_FLAG_MIDLINK option). */
            for (int i = 0; i < 9; ++i) w->h[i * n + x] = WT[i] * (mass + (CZ[i] * hz + CR[i] * hr) / CS2);
        }

    const int midlink = (p->flags & ORACLE_FLAG_MIDLINK) != 0;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r)
        for (int z = 0; z < nz; ++z) {
            size_t x = (size_t)r * nz + z;
            num rho = F[FLD_RHO][x], uz = F[FLD_UZ][x], ur = F[FLD_UR][x];
            num uqz = F[FLD_UEQZ][x], uqr = F[FLD_UEQR][x];
            num inv_tau = 1.0 / tau;
            const int guo = (p->flags & ORACLE_FLAG_GUO) != 0;
            num Fz = F[FLD_FZ][x], Fr = F[FLD_FR][x];
            for (int i = 0; i < 9; ++i) {
                num hi = w->h[i * n + x];
                if (midlink && i > 0) {
                    /* h_i at the other end of the link, from that node's fields */
                    int yr = r + CR[i];
                    double sr = 1.0;  /* sign of H_r there */
                    if (yr < 0) {
                        yr = -1 - yr;
                        sr = -1.0;
                    } else if (yr >= nr) {
                        yr = 2 * nr - 1 - yr;
                    }
                    const size_t y = (size_t)yr * nz + wrap(z + CZ[i], nz);
                    num my = 0.0;
                    if (p->axisym) my = -F[FLD_RHO][y] * F[FLD_UR][y] / (yr + 0.5);
                    num hy = WT[i] * (my + (CZ[i] * F[FLD_HZ][y] + CR[i] * sr * F[FLD_HR][y]) / CS2);
                    hi = 0.5 * (hi + hy);
                }
                num fi = f[i * n + x];
                /* BGK collision plus source (Eq. lbm2d_mod_new) */
                num fs = fi - (fi - feq(i, rho, uqz, uqr)) * inv_tau + hi;
                if (guo) {
                    /* forcing term of Guo et al., with u the hydrodynamic velocity */
                    num cu = CZ[i] * uz + CR[i] * ur;
                    num gz = (CZ[i] - uz) / CS2 + cu * CZ[i] / (CS2 * CS2);
                    num gr = (CR[i] - ur) / CS2 + cu * CR[i] / (CS2 * CS2);
                    fs += (1.0 - 0.5 * inv_tau) * WT[i] * (gz * Fz + gr * Fr);
                }
                w->fstar[i * n + x] = fs;
            }
        }

    /* open boundaries: imposed equilibrium populations, before streaming */
    if (p->in_row >= 0)
        for (int z = 0; z < nz; ++z)
            for (int i = 0; i < 9; ++i)
                w->fstar[i * n + (size_t)p->in_row * nz + z] = feq(i, p->rho_in, p->uz_in[z], p->ur_in[z]);
    if (p->out_row >= 0)
        for (int z = 0; z < nz; ++z) {
            const size_t xi = (size_t)(p->out_row - 1) * nz + z;
            for (int i = 0; i < 9; ++i)
                w->fstar[i * n + (size_t)p->out_row * nz + z] = feq(i, p->rho_out, F[FLD_UZ][xi], F[FLD_UR][xi]);
        }
}

/* Streaming with the pre-streaming boundary rules (Sec. II.E): the axis is a
 * mid-grid specular reflector; the outer wall is mid-grid bounce-back
 * (no-slip) or mid-grid specular reflection (free-slip); z is periodic, or
 * closed by mid-grid bounce-back walls (ORACLE_FLAG_ZWALLS), which take
 * precedence where a link leaves through both. */
static void stream(const or_params* p, const num* fstar, num* fout) {
    const int nz = p->nz, nr = p->nr;
    const int zw = (p->flags & ORACLE_FLAG_ZWALLS) != 0;
    const size_t n = (size_t)nz * nr;
    /* every (node, direction) receives exactly one population, so rows can
     * be processed in parallel without write conflicts */
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nr; ++r)
        for (int z = 0; z < nz; ++z)
            for (int i = 0; i < 9; ++i) {
                int tz = z + CZ[i], tr = r + CR[i], d = i;
                if (zw && (tz < 0 || tz >= nz)) {
                    /* a disc: the population returns to its node reversed */
                    tz = z;
                    tr = r;
                    d = dir_of(-CZ[i], -CR[i]);
                } else if (tr < 0) {
                    /* crossed the axis: mirror image re-enters row 0 with the
                     * radial velocity reversed */
                    tr = 0;
                    d = dir_of(CZ[i], -CR[i]);
                } else if (tr >= nr) {
                    if (p->wall == 0) {
                        tz = z;
                        tr = r;
                        d = dir_of(-CZ[i], -CR[i]);
                    } else {
                        tr = nr - 1;
                        d = dir_of(CZ[i], -CR[i]);
                    }
                }
                fout[(size_t)d * n + (size_t)tr * nz + wrap(tz, nz)] = fstar[(size_t)i * n + (size_t)r * nz + z];
            }
}

/* ------------------------------------------------------------------ API -- */

int API(check)(const or_params* p) {
    if (p->nz < 1 || p->nr < NG) return -1;
    if ((p->flags & ~(ORACLE_FLAG_GUO | ORACLE_FLAG_NO_WALL_DERIV | ORACLE_FLAG_ZWALLS | ORACLE_FLAG_MIDLINK)) != 0)
        return -1;
    if ((p->flags & ORACLE_FLAG_MIDLINK) && (p->flags & ORACLE_FLAG_ZWALLS))
        return -1;
    if (p->in_row < -1 || p->in_row >= p->nr || p->out_row < -1 || p->out_row >= p->nr) return -1;
    if (p->in_row >= 0 && (!p->uz_in || !p->ur_in)) return -1;
    if (p->out_row == 0 || (p->in_row >= 0 && p->out_row >= 0 && p->out_row <= p->in_row)) return -1;
    return 0;
}

/* f_i = f^eq_i(rho, u) for given fields rho, uz, ur ([nr][nz]). */
void API(equilibrium)(const or_params* p, const num* rho, const num* uz, const num* ur, num* f) {
    const size_t n = (size_t)p->nz * p->nr;
    for (size_t x = 0; x < n; ++x)
        for (int i = 0; i < 9; ++i) f[i * n + x] = feq(i, rho[x], uz[x], ur[x]);
}

/* n_steps full steps; f_in and f_out may be the same array. */
int API(run)(const or_params* p, const num* f_in, num* f_out, int64_t n_steps) {
    if (API(check)(p)) return -1;
    workspace w;
    const size_t n = (size_t)p->nz * p->nr;
    if (ws_alloc(&w, p->nz, p->nr)) {
        ws_free(&w);
        return -2;
    }
    num* cur = malloc(9 * n * sizeof(num));
    if (!cur) {
        ws_free(&w);
        return -2;
    }
    memcpy(cur, f_in, 9 * n * sizeof(num));
    for (int64_t s = 0; s < n_steps; ++s) {
        compute_fields(p, cur, &w);
        stream(p, w.fstar, cur);
    }
    memcpy(f_out, cur, 9 * n * sizeof(num));
    free(cur);
    ws_free(&w);
    return 0;
}

/* Every intermediate of one step from state f: FLD_COUNT fields of n values,
 * then h[9][n] and fstar[9][n] (post-collision, pre-streaming). */
int API(fields)(const or_params* p, const num* f, num* out) {
    if (API(check)(p)) return -1;
    workspace w;
    const size_t n = (size_t)p->nz * p->nr;
    if (ws_alloc(&w, p->nz, p->nr)) {
        ws_free(&w);
        return -2;
    }
    compute_fields(p, f, &w);
    for (int k = 0; k < FLD_COUNT; ++k) memcpy(out + (size_t)k * n, w.fld[k], n * sizeof(num));
    memcpy(out + (size_t)FLD_COUNT * n, w.h, 9 * n * sizeof(num));
    memcpy(out + (size_t)(FLD_COUNT + 9) * n, w.fstar, 9 * n * sizeof(num));
    ws_free(&w);
    return 0;
}

/* Density and hydrodynamic velocity (Eq. uhydro, total force) of state f. */
int API(moments)(const or_params* p, const num* f, num* rho, num* uz, num* ur) {
    if (API(check)(p)) return -1;
    workspace w;
    const size_t n = (size_t)p->nz * p->nr;
    if (ws_alloc(&w, p->nz, p->nr)) {
        ws_free(&w);
        return -2;
    }
    compute_fields(p, f, &w);
    memcpy(rho, w.fld[FLD_RHO], n * sizeof(num));
    memcpy(uz, w.fld[FLD_UZ], n * sizeof(num));
    memcpy(ur, w.fld[FLD_UR], n * sizeof(num));
    ws_free(&w);
    return 0;
}

/* Streaming alone (for tests of the boundary rules). */
void API(stream)(const or_params* p, const num* fstar, num* fout) { stream(p, fstar, fout); }

/* Point evaluation of one stencil on a caller-filled extended array E
 * (rows -NG..nr+NG-1, z periodic), for tests of the stencils themselves:
 *   kind 0: isotropic d_r      1: isotropic d_z
 *   kind 2: 1D d_r             3: 1D d_z of the 1D d_r (mixed d_zr)
 *   kind 4: isotropic d_r of isotropic d_r (d_rr)
 *   kind 5: sum_i W_i c_iz E(x+c_i)   6: sum_i W_i c_ir E(x+c_i)
 * The point must lie far enough from the extended edges for the stencil. */
num API(stencil_point)(int kind, int nz, int nr, const num* E, int z, int r) {
    (void)nr;
    switch (kind) {
        case 0: return d_iso(E, nz, z, r, 1, 0);
        case 1: return d_iso(E, nz, z, r, 0, 0);
        case 2: return d1_r(E, nz, z, r, 0);
        case 3: {
            num v[5];
            for (int k = -2; k <= 2; ++k) v[k + 2] = d1_r(E, nz, z + k, r, 0);
            return (-v[4] + 8.0 * v[3] - 8.0 * v[1] + v[0]) / 12.0;
        }
        case 4: {
            num s = 0.0;
            for (int i = 1; i < 9; ++i) {
                if (CR[i] == 0) continue;
                num t = 8.0 * d_iso(E, nz, z + CZ[i], r + CR[i], 1, 0) - d_iso(E, nz, z + 2 * CZ[i], r + 2 * CR[i], 1, 0);
                s += t * (double)CR[i];
            }
            return s / 36.0;
        }
        case 5:
        case 6: {
            num s = 0.0;
            for (int i = 1; i < 9; ++i) s += WT[i] * ext_at(E, nz, z + CZ[i], r + CR[i], 0) * (double)(kind == 5 ? CZ[i] : CR[i]);
            return s;
        }
        default: return 0.0;
    }
}

/* Lattice tables, exported so tests can check them against the identities
 * the appendix lists (Eq. weights). */
void API(lattice)(int* cz, int* cr, double* w) {
    for (int i = 0; i < 9; ++i) {
        cz[i] = CZ[i];
        cr[i] = CR[i];
        w[i] = WT[i];
    }
}

int API(num_fields)(void) { return FLD_COUNT; }
int API(ghost_rows)(void) { return NG; }
