/*
 * gcme_oracle.c -- plain FP64 CPU oracle for the GCMe nonbonded path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of bench.py load this library.  The product (the HIP library
 * under paper_2403_08148_amd/) never links, imports or calls it, and the two
 * share no code, headers or tables.
 *
 * What it computes (reduced units, k_B T = 1, lengths in the bead diameter):
 *   - GCM excluded-volume pair potential, eq. u_ex (Model and methods,
 *     "Gaussian core model"):  A_ij (3/(2 pi s2))^{3/2} exp(-3 r^2/(2 s2)),
 *     s2 = sigma_i^2 + sigma_j^2.
 *   - Smeared Coulomb pair potential, eq. u_elec:
 *     lB z_i z_j erf(sqrt(pi/2) r / a_ij) / r,  a_ij^2 = a_i^2 + a_j^2.
 *   - The four-term Ewald split of eq. ewald: real-space bracket
 *     [erf(alpha_ij r) - erf(beta r)]/r with beta = 1/(sqrt(2) G),
 *     the reciprocal sum (exact k-sum, or smooth PME on a mesh, the mesh
 *     method the paper cites for U_recip), the constant correction
 *     -lB beta/sqrt(pi) sum z^2 and the Born self term lB/2 sum z^2/a.
 *   - Forces F = -dE/dr, the virial tensor sum r_ij (x) f_ij (eq. pres_virial
 *     uses its trace) plus the reciprocal-space virial.
 *   - Parameter derivatives dE/dA (per type pair), dE/dsigma_t, dE/da_t, and
 *     per bead dE/dsigma_i, dE/da_i, and the forces' vector-Jacobian product
 *     sum_i v_i . dF_i/dtheta for force matching.
 *   - The slab correction for a slab in a box with a vacuum gap along z
 *     (nonmetal electrodes; section "Image charge effects on polyelectrolyte
 *     adsorption", with the Yeh--Berkowitz reference it cites):
 *     E = 2 pi lB M_z^2 / V, M_z = sum z_i z-coordinate_i.
 *   - Harmonic bonds u = k/2 (r - b)^2 (the bond potential of that section).
 *   - The method of image charges for perfectly conducting electrodes
 *     (section "Method of image charges"): the real system in 0 < z < Lz,
 *     its mirror image in -Lz < z < 0 with opposite charges, one periodic
 *     box of length 2 Lz; images follow their sources after every drift.
 *   - Velocity-Verlet and BAOAB Langevin steps (the paper integrates the
 *     Langevin equation; the splitting is this oracle's reading), with
 *     Philox4x64-10 (Salmon et al., SC'11) Gaussian noise keyed by
 *     (seed, step, bead id, replica).
 *
 * Every loop here is the definition written out: no blocking or reordering
 * beyond a cell list that only skips pairs beyond the cutoff (checked against
 * brute force in the tests).  Parity pins live in tests/test_oracle_*.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

typedef struct {
    double box[3];
    double rc;      /* real-space cutoff (pairs with r < rc) */
    double beta;    /* Ewald splitting, erf(beta r); beta = 1/(sqrt2 G) */
    double lB;      /* Bjerrum length */
    int nt;         /* number of bead types */
    const double* A;     /* [nt*nt] symmetric, kT * d^3 */
    const double* sigma; /* [nt] mass smearing radius */
    const double* a;     /* [nt] charge smearing radius */
} gco_params;

/* ------------------------------------------------------------------ */
/* Scalar pair functions                                               */
/* ------------------------------------------------------------------ */

/* eq. u_ex */
double gco_u_ex(double r, double A, double s2) {
    double pref = pow(3.0 / (2.0 * M_PI * s2), 1.5);
    return A * pref * exp(-3.0 * r * r / (2.0 * s2));
}

/* eq. u_elec; r -> 0 limit lB zz sqrt(2)/a_ij (SI, "Limits") */
double gco_u_elec(double r, double lB, double zz, double aij) {
    double alpha = sqrt(M_PI / 2.0) / aij;
    if (r == 0.0) return lB * zz * 2.0 * alpha / sqrt(M_PI);
    return lB * zz * erf(alpha * r) / r;
}

/* Real-space bracket of eq. ewald divided by r:
 * phi(r) = [erf(alpha r) - erf(beta r)] / r, and g(r) = -(1/r) dphi/dr so
 * that the force on i from j is lB zz g(r) (r_i - r_j). */
static void real_bracket(double r, double alpha, double beta, double* phi, double* g) {
    const double tsp = 2.0 / sqrt(M_PI);
    if (r == 0.0) {
        *phi = tsp * (alpha - beta);
        *g = tsp * (2.0 / 3.0) * (alpha * alpha * alpha - beta * beta * beta);
        return;
    }
    double ph = (erf(alpha * r) - erf(beta * r)) / r;
    double dphidr = (tsp * (alpha * exp(-alpha * alpha * r * r) - beta * exp(-beta * beta * r * r)) - ph) / r;
    *phi = ph;
    *g = -dphidr / r;
}

double gco_phi_real(double r, double alpha, double beta) {
    double p, g;
    real_bracket(r, alpha, beta, &p, &g);
    return p;
}

static inline double wrapd(double x, double L) {
    double y = fmod(x, L);
    if (y < 0) y += L;
    if (y >= L) y -= L;
    return y;
}

static inline double min_image(double d, double L) {
    return d - L * nearbyint(d / L);
}

/* ------------------------------------------------------------------ */
/* Real space: GCM + smeared-Coulomb bracket, minimum image, r < rc     */
/* ------------------------------------------------------------------ */

typedef struct {
    double ex, real;
    double W[6];
} pair_acc;

/* Contribution of one ordered pair (i, j) at separation d = r_i - r_j to the
 * force on i, and half of the pair energy / virial (the pair is visited from
 * both sides).  Adjoint sums (half, for the same reason) are optional. */
static void pair_term(const gco_params* p, int ti, int tj, int zi, int zj,
                      const double d[3], double* fi, pair_acc* acc,
                      double* Eex_tt, double* dEdsig, double* dEda) {
    double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
    if (r2 >= p->rc * p->rc) return;
    double r = sqrt(r2);
    int nt = p->nt;
    double s2 = p->sigma[ti] * p->sigma[ti] + p->sigma[tj] * p->sigma[tj];
    double A = p->A[ti * nt + tj];
    double u = gco_u_ex(r, A, s2);
    /* -du/dr / r = 3 u / s2 */
    double fs = 3.0 * u / s2;
    double elec_e = 0.0;
    if (zi != 0 && zj != 0) {
        double aij = sqrt(p->a[ti] * p->a[ti] + p->a[tj] * p->a[tj]);
        double alpha = sqrt(M_PI / 2.0) / aij;
        double ph, g;
        real_bracket(r, alpha, p->beta, &ph, &g);
        double zz = (double)zi * (double)zj;
        elec_e = p->lB * zz * ph;
        fs += p->lB * zz * g;
        if (dEda) {
            /* d/da_ij of lB zz erf(alpha r)/r, alpha = sqrt(pi/2)/a_ij:
             * -lB zz (2/sqrt(pi)) (alpha/a_ij) exp(-alpha^2 r^2); chain rule
             * da_ij/da_t = a_t/a_ij for each end of type t. */
            double dudaij = -p->lB * zz * (2.0 / sqrt(M_PI)) * (alpha / aij) * exp(-alpha * alpha * r2);
            dEda[ti] += 0.5 * dudaij * p->a[ti] / aij;
            dEda[tj] += 0.5 * dudaij * p->a[tj] / aij;
        }
    }
    for (int k = 0; k < 3; ++k) fi[k] += fs * d[k];
    acc->ex += 0.5 * u;
    acc->real += 0.5 * elec_e;
    /* virial of the pair r_ij (x) f_ij, halved */
    acc->W[0] += 0.5 * fs * d[0] * d[0];
    acc->W[1] += 0.5 * fs * d[1] * d[1];
    acc->W[2] += 0.5 * fs * d[2] * d[2];
    acc->W[3] += 0.5 * fs * d[0] * d[1];
    acc->W[4] += 0.5 * fs * d[0] * d[2];
    acc->W[5] += 0.5 * fs * d[1] * d[2];
    if (Eex_tt) {
        /* per unordered type pair energy, stored symmetrically */
        Eex_tt[ti * nt + tj] += 0.5 * u;
        if (ti != tj) Eex_tt[tj * nt + ti] += 0.5 * u;
    }
    if (dEdsig) {
        double s = sqrt(s2);
        /* du/ds = u (3 r^2 / s^3 - 3 / s), ds/dsigma_t = sigma_t / s */
        double duds = u * (3.0 * r2 / (s2 * s) - 3.0 / s);
        dEdsig[ti] += 0.5 * duds * p->sigma[ti] / s;
        dEdsig[tj] += 0.5 * duds * p->sigma[tj] / s;
    }
}

/* Sum over all i (or over a sample of i) of the pair terms within rc.
 * Energies and virial always run over all beads (E/W may be NULL to skip).
 * Requires rc <= L/2 on every axis (minimum image).  use_cells selects a
 * cell list with cells >= rc (needs >= 3 cells per axis, else brute force).
 * pos is AoS [N][3]; F is AoS [n_out][3] where n_out = n_sample or N. */
int gco_real_space(int N, const double* pos, const int* type, const int* z,
                   const gco_params* p, int use_cells, int n_sample, const int* sample,
                   double* F, double* E2, double* W, double* Eex_tt,
                   double* dEdsig, double* dEda) {
    for (int k = 0; k < 3; ++k)
        if (p->rc > 0.5 * p->box[k]) return -1;
    int nt = p->nt;
    double* wp = (double*)malloc(sizeof(double) * 3 * (size_t)N);
    for (int i = 0; i < N; ++i)
        for (int k = 0; k < 3; ++k) wp[3 * i + k] = wrapd(pos[3 * i + k], p->box[k]);

    int nc[3];
    int cells_ok = use_cells;
    for (int k = 0; k < 3; ++k) {
        nc[k] = (int)floor(p->box[k] / p->rc);
        if (nc[k] < 3) cells_ok = 0;
    }
    int* head = NULL;
    int* next = NULL;
    if (cells_ok) {
        size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
        head = (int*)malloc(sizeof(int) * ncell);
        next = (int*)malloc(sizeof(int) * (size_t)N);
        for (size_t c = 0; c < ncell; ++c) head[c] = -1;
        /* insert in reverse so each cell lists beads in increasing index */
        for (int i = N - 1; i >= 0; --i) {
            int c3[3];
            for (int k = 0; k < 3; ++k) {
                c3[k] = (int)(wp[3 * i + k] / p->box[k] * nc[k]);
                if (c3[k] >= nc[k]) c3[k] = nc[k] - 1;
            }
            size_t c = ((size_t)c3[0] * nc[1] + c3[1]) * nc[2] + c3[2];
            next[i] = head[c];
            head[c] = i;
        }
    }

    /* per-bead partial sums, reduced afterwards in index order */
    int want_all = (E2 || W || Eex_tt || dEdsig || dEda);
    int n_iter = want_all ? N : n_sample;
    pair_acc* acc = (pair_acc*)calloc((size_t)N, sizeof(pair_acc));
    double* ftmp = (double*)calloc((size_t)3 * N, sizeof(double));
    double* ett = Eex_tt ? (double*)calloc((size_t)N * nt * nt, sizeof(double)) : NULL;
    double* dsg = dEdsig ? (double*)calloc((size_t)N * nt, sizeof(double)) : NULL;
    double* dea = dEda ? (double*)calloc((size_t)N * nt, sizeof(double)) : NULL;

#pragma omp parallel for schedule(dynamic, 64)
    for (int ii = 0; ii < n_iter; ++ii) {
        int i = (want_all || !sample) ? ii : sample[ii];
        double fi[3] = {0, 0, 0};
        double* e_tt = ett ? ett + (size_t)i * nt * nt : NULL;
        double* d_s = dsg ? dsg + (size_t)i * nt : NULL;
        double* d_a = dea ? dea + (size_t)i * nt : NULL;
        if (cells_ok) {
            int c3[3];
            for (int k = 0; k < 3; ++k) {
                c3[k] = (int)(wp[3 * i + k] / p->box[k] * nc[k]);
                if (c3[k] >= nc[k]) c3[k] = nc[k] - 1;
            }
            for (int dx = -1; dx <= 1; ++dx)
                for (int dy = -1; dy <= 1; ++dy)
                    for (int dz = -1; dz <= 1; ++dz) {
                        int cx = (c3[0] + dx + nc[0]) % nc[0];
                        int cy = (c3[1] + dy + nc[1]) % nc[1];
                        int cz = (c3[2] + dz + nc[2]) % nc[2];
                        size_t c = ((size_t)cx * nc[1] + cy) * nc[2] + cz;
                        for (int j = head[c]; j >= 0; j = next[j]) {
                            if (j == i) continue;
                            double d[3];
                            for (int k = 0; k < 3; ++k)
                                d[k] = min_image(wp[3 * i + k] - wp[3 * j + k], p->box[k]);
                            pair_term(p, type[i], type[j], z[i], z[j], d, fi, &acc[i], e_tt, d_s, d_a);
                        }
                    }
        } else {
            for (int j = 0; j < N; ++j) {
                if (j == i) continue;
                double d[3];
                for (int k = 0; k < 3; ++k)
                    d[k] = min_image(wp[3 * i + k] - wp[3 * j + k], p->box[k]);
                pair_term(p, type[i], type[j], z[i], z[j], d, fi, &acc[i], e_tt, d_s, d_a);
            }
        }
        for (int k = 0; k < 3; ++k) ftmp[3 * i + k] = fi[k];
    }

    if (F) {
        if (sample) {
            for (int s = 0; s < n_sample; ++s)
                for (int k = 0; k < 3; ++k) F[3 * s + k] = ftmp[3 * sample[s] + k];
        } else {
            memcpy(F, ftmp, sizeof(double) * 3 * (size_t)N);
        }
    }
    if (want_all) {
        double ex = 0, re = 0, w[6] = {0, 0, 0, 0, 0, 0};
        for (int i = 0; i < N; ++i) {
            ex += acc[i].ex;
            re += acc[i].real;
            for (int k = 0; k < 6; ++k) w[k] += acc[i].W[k];
        }
        if (E2) { E2[0] = ex; E2[1] = re; }
        if (W) for (int k = 0; k < 6; ++k) W[k] = w[k];
        if (Eex_tt) {
            for (int q = 0; q < nt * nt; ++q) {
                double s = 0;
                for (int i = 0; i < N; ++i) s += ett[(size_t)i * nt * nt + q];
                Eex_tt[q] = s;
            }
        }
        if (dEdsig) {
            for (int t = 0; t < nt; ++t) {
                double s = 0;
                for (int i = 0; i < N; ++i) s += dsg[(size_t)i * nt + t];
                dEdsig[t] = s;
            }
        }
        if (dEda) {
            for (int t = 0; t < nt; ++t) {
                double s = 0;
                for (int i = 0; i < N; ++i) s += dea[(size_t)i * nt + t];
                dEda[t] = s;
            }
        }
    }
    free(wp); free(head); free(next); free(acc); free(ftmp);
    free(ett); free(dsg); free(dea);
    return 0;
}

/* Per-bead radius derivatives: the derivative of E with respect to bead i's
 * own mass radius sigma_i and charge radius a_i, as if every bead had its
 * own radii (evaluated at the per-type values), written out over all pairs
 * by brute force (minimum image, r < rc):
 *   dE/dsigma_i = sum_j du_ex/ds_ij * sigma_i / s_ij,  s_ij^2 = sigma_i^2 + sigma_j^2
 *     (eq. u_ex: du/ds = u (3 r^2/s^3 - 3/s)),
 *   dE/da_i = sum_j d/da_ij [lB z_i z_j erf(alpha_ij r)/r] * a_i / a_ij
 *             - lB z_i^2 / (2 a_i^2)
 *     (eq. u_elec through the real-space term of eq. ewald, and eq.
 *     self_energy; the reciprocal and correction terms do not depend on a).
 * Summed over the beads of a type they give dE/dsigma_t and dE/da_t. */
int gco_per_bead_adjoint(int N, const double* pos, const int* type, const int* z, const gco_params* p,
                         double* dsig, double* da) {
    for (int k = 0; k < 3; ++k)
        if (p->rc > 0.5 * p->box[k]) return -1;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N; ++i) {
        const int ti = type[i];
        double ds = 0.0, dq = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3], r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                d[k] = min_image(wrapd(pos[3 * i + k], p->box[k]) - wrapd(pos[3 * j + k], p->box[k]), p->box[k]);
                r2 += d[k] * d[k];
            }
            if (r2 >= p->rc * p->rc) continue;
            const int tj = type[j];
            const double s2 = p->sigma[ti] * p->sigma[ti] + p->sigma[tj] * p->sigma[tj], s = sqrt(s2);
            const double u = gco_u_ex(sqrt(r2), p->A[ti * p->nt + tj], s2);
            ds += u * (3.0 * r2 / (s2 * s) - 3.0 / s) * p->sigma[ti] / s;
            if (z[i] != 0 && z[j] != 0) {
                const double aij = sqrt(p->a[ti] * p->a[ti] + p->a[tj] * p->a[tj]);
                const double alpha = sqrt(M_PI / 2.0) / aij;
                const double dud = -p->lB * (double)z[i] * (double)z[j] * (2.0 / sqrt(M_PI)) * (alpha / aij) *
                                   exp(-alpha * alpha * r2);
                dq += dud * p->a[ti] / aij;
            }
        }
        dsig[i] = ds;
        da[i] = dq - 0.5 * p->lB * (double)z[i] * (double)z[i] / (p->a[ti] * p->a[ti]);
    }
    return 0;
}

/* Force vector-Jacobian product for force matching: for a per-bead vector
 * v (AoS [N][3]), the derivatives of sum_i v_i . F_i with respect to the
 * parameters, by brute force over ordered pairs (i, j), r < rc.  The pair
 * force on i is fs(r) d with d = r_i - r_j, so each ordered pair adds
 * (v_i . d) dfs/dtheta:
 *   GCM (eq. u_ex, fs = 3 u / s^2): dfs/dA_ij = fs / A_ij, evaluated as the
 *     A = 1 value; dfs/ds = (u / s^3)(9 r^2 / s^2 - 15), ds/dsigma_t =
 *     sigma_t / s for each end of type t;
 *   real-space electrostatics (eq. ewald's first term, fs = lB z_i z_j g):
 *     dg/dalpha = 2 (2/sqrt(pi)) alpha^2 exp(-alpha^2 r^2), alpha =
 *     sqrt(pi/2)/a_ij, dalpha/da_ij = -alpha/a_ij, da_ij/da_t = a_t/a_ij.
 * The reciprocal term's forces do not depend on A, sigma or a.
 * dA[nt*nt] is the derivative for the symmetric parameter (both orders of a
 * type pair), dsig[nt], da[nt]. */
int gco_force_vjp(int N, const double* pos, const int* type, const int* z, const gco_params* p, const double* v,
                  double* dA, double* dsig, double* da) {
    for (int k = 0; k < 3; ++k)
        if (p->rc > 0.5 * p->box[k]) return -1;
    const int nt = p->nt;
    double* M = (double*)calloc((size_t)N * (nt * nt + 2 * nt), sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < N; ++i) {
        double* m = M + (size_t)i * (nt * nt + 2 * nt);
        const int ti = type[i];
        for (int j = 0; j < N; ++j) {
            if (j == i) continue;
            double d[3], r2 = 0.0;
            for (int k = 0; k < 3; ++k) {
                d[k] = min_image(wrapd(pos[3 * i + k], p->box[k]) - wrapd(pos[3 * j + k], p->box[k]), p->box[k]);
                r2 += d[k] * d[k];
            }
            if (r2 >= p->rc * p->rc) continue;
            const int tj = type[j];
            const double vd = v[3 * i] * d[0] + v[3 * i + 1] * d[1] + v[3 * i + 2] * d[2];
            const double r = sqrt(r2);
            const double s2 = p->sigma[ti] * p->sigma[ti] + p->sigma[tj] * p->sigma[tj], s = sqrt(s2);
            const double u1 = gco_u_ex(r, 1.0, s2), u = p->A[ti * nt + tj] * u1;
            m[ti * nt + tj] += vd * 3.0 * u1 / s2;
            const double dfds = u / (s2 * s) * (9.0 * r2 / s2 - 15.0);
            m[nt * nt + ti] += vd * dfds * p->sigma[ti] / s;
            m[nt * nt + tj] += vd * dfds * p->sigma[tj] / s;
            if (z[i] != 0 && z[j] != 0) {
                const double aij = sqrt(p->a[ti] * p->a[ti] + p->a[tj] * p->a[tj]);
                const double al = sqrt(M_PI / 2.0) / aij;
                const double dfda = p->lB * (double)z[i] * (double)z[j] * 2.0 * (2.0 / sqrt(M_PI)) * al * al *
                                    exp(-al * al * r2) * (-al / aij);
                m[nt * nt + nt + ti] += vd * dfda * p->a[ti] / aij;
                m[nt * nt + nt + tj] += vd * dfda * p->a[tj] / aij;
            }
        }
    }
    for (int q = 0; q < nt * nt + 2 * nt; ++q) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += M[(size_t)i * (nt * nt + 2 * nt) + q];
        if (q < nt * nt) {
            /* ordered sums first, symmetrised below */
            dA[q] = acc;
        } else if (q < nt * nt + nt) {
            dsig[q - nt * nt] = acc;
        } else {
            da[q - nt * nt - nt] = acc;
        }
    }
    for (int t = 0; t < nt; ++t)
        for (int u2 = t + 1; u2 < nt; ++u2) {
            const double sym = dA[t * nt + u2] + dA[u2 * nt + t];
            dA[t * nt + u2] = dA[u2 * nt + t] = sym;
        }
    free(M);
    return 0;
}

/* Real space summed over periodic images n (any rc, no minimum-image
 * restriction): E = 1/2 sum_n sum'_{i,j} u(|r_i - r_j + nL|), the prime
 * dropping i = j at n = 0 (eq. ewald's real-space term).  GCM and the
 * smeared-Coulomb bracket both truncated at rc.  For the pins only: O(N^2
 * n_images). */
int gco_real_space_images(int N, const double* pos, const int* type, const int* z,
                          const gco_params* p, double* F, double* E2, double* W) {
    int nimg[3];
    for (int k = 0; k < 3; ++k) nimg[k] = (int)ceil(p->rc / p->box[k]) + 1;
    pair_acc* acc = (pair_acc*)calloc((size_t)N, sizeof(pair_acc));
    double* ftmp = (double*)calloc((size_t)3 * N, sizeof(double));
#pragma omp parallel for schedule(dynamic, 8)
    for (int i = 0; i < N; ++i) {
        double fi[3] = {0, 0, 0};
        for (int j = 0; j < N; ++j)
            for (int n0 = -nimg[0]; n0 <= nimg[0]; ++n0)
                for (int n1 = -nimg[1]; n1 <= nimg[1]; ++n1)
                    for (int n2 = -nimg[2]; n2 <= nimg[2]; ++n2) {
                        if (i == j && n0 == 0 && n1 == 0 && n2 == 0) continue;
                        double d[3] = {pos[3 * i] - pos[3 * j] + n0 * p->box[0],
                                       pos[3 * i + 1] - pos[3 * j + 1] + n1 * p->box[1],
                                       pos[3 * i + 2] - pos[3 * j + 2] + n2 * p->box[2]};
                        pair_term(p, type[i], type[j], z[i], z[j], d, fi, &acc[i], NULL, NULL, NULL);
                    }
        for (int k = 0; k < 3; ++k) ftmp[3 * i + k] = fi[k];
    }
    double ex = 0, re = 0, w[6] = {0, 0, 0, 0, 0, 0};
    for (int i = 0; i < N; ++i) {
        ex += acc[i].ex;
        re += acc[i].real;
        for (int k = 0; k < 6; ++k) w[k] += acc[i].W[k];
    }
    if (E2) { E2[0] = ex; E2[1] = re; }
    if (W) for (int k = 0; k < 6; ++k) W[k] = w[k];
    if (F) memcpy(F, ftmp, sizeof(double) * 3 * (size_t)N);
    free(acc); free(ftmp);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Constant terms of eq. ewald                                          */
/* ------------------------------------------------------------------ */

/* U_corr = -lB beta/sqrt(pi) sum z^2 ; U_self = lB/2 sum z^2 / a_i.
 * dEda_self[t] = d U_self / d a_t = -lB/2 sum_{i in t} z_i^2 / a_t^2. */
void gco_constants(int N, const int* type, const int* z, const gco_params* p,
                   double* Ecorr, double* Eself, double* dEda_self) {
    double s2 = 0, sa = 0;
    if (dEda_self)
        for (int t = 0; t < p->nt; ++t) dEda_self[t] = 0;
    for (int i = 0; i < N; ++i) {
        double zz = (double)z[i] * (double)z[i];
        s2 += zz;
        sa += zz / p->a[type[i]];
        if (dEda_self) dEda_self[type[i]] += -0.5 * p->lB * zz / (p->a[type[i]] * p->a[type[i]]);
    }
    if (Ecorr) *Ecorr = -p->lB * p->beta / sqrt(M_PI) * s2;
    if (Eself) *Eself = 0.5 * p->lB * sa;
}

/* ------------------------------------------------------------------ */
/* Exact reciprocal sum (eq. ewald, U_recip), tin-foil (k != 0)          */
/* ------------------------------------------------------------------ */

/* U_recip = (2 pi lB / V) sum_{k != 0, |k| <= kmax} exp(-k^2/(4 beta^2))/k^2 |S(k)|^2,
 * S(k) = sum_j z_j exp(i k.r_j), k = 2 pi (n0/L0, n1/L1, n2/L2).
 * Force F_i = (4 pi lB z_i / V) sum_k g(k) k Im(S* e^{i k.r_i}).
 * Virial W_ab = sum_k e(k) [delta_ab - 2 (1 + k^2/(4 beta^2)) k_a k_b / k^2]. */
int gco_ewald_recip(int N, const double* pos, const int* z, const double box[3],
                    double beta, double lB, double kmax, double* F, double* E, double* W) {
    double V = box[0] * box[1] * box[2];
    int nmax[3];
    for (int k = 0; k < 3; ++k) nmax[k] = (int)floor(kmax * box[k] / (2.0 * M_PI));
    /* enumerate half space: n0 > 0, or n0 == 0 && n1 > 0, or n0 == n1 == 0 && n2 > 0 */
    int nk = 0;
    int cap = (2 * nmax[0] + 1) * (2 * nmax[1] + 1) * (2 * nmax[2] + 1);
    double* kv = (double*)malloc(sizeof(double) * 3 * (size_t)cap);
    for (int n0 = 0; n0 <= nmax[0]; ++n0)
        for (int n1 = -nmax[1]; n1 <= nmax[1]; ++n1)
            for (int n2 = -nmax[2]; n2 <= nmax[2]; ++n2) {
                if (n0 == 0 && (n1 < 0 || (n1 == 0 && n2 <= 0))) continue;
                double k0 = 2 * M_PI * n0 / box[0], k1 = 2 * M_PI * n1 / box[1], k2 = 2 * M_PI * n2 / box[2];
                double kk = k0 * k0 + k1 * k1 + k2 * k2;
                if (kk > kmax * kmax) continue;
                kv[3 * nk] = k0; kv[3 * nk + 1] = k1; kv[3 * nk + 2] = k2;
                ++nk;
            }
    int nq = 0;
    for (int i = 0; i < N; ++i) if (z[i] != 0) ++nq;
    int* qi = (int*)malloc(sizeof(int) * (size_t)(nq > 0 ? nq : 1));
    nq = 0;
    for (int i = 0; i < N; ++i) if (z[i] != 0) qi[nq++] = i;

    double* ek = (double*)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    double* Sre = (double*)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
    double* Sim = (double*)malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1));
#pragma omp parallel for schedule(static)
    for (int q = 0; q < nk; ++q) {
        double sr = 0, si = 0;
        for (int t = 0; t < nq; ++t) {
            int j = qi[t];
            double ph = kv[3 * q] * pos[3 * j] + kv[3 * q + 1] * pos[3 * j + 1] + kv[3 * q + 2] * pos[3 * j + 2];
            sr += z[j] * cos(ph);
            si += z[j] * sin(ph);
        }
        Sre[q] = sr; Sim[q] = si;
        double kk = kv[3 * q] * kv[3 * q] + kv[3 * q + 1] * kv[3 * q + 1] + kv[3 * q + 2] * kv[3 * q + 2];
        /* factor 2 for the -k partner of each half-space vector */
        ek[q] = 2.0 * (2.0 * M_PI * lB / V) * exp(-kk / (4.0 * beta * beta)) / kk;
    }
    double e = 0, w[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < nk; ++q) {
        double kk = kv[3 * q] * kv[3 * q] + kv[3 * q + 1] * kv[3 * q + 1] + kv[3 * q + 2] * kv[3 * q + 2];
        double eq = ek[q] * (Sre[q] * Sre[q] + Sim[q] * Sim[q]);
        e += eq;
        double c = 2.0 * (1.0 + kk / (4.0 * beta * beta)) / kk;
        const double* kq = kv + 3 * q;
        w[0] += eq * (1.0 - c * kq[0] * kq[0]);
        w[1] += eq * (1.0 - c * kq[1] * kq[1]);
        w[2] += eq * (1.0 - c * kq[2] * kq[2]);
        w[3] += eq * (-c * kq[0] * kq[1]);
        w[4] += eq * (-c * kq[0] * kq[2]);
        w[5] += eq * (-c * kq[1] * kq[2]);
    }
    if (E) *E = e;
    if (W) for (int k = 0; k < 6; ++k) W[k] = w[k];
    if (F) {
        memset(F, 0, sizeof(double) * 3 * (size_t)N);
#pragma omp parallel for schedule(static)
        for (int t = 0; t < nq; ++t) {
            int i = qi[t];
            double f[3] = {0, 0, 0};
            for (int q = 0; q < nk; ++q) {
                double ph = kv[3 * q] * pos[3 * i] + kv[3 * q + 1] * pos[3 * i + 1] + kv[3 * q + 2] * pos[3 * i + 2];
                /* Im(S* e^{i ph}) = Sre sin(ph) - Sim cos(ph) */
                double im = Sre[q] * sin(ph) - Sim[q] * cos(ph);
                /* ek holds 2 (2 pi lB / V) g; the force prefactor is
                 * (4 pi lB / V) g per full-space k and the -k partner adds
                 * the same amount, so a half-space k carries 2 ek */
                double s = 2.0 * ek[q] * z[i] * im;
                f[0] += s * kv[3 * q];
                f[1] += s * kv[3 * q + 1];
                f[2] += s * kv[3 * q + 2];
            }
            for (int k = 0; k < 3; ++k) F[3 * i + k] = f[k];
        }
    }
    free(kv); free(qi); free(ek); free(Sre); free(Sim);
    return nk;
}

/* ------------------------------------------------------------------ */
/* Mixed-radix complex FFT (unnormalised), the mesh transform for SPME  */
/* ------------------------------------------------------------------ */

/* Recursive decimation in time: for n = r m, split the input into r
 * interleaved subsequences of length m, transform each, and combine with
 * twiddles W_n^e = exp(sign 2 pi i e / n).  tw holds the roots of unity of
 * the top-level length; a sub-transform of length n uses every (N/n)-th one.
 * sign = -1 forward, +1 inverse; unnormalised; x interleaved complex. */
static void fft_rec(int n, const double* in, int istride, double* out,
                    const double* tw, int twstep, double* scratch) {
    if (n == 1) { out[0] = in[0]; out[1] = in[1]; return; }
    int r = 0;
    for (int f = 2; f <= n; ++f) if (n % f == 0) { r = f; break; }
    int m = n / r;
    for (int s = 0; s < r; ++s)
        fft_rec(m, in + 2 * (size_t)s * istride, istride * r, out + 2 * (size_t)s * m,
                tw, twstep * r, scratch);
    /* X[k + q m] = sum_s W_n^{s (k + q m)} Y_s[k] */
    for (int k = 0; k < m; ++k) {
        for (int q = 0; q < r; ++q) {
            double re = 0, im = 0;
            for (int s = 0; s < r; ++s) {
                long long e = ((long long)s * (k + (long long)q * m)) % n;
                double c = tw[2 * e * twstep], sn = tw[2 * e * twstep + 1];
                double yr = out[2 * ((size_t)s * m + k)], yi = out[2 * ((size_t)s * m + k) + 1];
                re += c * yr - sn * yi;
                im += c * yi + sn * yr;
            }
            scratch[2 * ((size_t)k + (size_t)q * m)] = re;
            scratch[2 * ((size_t)k + (size_t)q * m) + 1] = im;
        }
    }
    memcpy(out, scratch, sizeof(double) * 2 * (size_t)n);
}

int gco_fft(int n, double* x, int sign) {
    double* in = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* scr = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    double* tw = (double*)malloc(sizeof(double) * 2 * (size_t)n);
    for (int e = 0; e < n; ++e) {
        double ang = sign * 2.0 * M_PI * (double)e / (double)n;
        tw[2 * e] = cos(ang);
        tw[2 * e + 1] = sin(ang);
    }
    memcpy(in, x, sizeof(double) * 2 * (size_t)n);
    /* children finish with scratch before the parent combines, so one
     * scratch buffer serves every level */
    fft_rec(n, in, 1, x, tw, 1, scr);
    free(in); free(scr); free(tw);
    return 0;
}

/* 3D transform of a [K0][K1][K2] complex grid, axis by axis. */
static void fft3d(const int K[3], double* g, int sign) {
    int maxk = K[0];
    if (K[1] > maxk) maxk = K[1];
    if (K[2] > maxk) maxk = K[2];
    /* axis 2 (contiguous) */
#pragma omp parallel
    {
        double* line = (double*)malloc(sizeof(double) * 2 * (size_t)maxk);
#pragma omp for collapse(2)
        for (int a = 0; a < K[0]; ++a)
            for (int b = 0; b < K[1]; ++b) {
                double* base = g + 2 * (((size_t)a * K[1] + b) * K[2]);
                memcpy(line, base, sizeof(double) * 2 * K[2]);
                gco_fft(K[2], line, sign);
                memcpy(base, line, sizeof(double) * 2 * K[2]);
            }
#pragma omp for collapse(2)
        for (int a = 0; a < K[0]; ++a)
            for (int c = 0; c < K[2]; ++c) {
                for (int b = 0; b < K[1]; ++b) {
                    size_t o = 2 * (((size_t)a * K[1] + b) * K[2] + c);
                    line[2 * b] = g[o]; line[2 * b + 1] = g[o + 1];
                }
                gco_fft(K[1], line, sign);
                for (int b = 0; b < K[1]; ++b) {
                    size_t o = 2 * (((size_t)a * K[1] + b) * K[2] + c);
                    g[o] = line[2 * b]; g[o + 1] = line[2 * b + 1];
                }
            }
#pragma omp for collapse(2)
        for (int b = 0; b < K[1]; ++b)
            for (int c = 0; c < K[2]; ++c) {
                for (int a = 0; a < K[0]; ++a) {
                    size_t o = 2 * (((size_t)a * K[1] + b) * K[2] + c);
                    line[2 * a] = g[o]; line[2 * a + 1] = g[o + 1];
                }
                gco_fft(K[0], line, sign);
                for (int a = 0; a < K[0]; ++a) {
                    size_t o = 2 * (((size_t)a * K[1] + b) * K[2] + c);
                    g[o] = line[2 * a]; g[o + 1] = line[2 * a + 1];
                }
            }
        free(line);
    }
}

/* ------------------------------------------------------------------ */
/* Smooth particle-mesh Ewald (Essmann et al. 1995) for U_recip          */
/* ------------------------------------------------------------------ */

/* Cardinal B-spline M_n(x), support [0, n], by the two-term recursion
 * M_n(x) = x/(n-1) M_{n-1}(x) + (n-x)/(n-1) M_{n-1}(x-1), M_1 = 1 on [0,1). */
double gco_bspline(int n, double x) {
    if (x < 0.0 || x >= (double)n) return 0.0;
    if (n == 1) return 1.0;
    return (x * gco_bspline(n - 1, x) + ((double)n - x) * gco_bspline(n - 1, x - 1.0)) / (double)(n - 1);
}

/* |b(m)|^{-2} = |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K)|^2 for m in [0,K).
 * For odd p this vanishes at m = K/2; such entries (below 1e-7) take the mean
 * of their two periodic neighbours (the reading used on both sides). */
void gco_bspline_moduli(int K, int p, double* mod) {
    for (int m = 0; m < K; ++m) {
        double re = 0, im = 0;
        for (int k = 0; k <= p - 2; ++k) {
            double w = gco_bspline(p, (double)(k + 1));
            double ang = 2.0 * M_PI * (double)m * (double)k / (double)K;
            re += w * cos(ang);
            im += w * sin(ang);
        }
        mod[m] = re * re + im * im;
    }
    for (int m = 0; m < K; ++m)
        if (mod[m] < 1e-7) mod[m] = 0.5 * (mod[(m - 1 + K) % K] + mod[(m + 1) % K]);
}

/* SPME reciprocal energy, forces and virial.
 * Q(k) = sum_i z_i prod_a M_p(u_ia - k_a) (periodic in k), u_ia = K_a frac(r_ia/L_a).
 * E = (lB/2) sum_{m != 0} G(m) |DFT(Q)(m)|^2,
 * G(m) = exp(-pi^2 |m|^2 / beta^2) / (pi V |m|^2) / prod_a mod_a(m_a),
 * |m|^2 = sum_a (m_a / L_a)^2 with m_a taken in (-K/2, K/2].
 * phi = IDFT(G DFT(Q)) (unnormalised), F_i = -lB z_i sum_k grad_i W_i(k) phi(k).
 * Returns the grid potential phi in phi_out if non-NULL ([K0][K1][K2]). */
int gco_spme_recip(int N, const double* pos, const int* z, const double box[3],
                   double beta, double lB, const int K[3], int p,
                   double* F, double* E, double* W, double* phi_out) {
    size_t ng = (size_t)K[0] * K[1] * K[2];
    double V = box[0] * box[1] * box[2];
    double* Q = (double*)calloc(2 * ng, sizeof(double));
    double* mod[3];
    for (int a = 0; a < 3; ++a) {
        mod[a] = (double*)malloc(sizeof(double) * K[a]);
        gco_bspline_moduli(K[a], p, mod[a]);
    }
    /* spread (sequential: the sum order is the bead order) */
    for (int i = 0; i < N; ++i) {
        if (z[i] == 0) continue;
        int k0[3];
        double w[3][16];
        for (int a = 0; a < 3; ++a) {
            double u = wrapd(pos[3 * i + a], box[a]) / box[a] * K[a];
            double fl = floor(u);
            k0[a] = (int)fl;
            for (int j = 0; j < p; ++j) w[a][j] = gco_bspline(p, u - fl + j);
        }
        for (int j0 = 0; j0 < p; ++j0)
            for (int j1 = 0; j1 < p; ++j1)
                for (int j2 = 0; j2 < p; ++j2) {
                    int g0 = ((k0[0] - j0) % K[0] + K[0]) % K[0];
                    int g1 = ((k0[1] - j1) % K[1] + K[1]) % K[1];
                    int g2 = ((k0[2] - j2) % K[2] + K[2]) % K[2];
                    Q[2 * (((size_t)g0 * K[1] + g1) * K[2] + g2)] += z[i] * w[0][j0] * w[1][j1] * w[2][j2];
                }
    }
    fft3d(K, Q, -1);
    double e = 0, wv[6] = {0, 0, 0, 0, 0, 0};
    for (int m0 = 0; m0 < K[0]; ++m0)
        for (int m1 = 0; m1 < K[1]; ++m1)
            for (int m2 = 0; m2 < K[2]; ++m2) {
                size_t o = ((size_t)m0 * K[1] + m1) * K[2] + m2;
                if (m0 == 0 && m1 == 0 && m2 == 0) { Q[2 * o] = 0; Q[2 * o + 1] = 0; continue; }
                int ms[3] = {m0, m1, m2};
                double mv[3];
                for (int a = 0; a < 3; ++a) {
                    int mm = ms[a] <= K[a] / 2 ? ms[a] : ms[a] - K[a];
                    mv[a] = (double)mm / box[a];
                }
                double m2s = mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2];
                double G = exp(-M_PI * M_PI * m2s / (beta * beta)) / (M_PI * V * m2s) /
                           (mod[0][m0] * mod[1][m1] * mod[2][m2]);
                double q2 = Q[2 * o] * Q[2 * o] + Q[2 * o + 1] * Q[2 * o + 1];
                double em = 0.5 * lB * G * q2;
                e += em;
                double c = 2.0 * (1.0 + M_PI * M_PI * m2s / (beta * beta)) / m2s;
                wv[0] += em * (1.0 - c * mv[0] * mv[0]);
                wv[1] += em * (1.0 - c * mv[1] * mv[1]);
                wv[2] += em * (1.0 - c * mv[2] * mv[2]);
                wv[3] += em * (-c * mv[0] * mv[1]);
                wv[4] += em * (-c * mv[0] * mv[2]);
                wv[5] += em * (-c * mv[1] * mv[2]);
                Q[2 * o] *= G;
                Q[2 * o + 1] *= G;
            }
    if (E) *E = e;
    if (W) for (int k = 0; k < 6; ++k) W[k] = wv[k];
    fft3d(K, Q, +1);
    if (phi_out)
        for (size_t o = 0; o < ng; ++o) phi_out[o] = Q[2 * o];
    if (F) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < N; ++i) {
            F[3 * i] = F[3 * i + 1] = F[3 * i + 2] = 0;
            if (z[i] == 0) continue;
            int k0[3];
            double w[3][16], dw[3][16];
            for (int a = 0; a < 3; ++a) {
                double u = wrapd(pos[3 * i + a], box[a]) / box[a] * K[a];
                double fl = floor(u);
                k0[a] = (int)fl;
                for (int j = 0; j < p; ++j) {
                    double x = u - fl + j;
                    w[a][j] = gco_bspline(p, x);
                    /* M_p'(x) = M_{p-1}(x) - M_{p-1}(x-1) */
                    dw[a][j] = gco_bspline(p - 1, x) - gco_bspline(p - 1, x - 1.0);
                }
            }
            double g[3] = {0, 0, 0};
            for (int j0 = 0; j0 < p; ++j0)
                for (int j1 = 0; j1 < p; ++j1)
                    for (int j2 = 0; j2 < p; ++j2) {
                        int g0 = ((k0[0] - j0) % K[0] + K[0]) % K[0];
                        int g1 = ((k0[1] - j1) % K[1] + K[1]) % K[1];
                        int g2 = ((k0[2] - j2) % K[2] + K[2]) % K[2];
                        double ph = Q[2 * (((size_t)g0 * K[1] + g1) * K[2] + g2)];
                        g[0] += dw[0][j0] * w[1][j1] * w[2][j2] * ph;
                        g[1] += w[0][j0] * dw[1][j1] * w[2][j2] * ph;
                        g[2] += w[0][j0] * w[1][j1] * dw[2][j2] * ph;
                    }
            for (int a = 0; a < 3; ++a) F[3 * i + a] = -lB * z[i] * g[a] * K[a] / box[a];
        }
    }
    free(Q);
    for (int a = 0; a < 3; ++a) free(mod[a]);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Gaussian noise */
/* ------------------------------------------------------------------ */

static inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    __uint128_t p = (__uint128_t)a * (__uint128_t)b;
    *hi = (uint64_t)(p >> 64);
    *lo = (uint64_t)p;
}

void gco_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B97F4A7C15ULL; /* golden ratio */
            k1 += 0xBB67AE8584CAA73BULL; /* sqrt(3) - 1 */
        }
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(0xD2E7470EE14C6C93ULL, x0, &hi0, &lo0);
        mulhilo64(0xCA5A826395121157ULL, x2, &hi1, &lo1);
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Three standard normals for (seed, step, bead id, replica):
 * counter = (step, id, replica, 0), key = (seed, 0x67636d65);
 * u_k = ((x_k >> 11) + 0.5) 2^-53 in (0,1); Box-Muller on (u0,u1) and (u2,u3). */
void gco_gauss3(uint64_t seed, uint64_t step, uint64_t id, uint64_t replica, double out[3]) {
    uint64_t ctr[4] = {step, id, replica, 0};
    uint64_t key[2] = {seed, 0x67636d65ULL};
    uint64_t x[4];
    gco_philox4x64_10(ctr, key, x);
    double u[4];
    for (int k = 0; k < 4; ++k) u[k] = ((double)(x[k] >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    out[0] = r0 * cos(2.0 * M_PI * u[1]);
    out[1] = r0 * sin(2.0 * M_PI * u[1]);
    out[2] = r1 * cos(2.0 * M_PI * u[3]);
}

/* ------------------------------------------------------------------ */
/* Full force field and integrators                                     */
/* ------------------------------------------------------------------ */

enum { GCO_RECIP_NONE = 0, GCO_RECIP_EWALD = 1, GCO_RECIP_SPME = 2 };

typedef struct {
    int mode;       /* GCO_RECIP_* */
    double kmax;    /* exact sum */
    int K[3];       /* SPME grid */
    int order;      /* SPME order */
} gco_recip;

/* Total forces (AoS) and energy terms E[5] = {ex, real, recip, corr, self}. */
int gco_forces(int N, const double* pos, const int* type, const int* z, const gco_params* p,
               const gco_recip* rec, double* F, double* E, double* W) {
    double E2[2], Wr[6] = {0, 0, 0, 0, 0, 0}, Wk[6] = {0, 0, 0, 0, 0, 0};
    int rc = gco_real_space(N, pos, type, z, p, 1, 0, NULL, F, E2, Wr, NULL, NULL, NULL);
    if (rc) return rc;
    double er = 0;
    double* Fk = (double*)calloc((size_t)3 * N, sizeof(double));
    if (rec->mode == GCO_RECIP_EWALD)
        gco_ewald_recip(N, pos, z, p->box, p->beta, p->lB, rec->kmax, Fk, &er, Wk);
    else if (rec->mode == GCO_RECIP_SPME)
        gco_spme_recip(N, pos, z, p->box, p->beta, p->lB, rec->K, rec->order, Fk, &er, Wk, NULL);
    for (size_t i = 0; i < 3 * (size_t)N; ++i) F[i] += Fk[i];
    free(Fk);
    double ec, es;
    gco_constants(N, type, z, p, &ec, &es, NULL);
    if (E) { E[0] = E2[0]; E[1] = E2[1]; E[2] = er; E[3] = ec; E[4] = es; }
    if (W) for (int k = 0; k < 6; ++k) W[k] = Wr[k] + Wk[k];
    return 0;
}

/* Terms beyond the nonbonded force field, used by the slab systems of the
 * section on polyelectrolyte adsorption at electrodes. */
typedef struct {
    int slab;            /* 1: add the slab correction (gco_slab) */
    int nbonds;          /* harmonic bonds */
    const int* bonds;    /* [nbonds][2] bead indices */
    double bond_k, bond_b;
    int nimages;         /* image charges */
    const int* images;   /* [nimages][2] (image bead, source bead) */
} gco_extra;

/* Method of image charges (metal electrodes at z = 0 and z = Lz of the real
 * system, box length 2 Lz along z): each image bead sits at the source's
 * reflection across z = 0, (x, y, -z), wrapped into the box; its charge is
 * the source's with the opposite sign and it has no excluded volume (the
 * caller gives it such a type).  Both electrodes are mirror planes, since
 * the reflection across z = 0 followed by the period 2 Lz is the reflection
 * across z = Lz. */
void gco_mirror_images(double* pos, const double box[3], int nimg, const int* images) {
    for (int m = 0; m < nimg; ++m) {
        const int i = images[2 * m], s = images[2 * m + 1];
        pos[3 * i + 0] = pos[3 * s + 0];
        pos[3 * i + 1] = pos[3 * s + 1];
        pos[3 * i + 2] = wrapd(-pos[3 * s + 2], box[2]);
    }
}

/* Slab correction for a slab that is periodic in x and y and separated from
 * its periodic images along z by vacuum (the nonmetal-electrode systems,
 * whose box is tripled along z for it; the correction of Yeh and Berkowitz,
 * which the paper cites): the Ewald sum of such a box counts the
 * interaction of every slab with the dipoles of the others, and the term
 *   E = 2 pi lB M_z^2 / V,   M_z = sum_i z_i zeta_i
 * (zeta_i the z coordinate in [0, Lz)) corrects the tin-foil sum of eq.
 * ewald to the sum over a two-dimensionally periodic slab.  Forces
 * F_iz = -dE/dzeta_i = -4 pi lB z_i M_z / V.  Virial (-dE/d strain, the
 * convention of the reciprocal virial, for diagonal strains, under which
 * M_z scales with the zz strain and V with the trace): diag(E, E, -E).
 * Adds to F (AoS) and W (xx,yy,zz,xy,xz,yz); returns E. */
double gco_slab(int N, const double* pos, const int* z, const double box[3], double lB, double* F,
                double* W) {
    const double V = box[0] * box[1] * box[2];
    double Mz = 0.0;
    for (int i = 0; i < N; ++i) Mz += z[i] * wrapd(pos[3 * i + 2], box[2]);
    const double E = 2.0 * M_PI * lB * Mz * Mz / V;
    for (int i = 0; i < N; ++i) F[3 * i + 2] += -4.0 * M_PI * lB * z[i] * Mz / V;
    if (W) {
        W[0] += E;
        W[1] += E;
        W[2] -= E;
    }
    return E;
}

/* Harmonic bonds, u = k/2 (r - b)^2 over the minimum-image separation of
 * each listed pair (the polyanion backbone of the adsorption study, with
 * k = 100 and b = 0.8).  Bonded pairs keep their nonbonded terms (the paper
 * lists no exclusions).  Adds to F and W (sum over bonds of r_ij (x) f_ij);
 * returns E. */
double gco_bonds(int N, const double* pos, const double box[3], int nb, const int* bonds, double k,
                 double b, double* F, double* W) {
    (void)N;
    double E = 0.0;
    for (int m = 0; m < nb; ++m) {
        const int i = bonds[2 * m], j = bonds[2 * m + 1];
        double d[3], r2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = min_image(pos[3 * i + a] - pos[3 * j + a], box[a]);
            r2 += d[a] * d[a];
        }
        const double r = sqrt(r2);
        E += 0.5 * k * (r - b) * (r - b);
        /* force on i: -k (r - b) d / r */
        const double g = r > 0.0 ? -k * (r - b) / r : 0.0;
        for (int a = 0; a < 3; ++a) {
            F[3 * i + a] += g * d[a];
            F[3 * j + a] -= g * d[a];
        }
        if (W) {
            W[0] += d[0] * g * d[0];
            W[1] += d[1] * g * d[1];
            W[2] += d[2] * g * d[2];
            W[3] += d[0] * g * d[1];
            W[4] += d[0] * g * d[2];
            W[5] += d[1] * g * d[2];
        }
    }
    return E;
}

/* gco_forces plus the extra terms: E[7] = {ex, real, recip, corr, self,
 * slab, bond}. */
int gco_forces_ext(int N, const double* pos, const int* type, const int* z, const gco_params* p,
                   const gco_recip* rec, const gco_extra* ex, double* F, double* E, double* W) {
    int rc = gco_forces(N, pos, type, z, p, rec, F, E, W);
    if (rc) return rc;
    E[5] = E[6] = 0.0;
    if (ex && ex->slab) E[5] = gco_slab(N, pos, z, p->box, p->lB, F, W);
    if (ex && ex->nbonds > 0) E[6] = gco_bonds(N, pos, p->box, ex->nbonds, ex->bonds, ex->bond_k, ex->bond_b, F, W);
    return 0;
}

/* n_steps of velocity Verlet (gamma == 0) or BAOAB Langevin (gamma > 0).
 * State: pos, vel AoS [N][3]; F must hold the forces at pos on entry and
 * holds the forces at the final positions on exit.  mass per type.  Step s
 * (0-based within this call) draws noise with step counter step0 + s.
 * Positions are wrapped into [0, L) after each drift.  A type of infinite
 * mass is held fixed (the electrode lattices of the slab systems): no kick,
 * no noise, no kinetic energy; its beads must start at rest.  Image beads
 * (ex->images, of such a type) are moved to their sources' reflections after
 * every drift.  ex may be NULL.
 * Per-step potential + kinetic energies go to Elog[n_steps][2] if non-NULL. */
int gco_md(int N, double* pos, double* vel, double* F, const int* type, const int* z,
           const int* id, const gco_params* p, const gco_recip* rec, const gco_extra* ex,
           const double* mass, double dt, double gamma, double kT, uint64_t seed, uint64_t replica,
           uint64_t step0, int n_steps, double* Elog) {
    double c1 = exp(-gamma * dt);
    double c2 = sqrt(1.0 - c1 * c1);
    double E[7];
    for (int s = 0; s < n_steps; ++s) {
        for (int i = 0; i < N; ++i) {
            double m = mass[type[i]];
            for (int k = 0; k < 3; ++k) vel[3 * i + k] += 0.5 * dt * F[3 * i + k] / m;
            if (gamma > 0.0) {
                double xi[3];
                gco_gauss3(seed, step0 + (uint64_t)s, (uint64_t)id[i], replica, xi);
                for (int k = 0; k < 3; ++k) {
                    pos[3 * i + k] += 0.5 * dt * vel[3 * i + k];
                    vel[3 * i + k] = c1 * vel[3 * i + k] + c2 * sqrt(kT / m) * xi[k];
                    pos[3 * i + k] += 0.5 * dt * vel[3 * i + k];
                }
            } else {
                for (int k = 0; k < 3; ++k) pos[3 * i + k] += dt * vel[3 * i + k];
            }
            for (int k = 0; k < 3; ++k) pos[3 * i + k] = wrapd(pos[3 * i + k], p->box[k]);
        }
        if (ex && ex->nimages > 0) gco_mirror_images(pos, p->box, ex->nimages, ex->images);
        int rc = gco_forces_ext(N, pos, type, z, p, rec, ex, F, E, NULL);
        if (rc) return rc;
        double ke = 0;
        for (int i = 0; i < N; ++i) {
            double m = mass[type[i]];
            if (isinf(m)) continue;
            for (int k = 0; k < 3; ++k) {
                vel[3 * i + k] += 0.5 * dt * F[3 * i + k] / m;
                ke += 0.5 * m * vel[3 * i + k] * vel[3 * i + k];
            }
        }
        if (Elog) {
            Elog[2 * s] = E[0] + E[1] + E[2] + E[3] + E[4] + E[5] + E[6];
            Elog[2 * s + 1] = ke;
        }
    }
    return 0;
}

int gco_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
