/*
 * FP64 CPU oracle of the fugacity-based well-balanced multicomponent lattice
 * Boltzmann method (arXiv:2212.10680).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py through oracle/lbm.py.  The GPU library shares no
 * code, header, table or helper with this file.
 *
 * One time step follows the nine-step procedure of Sec. III.B literally, node by
 * node, in plain loops (OpenMP over nodes, no blocking, no fusion):
 *   1. rho_i = sum_a g_ai; rho = sum_i rho_i;
 *      u = (1/rho) sum_i [sum_a g_ai e_a + F_i dt/2], with F_i the force of the
 *      previous time step ("given the distribution functions and body forces ...
 *      from the previous time step");
 *   2. rho~_i = rho_i/M_i, rho~ = sum rho~_i, x_i = rho~_i/rho~;
 *   3. mixing rules (App. C, eqs. eqmixingrulesaSRK, eqmixingrulesbm);
 *   4. pressure from the EOS (eqPREOS / eqSRKEOS / eqvdwEOS);
 *   5. ln f_i from the density-explicit forms eqfugupdatePR / SRK / VDW (Sec. V);
 *   6. mu_I,i = -sum_j kappa_ij lap(rho~_j), kappa_ij = sqrt(kappa_i kappa_j)
 *      (eqs. eqChemPotI2, eqkappa) with the 3-point second difference eq2ndder;
 *   7. F_i = -rho~_i RT grad ln f_i - rho~_i grad mu_I,i (eq. eqforceFugLBM) with
 *      the central first difference eq1stder;
 *   8. g_eq (eq. eqLBEMCb with rho_0 = rho_0,i = 0) and the forcing term
 *      (eq. eqLBEMCfinal3, which needs grad rho_i, again by eq1stder);
 *   9. collision (eq. eqLBEMCa, BGK; or the MRT reading documented in
 *      oracle/lattice.py) and periodic streaming.
 * Lattice spacing and time step are 1.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXC 8
#define ORC_MAXQ 19

typedef struct {
    int D, Q;
    int nx, ny, nz;
    int nc;
    int eos;               /* 0 PR, 1 SRK, 2 vdW */
    int collision;         /* 0 BGK, 1 MRT */
    int force_level;       /* 0: u uses the previous step's force (literal step 1);
                              1: u uses this step's force */
    int standard_force;    /* 0: well-balanced (eqLBEMCb/eqLBEMCfinal3);
                              1: standard LBM variant (eqForceGen) */
    double RT;
    double tau;
    double cs2;
    double b[ORC_MAXC];
    double M[ORC_MAXC];
    double kappa[ORC_MAXC];
    double aaij[ORC_MAXC * ORC_MAXC];
    double e[ORC_MAXQ * 3];    /* lattice velocities, row-major [Q][3] */
    double w[ORC_MAXQ];
    double Mm[ORC_MAXQ * ORC_MAXQ];    /* MRT basis (rows = moments) */
    double Minv[ORC_MAXQ * ORC_MAXQ];
    double S[ORC_MAXQ];
    int stencil;           /* 0: the paper's axis stencils (eq1stder, eq2ndder);
                              1: isotropic lattice stencils (reading for 3-D droplets) */
} orc_params;

enum { ORC_OK = 0, ORC_EDOMAIN = -2, ORC_ENOMEM = -3 };

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static long nnodes(const orc_params* P) { return (long)P->nx * P->ny * P->nz; }

/* node index with periodic wrap */
static long nidx(const orc_params* P, long x, long y, long z) {
    x = ((x % P->nx) + P->nx) % P->nx;
    y = ((y % P->ny) + P->ny) % P->ny;
    z = ((z % P->nz) + P->nz) % P->nz;
    return x + (long)P->nx * (y + (long)P->ny * z);
}

static void ncoord(const orc_params* P, long n, long* x, long* y, long* z) {
    *x = n % P->nx;
    *y = (n / P->nx) % P->ny;
    *z = n / ((long)P->nx * P->ny);
}

/* Steps 3-5 at one node: mixing rules, pressure and ln f_i from molar densities.
 * Returns 0, or ORC_EDOMAIN when a density is not positive or rho~ b_m >= 1. */
int orc_eos(const orc_params* P, const double* rt_i, double* p_out, double* lnf) {
    const int nc = P->nc;
    double rt = 0.0;
    for (int i = 0; i < nc; ++i) {
        if (!(rt_i[i] > 0.0)) return ORC_EDOMAIN;
        rt += rt_i[i];
    }
    double x[ORC_MAXC], s[ORC_MAXC];
    for (int i = 0; i < nc; ++i) x[i] = rt_i[i] / rt;
    /* mixing rules: b_m = sum x_i b_i; (a alpha)_m = sum_i sum_j x_i x_j (a alpha)_ij */
    double bm = 0.0, am = 0.0;
    for (int i = 0; i < nc; ++i) bm += x[i] * P->b[i];
    for (int i = 0; i < nc; ++i) {
        s[i] = 0.0;
        for (int j = 0; j < nc; ++j) s[i] += x[j] * P->aaij[i * nc + j];
        am += x[i] * s[i];
    }
    const double v = 1.0 / rt;
    const double RT = P->RT;
    if (!(v - bm > 0.0)) return ORC_EDOMAIN;
    double p;
    if (P->eos == 0)       /* PR, eqPREOS */
        p = RT / (v - bm) - am / (v * v + 2.0 * bm * v - bm * bm);
    else if (P->eos == 1)  /* SRK, eqSRKEOS */
        p = RT / (v - bm) - am / (v * (v + bm));
    else                   /* vdW, eqvdwEOS */
        p = RT / (v - bm) - am / (v * v);
    if (p_out) *p_out = p;
    for (int i = 0; i < nc; ++i) {
        double l;
        if (P->eos == 2) {
            /* eqfugupdateVDW */
            l = log(x[i]) + P->b[i] / (v - bm) - log((v - bm) / RT) - 2.0 / (RT * v) * s[i];
        } else {
            l = log(x[i]) + P->b[i] / bm * (p * v / RT - 1.0) - log((v - bm) / RT);
            double bracket = P->b[i] / bm - 2.0 / am * s[i];
            if (P->eos == 0) {
                /* eqfugupdatePR */
                const double r2 = sqrt(2.0);
                l += am / (2.0 * r2 * bm * RT) * bracket *
                     log((v + (1.0 + r2) * bm) / (v + (1.0 - r2) * bm));
            } else {
                /* eqfugupdateSRK */
                l += am / (bm * RT) * bracket * log(1.0 + bm / v);
            }
        }
        lnf[i] = l;
    }
    return ORC_OK;
}

/* Step 8, equilibrium of eqLBEMCb with rho_0 = rho_0,i = 0 (well-balanced), or
 * the standard equilibrium of eqLBE when standard != 0. */
void orc_equilibrium(const orc_params* P, double rho_i, const double* u, double* geq) {
    const double cs2 = P->cs2;
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int a = 0; a < P->Q; ++a) {
        const double* e = &P->e[3 * a];
        const double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
        const double bracket = eu / cs2 + eu * eu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2);
        if (P->standard_force)
            geq[a] = P->w[a] * rho_i * (1.0 + bracket);
        else if (a == 0)
            geq[a] = rho_i + P->w[0] * rho_i * bracket;
        else
            geq[a] = P->w[a] * rho_i * bracket;
    }
}

/* Step 8, forcing term of eqLBEMCfinal3 (the grad rho_i part is dropped for the
 * standard-LBM variant, which uses eqLBEfinal3 instead). */
void orc_forcing(const orc_params* P, const double* F, const double* grho, const double* u,
                 double* Fa) {
    const double cs2 = P->cs2;
    const int D = P->D;
    for (int a = 0; a < P->Q; ++a) {
        const double* e = &P->e[3 * a];
        const double eu = e[0] * u[0] + e[1] * u[1] + e[2] * u[2];
        const double e2 = e[0] * e[0] + e[1] * e[1] + e[2] * e[2];
        double t1 = 0.0, t2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            t1 += F[k] * ((e[k] - u[k]) / cs2 + eu * e[k] / (cs2 * cs2));
            t2 += grho[k] * (-u[k] + eu * e[k] / cs2 + 0.5 * (e2 / cs2 - D) * u[k]);
        }
        Fa[a] = P->w[a] * t1 + (P->standard_force ? 0.0 : P->w[a] * t2);
    }
}

/* Step 9, collision of one component at one node. */
static void collide(const orc_params* P, const double* g, const double* geq, const double* Fa,
                    double* gs) {
    const int Q = P->Q;
    if (P->collision == 0) {
        /* eqLBEMCa: g* = g - (g - g_eq)/tau + (1 - 1/(2 tau)) F_a */
        for (int a = 0; a < Q; ++a)
            gs[a] = g[a] - (g[a] - geq[a]) / P->tau + (1.0 - 1.0 / (2.0 * P->tau)) * Fa[a];
        return;
    }
    /* MRT: m = M g; m* = m - S (m - m_eq) + (I - S/2) M F; g* = M^-1 m* */
    double m[ORC_MAXQ], meq[ORC_MAXQ], mF[ORC_MAXQ], ms[ORC_MAXQ];
    for (int k = 0; k < Q; ++k) {
        m[k] = meq[k] = mF[k] = 0.0;
        for (int a = 0; a < Q; ++a) {
            m[k] += P->Mm[k * Q + a] * g[a];
            meq[k] += P->Mm[k * Q + a] * geq[a];
            mF[k] += P->Mm[k * Q + a] * Fa[a];
        }
        ms[k] = m[k] - P->S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * P->S[k]) * mF[k];
    }
    for (int a = 0; a < Q; ++a) {
        gs[a] = 0.0;
        for (int k = 0; k < Q; ++k) gs[a] += P->Minv[a * Q + k] * ms[k];
    }
}

/* Macroscopic fields of the current state (steps 1-5 and 6-7 of one step,
 * without collision).  Any output may be NULL.  rho_molar/lnf are [nc][N],
 * u [D][N], p [N], force [nc][D][N] (this step's F_i).  Returns the first
 * domain error or 0. */
/* Isotropic lattice stencils (the weights and velocities of the lattice):
 * grad f = (1/c_s^2) sum_a w_a e_a f(x + e_a), lap f = (2/c_s^2) sum_a w_a
 * (f(x + e_a) - f(x)); on a field that varies along one axis they reduce to
 * the central differences of eq1stder and eq2ndder. */
static double iso_grad(const orc_params* P, const double* f, long x, long y, long z, int k) {
    double s = 0.0;
    for (int a = 1; a < P->Q; ++a) {
        const double* e = &P->e[3 * a];
        if (e[k] != 0.0) s += P->w[a] * e[k] * f[nidx(P, x + (long)e[0], y + (long)e[1], z + (long)e[2])];
    }
    return s / P->cs2;
}

static double iso_lap(const orc_params* P, const double* f, long n, long x, long y, long z) {
    double s = 0.0;
    for (int a = 1; a < P->Q; ++a) {
        const double* e = &P->e[3 * a];
        s += P->w[a] * (f[nidx(P, x + (long)e[0], y + (long)e[1], z + (long)e[2])] - f[n]);
    }
    return 2.0 * s / P->cs2;
}

static int fields_and_force(const orc_params* P, const double* g, const double* fprev,
                            double* rho_i, double* jm, double* u, double* rt_i, double* p,
                            double* lnf, double* mu_i, double* force, long* bad_node) {
    const long N = nnodes(P);
    const int nc = P->nc, Q = P->Q, D = P->D;
    int err = ORC_OK;
    long bad = -1;
    /* steps 1-5 */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
        double rtn[ORC_MAXC], lf[ORC_MAXC], pn;
        for (int i = 0; i < nc; ++i) {
            double r = 0.0;
            for (int a = 0; a < Q; ++a) {
                const double ga = g[((long)i * Q + a) * N + n];
                r += ga;
                for (int k = 0; k < 3; ++k) j[k] += ga * P->e[3 * a + k];
            }
            rho_i[(long)i * N + n] = r;
            rho += r;
            rtn[i] = r / P->M[i];
            rt_i[(long)i * N + n] = rtn[i];
        }
        for (int k = 0; k < D; ++k) {
            jm[(long)k * N + n] = j[k];
            u[(long)k * N + n] = (j[k] + 0.5 * fprev[(long)k * N + n]) / rho;
        }
        int e = orc_eos(P, rtn, &pn, lf);
        if (e != ORC_OK) {
#pragma omp critical
            {
                if (bad < 0 || n < bad) { bad = n; err = e; }
            }
            continue;
        }
        p[n] = pn;
        for (int i = 0; i < nc; ++i) lnf[(long)i * N + n] = lf[i];
    }
    if (err != ORC_OK) {
        if (bad_node) *bad_node = bad;
        return err;
    }
    /* step 6: mu_I,i = -sum_j sqrt(kappa_i kappa_j) lap rho~_j */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < N; ++n) {
        long x, y, z;
        ncoord(P, n, &x, &y, &z);
        double lap[ORC_MAXC];
        for (int jc = 0; jc < nc; ++jc) {
            const double* r = rt_i + (long)jc * N;
            double L = 0.0;
            if (P->stencil == 1) {
                L = iso_lap(P, r, n, x, y, z);
            } else {
                for (int k = 0; k < D; ++k) {
                    const long dx = (k == 0), dy = (k == 1), dz = (k == 2);
                    L += r[nidx(P, x + dx, y + dy, z + dz)] - 2.0 * r[n] + r[nidx(P, x - dx, y - dy, z - dz)];
                }
            }
            lap[jc] = L;
        }
        for (int i = 0; i < nc; ++i) {
            double m = 0.0;
            for (int jc = 0; jc < nc; ++jc) m -= sqrt(P->kappa[i] * P->kappa[jc]) * lap[jc];
            mu_i[(long)i * N + n] = m;
        }
    }
    /* step 7: F_i = -rho~_i [RT grad ln f_i + grad mu_I,i] */
    if (force) {
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            long x, y, z;
            ncoord(P, n, &x, &y, &z);
            for (int i = 0; i < nc; ++i) {
                const double* lf = lnf + (long)i * N;
                const double* mu = mu_i + (long)i * N;
                for (int k = 0; k < D; ++k) {
                    const long dx = (k == 0), dy = (k == 1), dz = (k == 2);
                    const long np = nidx(P, x + dx, y + dy, z + dz), nm = nidx(P, x - dx, y - dy, z - dz);
                    const int iso = P->stencil == 1;
                    const double dlnf = iso ? iso_grad(P, lf, x, y, z, k) : (lf[np] - lf[nm]) / 2.0;
                    const double dmu = iso ? iso_grad(P, mu, x, y, z, k) : (mu[np] - mu[nm]) / 2.0;
                    double Fk = -rt_i[(long)i * N + n] * (P->RT * dlnf + dmu);
                    if (P->standard_force) {
                        /* eqForceGen: + c_s^2 grad rho_i */
                        const double* ri = rho_i + (long)i * N;
                        Fk += P->cs2 * (iso ? iso_grad(P, ri, x, y, z, k) : (ri[np] - ri[nm]) / 2.0);
                    }
                    force[((long)i * D + k) * N + n] = Fk;
                }
            }
        }
    }
    return ORC_OK;
}

typedef struct {
    double *rho_i, *j, *u, *rt_i, *p, *lnf, *mu, *force;
} orc_work;

static int work_alloc(const orc_params* P, orc_work* W) {
    const long N = nnodes(P);
    const int nc = P->nc, D = P->D;
    W->rho_i = malloc(sizeof(double) * nc * N);
    W->u = malloc(sizeof(double) * D * N);
    W->j = malloc(sizeof(double) * D * N);
    W->rt_i = malloc(sizeof(double) * nc * N);
    W->p = malloc(sizeof(double) * N);
    W->lnf = malloc(sizeof(double) * nc * N);
    W->mu = malloc(sizeof(double) * nc * N);
    W->force = malloc(sizeof(double) * nc * D * N);
    if (!W->rho_i || !W->u || !W->j || !W->rt_i || !W->p || !W->lnf || !W->mu || !W->force) return ORC_ENOMEM;
    return ORC_OK;
}

static void work_free(orc_work* W) {
    free(W->rho_i); free(W->u); free(W->j); free(W->rt_i); free(W->p); free(W->lnf); free(W->mu); free(W->force);
}

/* Advance nsteps.  g: populations [nc][Q][N] (updated in place);
 * fprev: sum_i F_i of the previous step [D][N] (updated in place).
 * On a domain error returns ORC_EDOMAIN, *steps_done = completed steps,
 * *bad_node = first offending node; g and fprev then hold the last good state. */
int orc_run(const orc_params* P, double* g, double* fprev, long nsteps, long* steps_done,
            long* bad_node) {
    const long N = nnodes(P);
    const int nc = P->nc, Q = P->Q, D = P->D;
    orc_work W;
    double* gn = malloc(sizeof(double) * nc * Q * N);
    if (!gn || work_alloc(P, &W) != ORC_OK) { free(gn); return ORC_ENOMEM; }
    int err = ORC_OK;
    long s;
    for (s = 0; s < nsteps; ++s) {
        err = fields_and_force(P, g, fprev, W.rho_i, W.j, W.u, W.rt_i, W.p, W.lnf, W.mu, W.force, bad_node);
        if (err != ORC_OK) break;
        /* steps 8-9 per node; streaming writes node x + e_a of the new lattice */
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n) {
            long x, y, z;
            ncoord(P, n, &x, &y, &z);
            double u[3] = {0.0, 0.0, 0.0};
            double Fsum[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < nc; ++i)
                for (int k = 0; k < D; ++k) Fsum[k] += W.force[((long)i * D + k) * N + n];
            for (int k = 0; k < D; ++k) u[k] = W.u[(long)k * N + n];
            if (P->force_level == 1) {
                /* same-step variant: u = (sum_i j_i + sum_i F_i^n / 2) / rho */
                double rho = 0.0;
                for (int i = 0; i < nc; ++i) rho += W.rho_i[(long)i * N + n];
                for (int k = 0; k < D; ++k) u[k] = (W.j[(long)k * N + n] + 0.5 * Fsum[k]) / rho;
            }
            for (int i = 0; i < nc; ++i) {
                double ga[ORC_MAXQ], geq[ORC_MAXQ], Fa[ORC_MAXQ], gs[ORC_MAXQ];
                double F[3] = {0.0, 0.0, 0.0}, grho[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < D; ++k) {
                    const long dx = (k == 0), dy = (k == 1), dz = (k == 2);
                    const double* ri = W.rho_i + (long)i * N;
                    F[k] = W.force[((long)i * D + k) * N + n];
                    grho[k] = P->stencil == 1
                                  ? iso_grad(P, ri, x, y, z, k)
                                  : (ri[nidx(P, x + dx, y + dy, z + dz)] - ri[nidx(P, x - dx, y - dy, z - dz)]) / 2.0;
                }
                for (int a = 0; a < Q; ++a) ga[a] = g[((long)i * Q + a) * N + n];
                orc_equilibrium(P, W.rho_i[(long)i * N + n], u, geq);
                orc_forcing(P, F, grho, u, Fa);
                collide(P, ga, geq, Fa, gs);
                for (int a = 0; a < Q; ++a) {
                    const long dst = nidx(P, x + (long)P->e[3 * a], y + (long)P->e[3 * a + 1],
                                          z + (long)P->e[3 * a + 2]);
                    gn[((long)i * Q + a) * N + dst] = gs[a];
                }
            }
        }
        /* keep this step's force for the next step's velocity (step 1) */
#pragma omp parallel for schedule(static)
        for (long n = 0; n < N; ++n)
            for (int k = 0; k < D; ++k) {
                double f = 0.0;
                for (int i = 0; i < nc; ++i) f += W.force[((long)i * D + k) * N + n];
                fprev[(long)k * N + n] = f;
            }
        memcpy(g, gn, sizeof(double) * nc * Q * N);
    }
    if (steps_done) *steps_done = s;
    free(gn);
    work_free(&W);
    return err;
}

/* Populations at equilibrium with the given molar densities [nc][N] and
 * velocity [D][N] (u may be NULL for rest); the force history is zero. */
void orc_init(const orc_params* P, const double* rho_molar, const double* u, double* g,
              double* fprev) {
    const long N = nnodes(P);
    const int nc = P->nc, Q = P->Q, D = P->D;
    for (long n = 0; n < N; ++n) {
        double un[3] = {0.0, 0.0, 0.0};
        if (u)
            for (int k = 0; k < D; ++k) un[k] = u[(long)k * N + n];
        for (int i = 0; i < nc; ++i) {
            double geq[ORC_MAXQ];
            orc_equilibrium(P, rho_molar[(long)i * N + n] * P->M[i], un, geq);
            for (int a = 0; a < Q; ++a) g[((long)i * Q + a) * N + n] = geq[a];
        }
        for (int k = 0; k < D; ++k) fprev[(long)k * N + n] = 0.0;
    }
}

/* Macroscopic fields of the current state: molar densities [nc][N],
 * velocity of step 1 [D][N], EOS pressure [N], ln f [nc][N], this step's
 * force [nc][D][N] and interface potential [nc][N]; any may be NULL. */
int orc_fields(const orc_params* P, const double* g, const double* fprev, double* rho_molar,
               double* u, double* p, double* lnf, double* force, double* mu_I) {
    const long N = nnodes(P);
    const int nc = P->nc, D = P->D;
    orc_work W;
    if (work_alloc(P, &W) != ORC_OK) { work_free(&W); return ORC_ENOMEM; }
    long bad = -1;
    int err = fields_and_force(P, g, fprev, W.rho_i, W.j, W.u, W.rt_i, W.p, W.lnf, W.mu, W.force, &bad);
    if (err == ORC_OK) {
        if (rho_molar) memcpy(rho_molar, W.rt_i, sizeof(double) * nc * N);
        if (u) memcpy(u, W.u, sizeof(double) * D * N);
        if (p) memcpy(p, W.p, sizeof(double) * N);
        if (lnf) memcpy(lnf, W.lnf, sizeof(double) * nc * N);
        if (force) memcpy(force, W.force, sizeof(double) * nc * D * N);
        if (mu_I) memcpy(mu_I, W.mu, sizeof(double) * nc * N);
    }
    work_free(&W);
    return err;
}

/* The isotropic stencils of one scalar field f [N] at every node, for checks
 * of the stencils on their own: grad [3][N] (rows beyond D are zero) and
 * lap [N]. */
void orc_iso_stencils(const orc_params* P, const double* f, double* grad, double* lap) {
    const long N = nnodes(P);
    for (long n = 0; n < N; ++n) {
        long x, y, z;
        ncoord(P, n, &x, &y, &z);
        for (int k = 0; k < 3; ++k) grad[(long)k * N + n] = k < P->D ? iso_grad(P, f, x, y, z, k) : 0.0;
        lap[n] = iso_lap(P, f, n, x, y, z);
    }
}

/* Host threads of the OpenMP loops (timing on one core, or on all). */
void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
