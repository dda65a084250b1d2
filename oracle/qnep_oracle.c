/*
 * qnep_oracle.c -- plain FP64 CPU reference of the qNEP force evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library.  It shares no code with the HIP
 * path (no headers, helpers, tables or constants); only the seeded input arrays
 * are common to both.
 *
 * Everything here follows the definitions of arXiv:2601.19034 (qNEP) written out
 * directly, in double precision, with no blocking, fusion or reordering beyond what
 * the definitions state:
 *   - neighbours by brute force over periodic images (a cell-list variant is
 *     checked against it);
 *   - NEP radial and angular descriptors in the published NEP3/NEP4 form (the
 *     paper defers their definition to the GPUMD/NEP references, Sec. 2.1); the
 *     angular descriptor is the Legendre double sum over neighbour pairs;
 *   - the single-hidden-layer network with an energy and a charge output
 *     (Sec. 2.1 Eq. 1, Sec. 2.2);
 *   - charge scaling and the neutrality correction (Sec. 2.4 Eq. 24, Sec. 2.5 Eq. 33);
 *   - real-space, reciprocal-space (direct Ewald) and self energies (Sec. 2.2.1-2.2.3,
 *     Eqs. 6-10), or PPPM with the optimized influence function (Sec. 2.6, Eqs. 34-38)
 *     using a separable direct DFT on the mesh;
 *   - analytic forces and virial with the static and dynamic-charge terms
 *     (Sec. 2.3, Eqs. 11-23), Born effective charges in the periodic form
 *     (Sec. 2.4 Eq. 28) and the polarization (Eq. 26).
 *
 * Readings where the paper is silent or garbled:
 *   - neutrality correction:  q~'_i = q~_i + (Q - sum_j q~_j)/N  (the printed sign
 *     would double the net charge);
 *   - its derivative: dE/dq_i = phi_i - mean(phi) (exact chain rule);
 *   - U_ES uses the screened charges q' = q~'/s with k_e; P and Z* use q~';
 *   - the influence function's denominator is squared and its z^6 coefficient is
 *     -17/189 (the value of the P = 5 alias sum);
 *   - the PPPM virial uses the Ewald stress kernel B(k) with G_opt in place of G;
 *   - background term -k_e pi Q'^2 / (2 Omega alpha^2) in mode 1 for Q != 0;
 *   - per-atom virial W_i = sum_j r_ij (x) F_ji over every partial force, the static
 *     real-space pair virial shared equally, the reciprocal per-atom forms, and the
 *     background virial split evenly over the atoms;
 *   - an external field E adds F_i += sum_a E_a Z_i[a][:] (Eq. 29) to the forces only
 *     (no energy or virial term: the paper gives the force alone);
 *   - isolated systems (no periodic images): direct Coulomb sum over all pairs and the
 *     Born charges of Eq. 27, the derivative of P with absolute positions.
 *
 * Units: eV, Angstrom, elementary charge.  Virial W = -dE/d(strain).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_KE 14.399645 /* e^2/(4 pi eps0) in eV*Angstrom */
#define ORC_PI 3.14159265358979323846
#define ORC_MAXB 32      /* largest Chebyshev order handled */
#define ORC_MAXL 8       /* largest angular order handled */

typedef struct {
    int n_types, n_max_R, n_max_A, basis_R, basis_A, l_max, n_neu;
    double rc_R, rc_A;
} oq_hparams;

typedef struct {
    int mode;            /* 1: real + reciprocal + self; 2: reciprocal only (Eq. 5) */
    int method;          /* 0: direct Ewald; 1: PPPM */
    double alpha, rc_coul, kmax;
    int kmax_inclusive;  /* 1: |k| <= kmax, 0: |k| < kmax */
    int mesh[3];
    int order;           /* assignment order P (5, Sec. 2.6) */
    double q_total;      /* target total charge Q */
    double efield[3];    /* external electric field E (V/Angstrom), Sec. 2.4 */
} oq_es;

/* any pointer may be NULL */
typedef struct {
    double *terms;        /* [10]: E, U_NEP, U_r, U_k, U_s, U_bg, sum q_raw, mean phi, sum q~', n_k */
    double *forces;       /* N*3 */
    double *virial;       /* 9, W[a][b] */
    double *q_screened;   /* N: q'_i */
    double *q_naked;      /* N: q~'_i */
    double *q_raw;        /* N: network output q_i */
    double *bec;          /* N*9: Z[i][a][b] */
    double *pol;          /* 3 */
    double *desc;         /* N*n_des */
    double *site_energy;  /* N */
    double *phi;          /* N: dU_ES/dq'_i */
    double *vatom;        /* N*9: per-atom virial W_i[a][b] (Sec. 2.3 Eq. 12 and the per-atom reciprocal terms) */
} oq_out;

/* ------------------------------------------------------------------ */
/* cell geometry (rows of h are the cell vectors a, b, c)               */
/* ------------------------------------------------------------------ */
static double det3(const double *h)
{
    return h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
           h[2] * (h[3] * h[7] - h[4] * h[6]);
}

static void inv3(const double *h, double *o)
{
    double d = det3(h);
    o[0] = (h[4] * h[8] - h[5] * h[7]) / d;
    o[1] = (h[2] * h[7] - h[1] * h[8]) / d;
    o[2] = (h[1] * h[5] - h[2] * h[4]) / d;
    o[3] = (h[5] * h[6] - h[3] * h[8]) / d;
    o[4] = (h[0] * h[8] - h[2] * h[6]) / d;
    o[5] = (h[2] * h[3] - h[0] * h[5]) / d;
    o[6] = (h[3] * h[7] - h[4] * h[6]) / d;
    o[7] = (h[1] * h[6] - h[0] * h[7]) / d;
    o[8] = (h[0] * h[4] - h[1] * h[3]) / d;
}

/* perpendicular widths: Omega / |b x c| and cyclic */
static void cell_widths(const double *h, double *w)
{
    double vol = fabs(det3(h));
    for (int a = 0; a < 3; ++a) {
        const double *u = h + 3 * ((a + 1) % 3), *v = h + 3 * ((a + 2) % 3);
        double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
        w[a] = vol / sqrt(cx * cx + cy * cy + cz * cz);
    }
}

/* fractional coordinates s = r h^{-1} wrapped into [0,1), and wrapped positions */
static void wrap_positions(int n, const double *pos, const double *h, double *frac, double *wpos)
{
    double hi[9];
    inv3(h, hi);
    for (int i = 0; i < n; ++i) {
        for (int a = 0; a < 3; ++a) {
            double s = pos[3 * i] * hi[a] + pos[3 * i + 1] * hi[3 + a] + pos[3 * i + 2] * hi[6 + a];
            s -= floor(s);
            if (s >= 1.0) s -= 1.0;
            frac[3 * i + a] = s;
        }
        for (int b = 0; b < 3; ++b)
            wpos[3 * i + b] = frac[3 * i] * h[b] + frac[3 * i + 1] * h[3 + b] + frac[3 * i + 2] * h[6 + b];
    }
}

/* ------------------------------------------------------------------ */
/* neighbour lists: every (j, image n) with |r_j + n.h - r_i| < rc and  */
/* (j, n) != (i, 0); d = r_ij = r_j(image) - r_i (Eq. 13)               */
/* ------------------------------------------------------------------ */
typedef struct { int j; double d[3]; double r; } oq_pair;
typedef struct { int n, cap; oq_pair *p; } oq_plist;

static void plist_push(oq_plist *L, int j, const double *d, double r)
{
    if (L->n == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 64;
        L->p = (oq_pair *)realloc(L->p, sizeof(oq_pair) * (size_t)L->cap);
    }
    oq_pair *q = &L->p[L->n++];
    q->j = j;
    q->d[0] = d[0]; q->d[1] = d[1]; q->d[2] = d[2];
    q->r = r;
}

static void free_lists(int n, oq_plist *L)
{
    if (!L) return;
    for (int i = 0; i < n; ++i) free(L[i].p);
    free(L);
}

static oq_plist *nbr_brute(int n, const double *wpos, const double *h, double rc)
{
    oq_plist *L = (oq_plist *)calloc((size_t)(n > 0 ? n : 1), sizeof(oq_plist));
    double w[3];
    cell_widths(h, w);
    int m[3];
    for (int a = 0; a < 3; ++a) m[a] = (int)floor(rc / w[a]) + 1;
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j)
            for (int n1 = -m[0]; n1 <= m[0]; ++n1)
                for (int n2 = -m[1]; n2 <= m[1]; ++n2)
                    for (int n3 = -m[2]; n3 <= m[2]; ++n3) {
                        if (i == j && n1 == 0 && n2 == 0 && n3 == 0) continue;
                        double d[3];
                        for (int b = 0; b < 3; ++b)
                            d[b] = wpos[3 * j + b] - wpos[3 * i + b] + n1 * h[b] + n2 * h[3 + b] + n3 * h[6 + b];
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < rc2) plist_push(&L[i], j, d, sqrt(r2));
                    }
    }
    return L;
}

/* cell-list variant: cells no thinner than rc and a 3x3x3 stencil; boxes with
   fewer than three cells along an axis use the brute-force search */
static oq_plist *nbr_cells(int n, const double *frac, const double *wpos, const double *h, double rc)
{
    double w[3];
    cell_widths(h, w);
    int nc[3];
    for (int a = 0; a < 3; ++a) nc[a] = (int)floor(w[a] / rc);
    if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) return nbr_brute(n, wpos, h, rc);
    int ncell = nc[0] * nc[1] * nc[2];
    int nn = n > 0 ? n : 1;
    int *head = (int *)malloc(sizeof(int) * (size_t)ncell), *next = (int *)malloc(sizeof(int) * (size_t)nn);
    int *cid = (int *)malloc(sizeof(int) * 3 * (size_t)nn);
    for (int c = 0; c < ncell; ++c) head[c] = -1;
    for (int i = n - 1; i >= 0; --i) {
        int c[3];
        for (int a = 0; a < 3; ++a) {
            c[a] = (int)floor(frac[3 * i + a] * nc[a]);
            if (c[a] >= nc[a]) c[a] = nc[a] - 1;
            cid[3 * i + a] = c[a];
        }
        int lin = (c[0] * nc[1] + c[1]) * nc[2] + c[2];
        next[i] = head[lin];
        head[lin] = i;
    }
    oq_plist *L = (oq_plist *)calloc((size_t)nn, sizeof(oq_plist));
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        for (int d0 = -1; d0 <= 1; ++d0)
            for (int d1 = -1; d1 <= 1; ++d1)
                for (int d2 = -1; d2 <= 1; ++d2) {
                    int cc[3] = {cid[3 * i] + d0, cid[3 * i + 1] + d1, cid[3 * i + 2] + d2}, img[3];
                    for (int a = 0; a < 3; ++a) {
                        img[a] = (int)floor((double)cc[a] / nc[a]);
                        cc[a] -= img[a] * nc[a];
                    }
                    int lin = (cc[0] * nc[1] + cc[1]) * nc[2] + cc[2];
                    for (int j = head[lin]; j >= 0; j = next[j]) {
                        if (j == i && img[0] == 0 && img[1] == 0 && img[2] == 0) continue;
                        double d[3];
                        for (int b = 0; b < 3; ++b)
                            d[b] = wpos[3 * j + b] - wpos[3 * i + b] + img[0] * h[b] + img[1] * h[3 + b] +
                                   img[2] * h[6 + b];
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (r2 < rc2) plist_push(&L[i], j, d, sqrt(r2));
                    }
                }
    }
    free(head); free(next); free(cid);
    return L;
}

static oq_plist *build_list(int method, int n, const double *frac, const double *wpos, const double *h, double rc)
{
    return method == 1 ? nbr_cells(n, frac, wpos, h, rc) : nbr_brute(n, wpos, h, rc);
}

/* isolated system: every j != i with |r_j - r_i| < rc, no periodic images */
static oq_plist *nbr_free(int n, const double *pos, double rc)
{
    oq_plist *L = (oq_plist *)calloc((size_t)(n > 0 ? n : 1), sizeof(oq_plist));
    double rc2 = rc * rc;
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            for (int b = 0; b < 3; ++b) d[b] = pos[3 * j + b] - pos[3 * i + b];
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) plist_push(&L[i], j, d, sqrt(r2));
        }
    return L;
}

/* exported for the tests: per-atom neighbour counts and, when js/ds are given,
   the neighbours themselves (index and distance), cap entries per atom */
int oq_neighbors(int method, int n, const double *pos, const double *h, double rc, int *counts, int *js,
                 double *ds, int cap)
{
    int nn = n > 0 ? n : 1;
    double *frac = (double *)malloc(sizeof(double) * 3 * (size_t)nn), *wpos = (double *)malloc(sizeof(double) * 3 * (size_t)nn);
    wrap_positions(n, pos, h, frac, wpos);
    oq_plist *L = build_list(method, n, frac, wpos, h, rc);
    int overflow = 0;
    for (int i = 0; i < n; ++i) {
        counts[i] = L[i].n;
        if (js && ds)
            for (int p = 0; p < L[i].n; ++p) {
                if (p >= cap) { overflow = 1; break; }
                js[(size_t)i * cap + p] = L[i].p[p].j;
                ds[(size_t)i * cap + p] = L[i].p[p].r;
            }
    }
    free_lists(n, L);
    free(frac); free(wpos);
    return overflow;
}

/* ------------------------------------------------------------------ */
/* NEP radial basis (published NEP form, Sec. 2.1 references):          */
/*   f_c(r) = (1 + cos(pi r / rc)) / 2                                  */
/*   f_k(r) = (T_k(2 (r/rc - 1)^2 - 1) + 1) / 2 * f_c(r), k = 0..nb      */
/* T_k Chebyshev polynomials of the first kind; T_k' = k U_{k-1}.       */
/* ------------------------------------------------------------------ */
static void radial_basis(double r, double rc, int nb, double *f, double *df)
{
    double fc = 0.5 * (1.0 + cos(ORC_PI * r / rc));
    double dfc = -0.5 * ORC_PI / rc * sin(ORC_PI * r / rc);
    double t = r / rc - 1.0;
    double x = 2.0 * t * t - 1.0, dx = 4.0 * t / rc;
    double T[ORC_MAXB + 2], U[ORC_MAXB + 2];
    T[0] = 1.0; T[1] = x;
    U[0] = 1.0; U[1] = 2.0 * x;
    for (int k = 2; k <= nb; ++k) {
        T[k] = 2.0 * x * T[k - 1] - T[k - 2];
        U[k] = 2.0 * x * U[k - 1] - U[k - 2];
    }
    for (int k = 0; k <= nb; ++k) {
        double dT = k == 0 ? 0.0 : k * U[k - 1];
        f[k] = 0.5 * (T[k] + 1.0) * fc;
        if (df) df[k] = 0.5 * dT * dx * fc + 0.5 * (T[k] + 1.0) * dfc;
    }
}

void oq_radial_basis(double r, double rc, int nb, double *f, double *df) { radial_basis(r, rc, nb, f, df); }

/* Legendre polynomials P_l(c) and P_l'(c), l = 0..lmax */
static void legendre(double c, int lmax, double *P, double *dP)
{
    P[0] = 1.0; dP[0] = 0.0;
    if (lmax >= 1) { P[1] = c; dP[1] = 1.0; }
    for (int l = 1; l < lmax; ++l) {
        P[l + 1] = ((2 * l + 1) * c * P[l] - l * P[l - 1]) / (l + 1);
        dP[l + 1] = dP[l - 1] + (2 * l + 1) * P[l];
    }
}

/* ------------------------------------------------------------------ */
/* parameter vector layout:                                             */
/*   cR[ti][tj][n][k]  (n = 0..n_max_R, k = 0..basis_R)                 */
/*   cA[ti][tj][n][k]  (n = 0..n_max_A, k = 0..basis_A)                 */
/*   per species t: W0[mu][nu], b0[mu], w1E[mu], w1q[mu], b1q           */
/*   b1E (shared output bias, Eq. 1), s = sqrt(eps_inf) (Eq. 24)        */
/* ------------------------------------------------------------------ */
#define ORC_MAXT 16
typedef struct {
    int T, nR, nA, bR, bA, L, H, ndes;
    double rcR, rcA;
    const double *cR, *cA, *b1E, *s;
    const double *W0[ORC_MAXT], *b0[ORC_MAXT], *w1E[ORC_MAXT], *w1q[ORC_MAXT], *b1q[ORC_MAXT];
} oq_theta;

int64_t oq_theta_count(const oq_hparams *hp)
{
    int64_t T = hp->n_types, ndes = (hp->n_max_R + 1) + (int64_t)(hp->n_max_A + 1) * hp->l_max;
    return T * T * (hp->n_max_R + 1) * (hp->basis_R + 1) + T * T * (hp->n_max_A + 1) * (hp->basis_A + 1) +
           T * (hp->n_neu * ndes + 3 * hp->n_neu + 1) + 2;
}

static void theta_view(const oq_hparams *hp, const double *th, oq_theta *v)
{
    v->T = hp->n_types; v->nR = hp->n_max_R; v->nA = hp->n_max_A;
    v->bR = hp->basis_R; v->bA = hp->basis_A; v->L = hp->l_max; v->H = hp->n_neu;
    v->rcR = hp->rc_R; v->rcA = hp->rc_A;
    v->ndes = (v->nR + 1) + (v->nA + 1) * v->L;
    const double *p = th;
    v->cR = p; p += v->T * v->T * (v->nR + 1) * (v->bR + 1);
    v->cA = p; p += v->T * v->T * (v->nA + 1) * (v->bA + 1);
    for (int t = 0; t < v->T; ++t) {
        v->W0[t] = p; p += v->H * v->ndes;
        v->b0[t] = p; p += v->H;
        v->w1E[t] = p; p += v->H;
        v->w1q[t] = p; p += v->H;
        v->b1q[t] = p; p += 1;
    }
    v->b1E = p; v->s = p + 1;
}

static double cR_at(const oq_theta *v, int ti, int tj, int n, int k)
{
    return v->cR[((ti * v->T + tj) * (v->nR + 1) + n) * (v->bR + 1) + k];
}
static double cA_at(const oq_theta *v, int ti, int tj, int n, int k)
{
    return v->cA[((ti * v->T + tj) * (v->nA + 1) + n) * (v->bA + 1) + k];
}

/* descriptor order: radial q_0..q_nR, then angular q_nl, l-major and n-minor */
static int ang_index(const oq_theta *v, int n, int l) { return (v->nR + 1) + (l - 1) * (v->nA + 1) + n; }

/* g_n(r) = sum_k c^{ti tj}_{nk} f_k(r) and its r-derivative, angular set */
static void g_angular(const oq_theta *v, int ti, int tj, double r, double *g, double *dg)
{
    double f[ORC_MAXB + 1], df[ORC_MAXB + 1];
    radial_basis(r, v->rcA, v->bA, f, df);
    for (int n = 0; n <= v->nA; ++n) {
        g[n] = 0.0; dg[n] = 0.0;
        for (int k = 0; k <= v->bA; ++k) {
            g[n] += cA_at(v, ti, tj, n, k) * f[k];
            dg[n] += cA_at(v, ti, tj, n, k) * df[k];
        }
    }
}

/* ------------------------------------------------------------------ */
/* descriptor of one atom:                                              */
/*   radial  q_n  = sum_j g^R_n(r_ij)                                   */
/*   angular q_nl = sum_j sum_k g^A_n(r_ij) g^A_n(r_ik) P_l(cos th_jik)  */
/*           (j = k included, l = 1..l_max)                             */
/* LA is the sub-list of LR with r < rc_A                               */
/* ------------------------------------------------------------------ */
static void descriptor_atom(const oq_theta *v, int ti, const int *type, const oq_plist *LR, const oq_plist *LA,
                            double *D)
{
    double f[ORC_MAXB + 1];
    for (int q = 0; q < v->ndes; ++q) D[q] = 0.0;
    for (int p = 0; p < LR->n; ++p) {
        const oq_pair *pp = &LR->p[p];
        int tj = type[pp->j];
        radial_basis(pp->r, v->rcR, v->bR, f, NULL);
        for (int n = 0; n <= v->nR; ++n)
            for (int k = 0; k <= v->bR; ++k) D[n] += cR_at(v, ti, tj, n, k) * f[k];
    }
    int m = LA->n;
    if (m == 0) return;
    double *g = (double *)malloc(sizeof(double) * (size_t)m * (v->nA + 1));
    double *dg = (double *)malloc(sizeof(double) * (size_t)m * (v->nA + 1));
    for (int a = 0; a < m; ++a) g_angular(v, ti, type[LA->p[a].j], LA->p[a].r, g + a * (v->nA + 1), dg + a * (v->nA + 1));
    double P[ORC_MAXL + 1], dP[ORC_MAXL + 1];
    for (int a = 0; a < m; ++a)
        for (int b = 0; b < m; ++b) {
            const double *da = LA->p[a].d, *db = LA->p[b].d;
            double c = (da[0] * db[0] + da[1] * db[1] + da[2] * db[2]) / (LA->p[a].r * LA->p[b].r);
            if (a == b) c = 1.0;
            legendre(c, v->L, P, dP);
            for (int l = 1; l <= v->L; ++l)
                for (int n = 0; n <= v->nA; ++n)
                    D[ang_index(v, n, l)] += g[a * (v->nA + 1) + n] * g[b * (v->nA + 1) + n] * P[l];
        }
    free(g); free(dg);
}

/* ------------------------------------------------------------------ */
/* network (Sec. 2.1 Eq. 1 and Sec. 2.2): shared hidden layer,          */
/*   h   = tanh(W0 D - b0)                                              */
/*   U_i = w1E . h - b1E,   q_i = w1q . h - b1q                         */
/* plus dU_i/dD and dq_i/dD                                             */
/* ------------------------------------------------------------------ */
static void network_atom(const oq_theta *v, int t, const double *D, double *U, double *q, double *gU, double *gq)
{
    const double *W0 = v->W0[t];
    *U = -v->b1E[0];
    *q = -v->b1q[t][0];
    if (gU) for (int nu = 0; nu < v->ndes; ++nu) { gU[nu] = 0.0; gq[nu] = 0.0; }
    for (int mu = 0; mu < v->H; ++mu) {
        double z = -v->b0[t][mu];
        for (int nu = 0; nu < v->ndes; ++nu) z += W0[mu * v->ndes + nu] * D[nu];
        double hmu = tanh(z);
        *U += v->w1E[t][mu] * hmu;
        *q += v->w1q[t][mu] * hmu;
        if (gU) {
            double dE = v->w1E[t][mu] * (1.0 - hmu * hmu), dq = v->w1q[t][mu] * (1.0 - hmu * hmu);
            for (int nu = 0; nu < v->ndes; ++nu) {
                gU[nu] += dE * W0[mu * v->ndes + nu];
                gq[nu] += dq * W0[mu * v->ndes + nu];
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* PPPM pieces (Sec. 2.6)                                               */
/* ------------------------------------------------------------------ */
/* cardinal B-spline M_P(x) on [0, P], by its recursive definition */
static double bspline(int P, double x)
{
    if (P == 1) return (x >= 0.0 && x < 1.0) ? 1.0 : 0.0;
    return (x * bspline(P - 1, x) + (P - x) * bspline(P - 1, x - 1.0)) / (P - 1);
}

/* assignment weight along one axis for odd P: W(x) = M_P(x + P/2), |x| < P/2 */
static double assign_w(int P, double x) { return bspline(P, x + 0.5 * P); }

double oq_assign_weight(int P, double x) { return assign_w(P, x); }

/* P = 5 alias sum  sum_m sinc^10(pi (n/N + m)) as a polynomial in z = sin(pi n/N) */
static double alias_poly5(double z)
{
    double z2 = z * z;
    return 1.0 - 5.0 / 3.0 * z2 + 7.0 / 9.0 * z2 * z2 - 17.0 / 189.0 * z2 * z2 * z2 + 2.0 / 2835.0 * z2 * z2 * z2 * z2;
}

double oq_alias_poly5(double z) { return alias_poly5(z); }

static double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

/* mesh index j in [0, N) -> wave number n in [-N/2, N/2) */
static int wave_index(int j, int N) { return 2 * j < N ? j : j - N; }

/* direct DFT of every line of a complex 3D array along one axis;
   sign = -1: sum_m x_m e^{-2 pi i n m / N}, sign = +1: the unnormalized inverse */
static void dft_axis(double *re, double *im, const int *N, int axis, int sign)
{
    int Na = N[axis];
    int stride = axis == 2 ? 1 : (axis == 1 ? N[2] : N[1] * N[2]);
    int nlines = N[0] * N[1] * N[2] / Na;
    double *cs = (double *)malloc(sizeof(double) * (size_t)Na), *sn = (double *)malloc(sizeof(double) * (size_t)Na);
    for (int t = 0; t < Na; ++t) { cs[t] = cos(2.0 * ORC_PI * t / Na); sn[t] = sign * sin(2.0 * ORC_PI * t / Na); }
#pragma omp parallel
    {
        double *tr = (double *)malloc(sizeof(double) * (size_t)Na), *ti = (double *)malloc(sizeof(double) * (size_t)Na);
#pragma omp for
        for (int line = 0; line < nlines; ++line) {
            /* base offset of this line */
            int base;
            if (axis == 2) base = line * Na;
            else if (axis == 1) base = (line / N[2]) * N[1] * N[2] + (line % N[2]);
            else base = line;
            for (int n = 0; n < Na; ++n) {
                double sr = 0.0, si = 0.0;
                for (int m = 0; m < Na; ++m) {
                    int t = (int)(((long)n * m) % Na);
                    double xr = re[base + m * stride], xi = im[base + m * stride];
                    sr += xr * cs[t] - xi * sn[t];
                    si += xr * sn[t] + xi * cs[t];
                }
                tr[n] = sr; ti[n] = si;
            }
            for (int n = 0; n < Na; ++n) { re[base + n * stride] = tr[n]; im[base + n * stride] = ti[n]; }
        }
        free(tr); free(ti);
    }
    free(cs); free(sn);
}

/* 3D DFT of a complex mesh; exported for the tests */
void oq_dft3(double *re, double *im, const int *N, int sign)
{
    for (int a = 2; a >= 0; --a) dft_axis(re, im, N, a, sign);
}

/* ------------------------------------------------------------------ */
/* reciprocal part: U^k, per-atom phi^k, static force and virial        */
/* Ewald: Sec. 2.2.2 Eqs. 7-9, Sec. 2.3.2 Eqs. 18, 21, 22               */
/* PPPM : Sec. 2.6 Eqs. 34-37 with the readings stated at the top       */
/* q is the screened corrected charge q'                                */
/* ------------------------------------------------------------------ */
static void recip_ewald(const oq_es *es, int n, const double *pos, const double *h, const double *q, double *Uk,
                        double *phik, double *Fk, double *Wk, double *nk_out, double *Wa)
{
    double hi[9];
    inv3(h, hi);
    double vol = fabs(det3(h));
    double alpha = es->alpha;
    int m[3];
    for (int a = 0; a < 3; ++a) {
        double len = sqrt(h[3 * a] * h[3 * a] + h[3 * a + 1] * h[3 * a + 1] + h[3 * a + 2] * h[3 * a + 2]);
        m[a] = (int)floor(es->kmax * len / (2.0 * ORC_PI)) + 1;
    }
    /* enumerate the full sphere of wave vectors k = 2 pi h^{-1} n, n != 0 */
    int cap = (2 * m[0] + 1) * (2 * m[1] + 1) * (2 * m[2] + 1);
    double *kv = (double *)malloc(sizeof(double) * 3 * (size_t)cap);
    int nk = 0;
    for (int n1 = -m[0]; n1 <= m[0]; ++n1)
        for (int n2 = -m[1]; n2 <= m[1]; ++n2)
            for (int n3 = -m[2]; n3 <= m[2]; ++n3) {
                if (n1 == 0 && n2 == 0 && n3 == 0) continue;
                double k[3];
                for (int b = 0; b < 3; ++b) k[b] = 2.0 * ORC_PI * (hi[3 * b] * n1 + hi[3 * b + 1] * n2 + hi[3 * b + 2] * n3);
                /* |k| <= kmax (inclusive) or |k| < kmax, ties at the sphere resolved with a
                   relative tolerance of 1e-9 on k^2 */
                double kk2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2], km2 = es->kmax * es->kmax;
                int keep = es->kmax_inclusive ? (kk2 <= km2 * (1.0 + 1e-9)) : (kk2 < km2 * (1.0 - 1e-9));
                if (!keep) continue;
                kv[3 * nk] = k[0]; kv[3 * nk + 1] = k[1]; kv[3 * nk + 2] = k[2];
                ++nk;
            }
    *nk_out = nk;
    double *Sre = (double *)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
    double *Sim = (double *)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
    double *G = (double *)calloc((size_t)(nk > 0 ? nk : 1), sizeof(double));
    /* S(k) = sum_i q_i exp(-i k.r_i)  (Eq. 8);  G(k) = 2 pi / Omega exp(-k^2/4a^2) / k^2 (Eq. 9) */
#pragma omp parallel for schedule(static)
    for (int s = 0; s < nk; ++s) {
        const double *k = kv + 3 * s;
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        G[s] = 2.0 * ORC_PI / vol * exp(-k2 / (4.0 * alpha * alpha)) / k2;
        double sr = 0.0, si = 0.0;
        for (int i = 0; i < n; ++i) {
            double ph = k[0] * pos[3 * i] + k[1] * pos[3 * i + 1] + k[2] * pos[3 * i + 2];
            sr += q[i] * cos(ph);
            si -= q[i] * sin(ph);
        }
        Sre[s] = sr; Sim[s] = si;
    }
    double U = 0.0, W[9] = {0};
    for (int s = 0; s < nk; ++s) {
        const double *k = kv + 3 * s;
        double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        double e = ORC_KE * G[s] * (Sre[s] * Sre[s] + Sim[s] * Sim[s]);
        U += e;
        /* B = I - (2/(4 alpha^2) + 2/k^2) k k  (Eq. 21), W = sum k_e G |S|^2 B (Eq. 22) */
        double c = 2.0 / (4.0 * alpha * alpha) + 2.0 / k2;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) W[3 * a + b] += e * ((a == b ? 1.0 : 0.0) - c * k[a] * k[b]);
    }
    *Uk = U;
    for (int t = 0; t < 9; ++t) Wk[t] = W[t];
    /* phi^k_i = 2 k_e sum_k G Re[S e^{i k.r_i}],  F^k_i = 2 k_e q_i sum_k k G Im[S e^{i k.r_i}] (Eq. 18);
       per-atom virial W^k_i = k_e q_i sum_k G Re[S e^{i k.r_i}] B(k) (Eq. 20) */
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double ph = 0.0, f[3] = {0, 0, 0}, wa[9] = {0};
        for (int s = 0; s < nk; ++s) {
            const double *k = kv + 3 * s;
            double a = k[0] * pos[3 * i] + k[1] * pos[3 * i + 1] + k[2] * pos[3 * i + 2];
            double c = cos(a), sn = sin(a);
            double re = Sre[s] * c - Sim[s] * sn, im = Sre[s] * sn + Sim[s] * c;
            ph += G[s] * re;
            for (int b = 0; b < 3; ++b) f[b] += k[b] * G[s] * im;
            if (Wa) {
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                double cb = 2.0 / (4.0 * alpha * alpha) + 2.0 / k2;
                for (int x = 0; x < 3; ++x)
                    for (int y = 0; y < 3; ++y) wa[3 * x + y] += G[s] * re * ((x == y ? 1.0 : 0.0) - cb * k[x] * k[y]);
            }
        }
        phik[i] = 2.0 * ORC_KE * ph;
        for (int b = 0; b < 3; ++b) Fk[3 * i + b] = 2.0 * ORC_KE * q[i] * f[b];
        if (Wa)
            for (int t = 0; t < 9; ++t) Wa[9 * i + t] = ORC_KE * q[i] * wa[t];
    }
    free(kv); free(Sre); free(Sim); free(G);
}

static void recip_pppm(const oq_es *es, int n, const double *pos, const double *h, const double *q, double *Uk,
                       double *phik, double *Fk, double *Wk, double *Wa)
{
    const int P = es->order;
    const int *N = es->mesh;
    int M = N[0] * N[1] * N[2];
    double hi[9];
    inv3(h, hi);
    double vol = fabs(det3(h));
    double alpha = es->alpha;
    /* mesh coordinates u_a = N_a s_a with s = r h^{-1} (positions need not be wrapped) */
    double *u = (double *)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) {
            double s = pos[3 * i] * hi[a] + pos[3 * i + 1] * hi[3 + a] + pos[3 * i + 2] * hi[6 + a];
            s -= floor(s);
            u[3 * i + a] = s * N[a];
        }
    /* charge assignment rho_m = sum_i q_i W(u_i - m) (Eq. 35), separable */
    double *rre = (double *)calloc((size_t)M, sizeof(double)), *rim = (double *)calloc((size_t)M, sizeof(double));
    int half = P / 2;
    for (int i = 0; i < n; ++i) {
        int m0[3];
        double w[3][16];
        for (int a = 0; a < 3; ++a) {
            m0[a] = (int)floor(u[3 * i + a] + 0.5);
            for (int t = -half; t <= half; ++t) w[a][t + half] = assign_w(P, u[3 * i + a] - (m0[a] + t));
        }
        for (int t0 = -half; t0 <= half; ++t0)
            for (int t1 = -half; t1 <= half; ++t1)
                for (int t2 = -half; t2 <= half; ++t2) {
                    int j0 = ((m0[0] + t0) % N[0] + N[0]) % N[0];
                    int j1 = ((m0[1] + t1) % N[1] + N[1]) % N[1];
                    int j2 = ((m0[2] + t2) % N[2] + N[2]) % N[2];
                    rre[(j0 * N[1] + j1) * N[2] + j2] += q[i] * w[0][t0 + half] * w[1][t1 + half] * w[2][t2 + half];
                }
    }
    /* S(k) on the mesh: forward DFT */
    oq_dft3(rre, rim, N, -1);
    /* G_opt(k) = G(k) [prod sinc^P(pi n_a/N_a)]^2 / [prod poly(z_a)]^2 (Eq. 36, squared denominator) */
    double *Are = (double *)calloc((size_t)M, sizeof(double)), *Aim = (double *)calloc((size_t)M, sizeof(double));
    double *Ex[3];
    for (int a = 0; a < 3; ++a) Ex[a] = (double *)calloc((size_t)M * 2, sizeof(double));
    /* per-atom virial: S G_opt B_xy for the six independent components (Eq. 39) */
    static const int VX[6] = {0, 1, 2, 0, 0, 1}, VY[6] = {0, 1, 2, 1, 2, 2};
    double *Vm[6] = {0};
    if (Wa)
        for (int c = 0; c < 6; ++c) Vm[c] = (double *)calloc((size_t)M * 2, sizeof(double));
    double U = 0.0, W[9] = {0};
    for (int j0 = 0; j0 < N[0]; ++j0)
        for (int j1 = 0; j1 < N[1]; ++j1)
            for (int j2 = 0; j2 < N[2]; ++j2) {
                int nv[3] = {wave_index(j0, N[0]), wave_index(j1, N[1]), wave_index(j2, N[2])};
                int lin = (j0 * N[1] + j1) * N[2] + j2;
                if (nv[0] == 0 && nv[1] == 0 && nv[2] == 0) continue;
                double k[3], kt[3];
                int nt[3];
                for (int a = 0; a < 3; ++a) nt[a] = (N[a] % 2 == 0 && 2 * nv[a] == -N[a]) ? 0 : nv[a];
                for (int b = 0; b < 3; ++b) {
                    k[b] = 2.0 * ORC_PI * (hi[3 * b] * nv[0] + hi[3 * b + 1] * nv[1] + hi[3 * b + 2] * nv[2]);
                    kt[b] = 2.0 * ORC_PI * (hi[3 * b] * nt[0] + hi[3 * b + 1] * nt[1] + hi[3 * b + 2] * nt[2]);
                }
                double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
                double G = 2.0 * ORC_PI / vol * exp(-k2 / (4.0 * alpha * alpha)) / k2;
                double num = 1.0, den = 1.0;
                for (int a = 0; a < 3; ++a) {
                    double x = ORC_PI * nv[a] / N[a];
                    num *= pow(sinc(x), P);
                    den *= alias_poly5(sin(x));
                }
                double Gopt = G * num * num / (den * den);
                double S2 = rre[lin] * rre[lin] + rim[lin] * rim[lin];
                double e = ORC_KE * Gopt * S2;
                U += e;
                double c = 2.0 / (4.0 * alpha * alpha) + 2.0 / k2;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) W[3 * a + b] += e * ((a == b ? 1.0 : 0.0) - c * k[a] * k[b]);
                /* S G_opt and i k~ S G_opt */
                Are[lin] = rre[lin] * Gopt;
                Aim[lin] = rim[lin] * Gopt;
                for (int a = 0; a < 3; ++a) {
                    Ex[a][lin] = -kt[a] * Aim[lin];          /* real part of i k (A_re + i A_im) */
                    Ex[a][M + lin] = kt[a] * Are[lin];       /* imaginary part */
                }
                if (Wa)
                    for (int cc = 0; cc < 6; ++cc) {
                        double B = (VX[cc] == VY[cc] ? 1.0 : 0.0) - c * k[VX[cc]] * k[VY[cc]];
                        Vm[cc][lin] = Are[lin] * B;
                        Vm[cc][M + lin] = Aim[lin] * B;
                    }
            }
    *Uk = U;
    for (int t = 0; t < 9; ++t) Wk[t] = W[t];
    /* inverse transforms (unnormalized, e^{+ik.r}) */
    oq_dft3(Are, Aim, N, +1);
    for (int a = 0; a < 3; ++a) oq_dft3(Ex[a], Ex[a] + M, N, +1);
    if (Wa)
        for (int cc = 0; cc < 6; ++cc) oq_dft3(Vm[cc], Vm[cc] + M, N, +1);
    /* gather: phi^k_i = 2 k_e sum_s W F^-1[S G_opt]  (Eq. 38 form),
               F^k_i  = -2 k_e q_i sum_s W F^-1[i k S G_opt]  (Eq. 37) */
    for (int i = 0; i < n; ++i) {
        int m0[3];
        double w[3][16];
        for (int a = 0; a < 3; ++a) {
            m0[a] = (int)floor(u[3 * i + a] + 0.5);
            for (int t = -half; t <= half; ++t) w[a][t + half] = assign_w(P, u[3 * i + a] - (m0[a] + t));
        }
        double ph = 0.0, e[3] = {0, 0, 0}, vv[6] = {0, 0, 0, 0, 0, 0};
        for (int t0 = -half; t0 <= half; ++t0)
            for (int t1 = -half; t1 <= half; ++t1)
                for (int t2 = -half; t2 <= half; ++t2) {
                    int j0 = ((m0[0] + t0) % N[0] + N[0]) % N[0];
                    int j1 = ((m0[1] + t1) % N[1] + N[1]) % N[1];
                    int j2 = ((m0[2] + t2) % N[2] + N[2]) % N[2];
                    int lin = (j0 * N[1] + j1) * N[2] + j2;
                    double ww = w[0][t0 + half] * w[1][t1 + half] * w[2][t2 + half];
                    ph += ww * Are[lin];
                    for (int a = 0; a < 3; ++a) e[a] += ww * Ex[a][lin];
                    if (Wa)
                        for (int cc = 0; cc < 6; ++cc) vv[cc] += ww * Vm[cc][lin];
                }
        phik[i] = 2.0 * ORC_KE * ph;
        for (int a = 0; a < 3; ++a) Fk[3 * i + a] = -2.0 * ORC_KE * q[i] * e[a];
        /* W^k_i = k_e q_i sum_s W(r_i - r_s) F^-1[S G_opt B] (Eq. 39) */
        if (Wa)
            for (int cc = 0; cc < 6; ++cc) {
                Wa[9 * i + 3 * VX[cc] + VY[cc]] = ORC_KE * q[i] * vv[cc];
                Wa[9 * i + 3 * VY[cc] + VX[cc]] = ORC_KE * q[i] * vv[cc];
            }
    }
    free(u); free(rre); free(rim); free(Are); free(Aim);
    for (int a = 0; a < 3; ++a) free(Ex[a]);
    for (int cc = 0; cc < 6; ++cc) free(Vm[cc]);
}

/* ------------------------------------------------------------------ */
/* full evaluation                                                      */
/* ------------------------------------------------------------------ */
/* Ablation switch for the tests (0 = off, the default): bit 1 drops the -mean(phi)
   part of the chain rule through the neutrality correction, i.e. the forces use
   chi_i = phi_i; the energy is unchanged.  A test sets it to show that the finite-
   difference check of the forces detects that mistake. */
static int oq_ablation = 0;
void oq_set_ablation(int flags) { oq_ablation = flags; }

int oq_compute(const oq_hparams *hp, const oq_es *es, int n, const double *pos, const int *type, const double *cell,
               const double *theta, int nbr_method, int want_forces, oq_out *out, int periodic)
{
    /* isolated systems (periodic = 0) take the direct Coulomb sum (method 2) only, and
       periodic ones Ewald or PPPM */
    if (periodic ? es->method == 2 : es->method != 2) return -3;
    if (n < 1 || hp->n_types > ORC_MAXT || hp->basis_R > ORC_MAXB || hp->basis_A > ORC_MAXB || hp->l_max > ORC_MAXL)
        return -1;
    if (es->method == 1 && es->order != 5) return -2;
    for (int i = 0; i < n; ++i)
        if (type[i] < 0 || type[i] >= hp->n_types) return -1;
    oq_theta v;
    theta_view(hp, theta, &v);
    const int ndes = v.ndes;
    const double s = v.s[0];
    const double alpha = es->alpha;
    const double vol = fabs(det3(cell));

    double *frac = (double *)malloc(sizeof(double) * 3 * (size_t)n), *wpos = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (periodic) wrap_positions(n, pos, cell, frac, wpos);
    else memcpy(wpos, pos, sizeof(double) * 3 * (size_t)n);

    /* neighbour lists: radial (NEP radial cutoff), angular (sub-list), Coulomb */
    oq_plist *LR = periodic ? build_list(nbr_method, n, frac, wpos, cell, v.rcR) : nbr_free(n, pos, v.rcR);
    oq_plist *LA = (oq_plist *)calloc((size_t)n, sizeof(oq_plist));
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < LR[i].n; ++p)
            if (LR[i].p[p].r < v.rcA) plist_push(&LA[i], LR[i].p[p].j, LR[i].p[p].d, LR[i].p[p].r);
    oq_plist *LC = periodic && es->mode == 1 ? build_list(nbr_method, n, frac, wpos, cell, es->rc_coul) : NULL;

    /* descriptors, network outputs and their gradients */
    double *D = (double *)malloc(sizeof(double) * (size_t)n * ndes);
    double *gU = (double *)malloc(sizeof(double) * (size_t)n * ndes), *gq = (double *)malloc(sizeof(double) * (size_t)n * ndes);
    double *U = (double *)malloc(sizeof(double) * (size_t)n), *qraw = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; ++i) {
        descriptor_atom(&v, type[i], type, &LR[i], &LA[i], D + (size_t)i * ndes);
        network_atom(&v, type[i], D + (size_t)i * ndes, &U[i], &qraw[i], gU + (size_t)i * ndes, gq + (size_t)i * ndes);
    }

    /* charges: q~ = s q (Eq. 24); q~' = q~ + (Q - sum q~)/N (Eq. 33 as read); q' = q~'/s */
    double sum_qraw = 0.0, U_nep = 0.0;
    for (int i = 0; i < n; ++i) { sum_qraw += qraw[i]; U_nep += U[i]; }
    double *qt = (double *)malloc(sizeof(double) * (size_t)n), *qs = (double *)malloc(sizeof(double) * (size_t)n);
    double sum_qt = 0.0;
    for (int i = 0; i < n; ++i) {
        qt[i] = s * qraw[i] + (es->q_total - s * sum_qraw) / n;
        qs[i] = qt[i] / s;
        sum_qt += qt[i];
    }

    /* electrostatics on q' */
    double *phi = (double *)calloc((size_t)n, sizeof(double));
    double *Fst = (double *)calloc((size_t)n * 3, sizeof(double));
    double *Va = want_forces && out->vatom ? (double *)calloc((size_t)n * 9, sizeof(double)) : NULL;
    double Ur = 0.0, Us = 0.0, Ubg = 0.0, Uk = 0.0, Wst[9] = {0}, nk = 0.0;
    if (!periodic) {
        /* isolated system: direct Coulomb sum over all pairs, U = 1/2 k_e sum_{i != j}
           q'_i q'_j / r_ij (Eq. 6 with alpha -> 0 and no images) */
        double Wl[9] = {0};
        for (int i = 0; i < n; ++i) {
            double ph = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3];
                for (int b = 0; b < 3; ++b) d[b] = pos[3 * j + b] - pos[3 * i + b];
                double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                ph += ORC_KE * qs[j] / r;
                double du = -ORC_KE * qs[i] * qs[j] / (r * r);
                for (int b = 0; b < 3; ++b) Fst[3 * i + b] += du * d[b] / r;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) {
                        Wl[3 * a + b] -= 0.5 * du * d[a] * d[b] / r;
                        if (Va) Va[9 * i + 3 * a + b] -= 0.5 * du * d[a] * d[b] / r;
                    }
            }
            phi[i] = ph;
            Ur += 0.5 * qs[i] * ph;
        }
        for (int t = 0; t < 9; ++t) Wst[t] += Wl[t];
    } else if (es->mode == 1) {
        /* real space (Sec. 2.2.1 Eq. 6; static pair force Eq. 15) */
        double Wr[9] = {0};
#pragma omp parallel
        {
            double Wl[9] = {0};
#pragma omp for reduction(+ : Ur)
            for (int i = 0; i < n; ++i) {
                double ph = 0.0;
                for (int p = 0; p < LC[i].n; ++p) {
                    const oq_pair *pp = &LC[i].p[p];
                    double r = pp->r, qj = qs[pp->j];
                    double ec = erfc(alpha * r);
                    ph += ORC_KE * qj * ec / r;
                    /* u(r) = k_e q_i q_j erfc(alpha r)/r, u'(r) */
                    double du = -ORC_KE * qs[i] * qj * (ec / (r * r) + 2.0 * alpha / sqrt(ORC_PI) * exp(-alpha * alpha * r * r) / r);
                    for (int b = 0; b < 3; ++b) Fst[3 * i + b] += du * pp->d[b] / r; /* F_i = -du/dr_i = du * r_hat_ij */
                    /* W = -sum_{pairs} u'(r) r_a r_b / r, each unordered pair seen twice */
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) Wl[3 * a + b] -= 0.5 * du * pp->d[a] * pp->d[b] / r;
                    /* per atom: W_i += r_ij (x) F_ji with the static partial force F_ji = u'(r) r_ji / (2 r) */
                    if (Va)
                        for (int a = 0; a < 3; ++a)
                            for (int b = 0; b < 3; ++b) Va[9 * i + 3 * a + b] -= 0.5 * du * pp->d[a] * pp->d[b] / r;
                }
                phi[i] += ph;
                Ur += 0.5 * qs[i] * ph;
            }
#pragma omp critical
            for (int t = 0; t < 9; ++t) Wr[t] += Wl[t];
        }
        for (int t = 0; t < 9; ++t) Wst[t] += Wr[t];
        /* self energy (Sec. 2.2.3 Eq. 10) */
        for (int i = 0; i < n; ++i) {
            Us -= ORC_KE * alpha / sqrt(ORC_PI) * qs[i] * qs[i];
            phi[i] -= 2.0 * ORC_KE * alpha / sqrt(ORC_PI) * qs[i];
        }
        /* neutralizing background for a net charge (k = 0 term excluded in Eq. 7) */
        double Qs = sum_qt / s;
        Ubg = -ORC_KE * ORC_PI * Qs * Qs / (2.0 * vol * alpha * alpha);
        for (int i = 0; i < n; ++i) phi[i] += -ORC_KE * ORC_PI * Qs / (vol * alpha * alpha);
        for (int a = 0; a < 3; ++a) Wst[4 * a] += Ubg;
        if (Va)
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a) Va[9 * i + 4 * a] += Ubg / n;
    }
    if (periodic) {
        double *phik = (double *)calloc((size_t)n, sizeof(double)), *Fk = (double *)calloc((size_t)n * 3, sizeof(double));
        double Wk[9] = {0};
        double *Wka = Va ? (double *)calloc((size_t)n * 9, sizeof(double)) : NULL;
        if (es->method == 0) recip_ewald(es, n, pos, cell, qs, &Uk, phik, Fk, Wk, &nk, Wka);
        else recip_pppm(es, n, pos, cell, qs, &Uk, phik, Fk, Wk, Wka);
        for (int i = 0; i < n; ++i) {
            phi[i] += phik[i];
            for (int b = 0; b < 3; ++b) Fst[3 * i + b] += Fk[3 * i + b];
            if (Va)
                for (int t = 0; t < 9; ++t) Va[9 * i + t] += Wka[9 * i + t];
        }
        free(Wka);
        for (int t = 0; t < 9; ++t) Wst[t] += Wk[t];
        free(phik); free(Fk);
    }
    double phibar = 0.0;
    for (int i = 0; i < n; ++i) phibar += phi[i];
    phibar /= n;

    if (out->terms) {
        double *t = out->terms;
        t[0] = U_nep + Ur + Uk + Us + Ubg; t[1] = U_nep; t[2] = Ur; t[3] = Uk; t[4] = Us; t[5] = Ubg;
        t[6] = sum_qraw; t[7] = phibar; t[8] = sum_qt; t[9] = nk;
    }
    for (int i = 0; i < n; ++i) {
        if (out->q_screened) out->q_screened[i] = qs[i];
        if (out->q_naked) out->q_naked[i] = qt[i];
        if (out->q_raw) out->q_raw[i] = qraw[i];
        if (out->site_energy) out->site_energy[i] = U[i];
        if (out->phi) out->phi[i] = phi[i];
        if (out->desc) for (int q = 0; q < ndes; ++q) out->desc[(size_t)i * ndes + q] = D[(size_t)i * ndes + q];
    }
    if (out->pol) {
        /* P = sum_i q~'_i r_i with the caller's coordinates (Eq. 26) */
        for (int a = 0; a < 3; ++a) {
            out->pol[a] = 0.0;
            for (int i = 0; i < n; ++i) out->pol[a] += qt[i] * pos[3 * i + a];
        }
    }

    if (want_forces) {
        /* partial forces F_ij = g_i . dD^i/dr_ij with g_i = dU_i/dD + chi_i dq_i/dD,
           chi_i = phi_i - mean(phi) (Eqs. 14, 16, 17, 19, 23 through the correction);
           a_ij = s dq_i/dD . dD^i/dr_ij (charge derivative for Eq. 28) */
        size_t *offR = (size_t *)malloc(sizeof(size_t) * (size_t)(n + 1)), *offA = (size_t *)malloc(sizeof(size_t) * (size_t)(n + 1));
        offR[0] = 0; offA[0] = 0;
        for (int i = 0; i < n; ++i) { offR[i + 1] = offR[i] + LR[i].n; offA[i + 1] = offA[i] + LA[i].n; }
        double *FR = (double *)calloc(offR[n] * 3 + 1, sizeof(double)), *AR = (double *)calloc(offR[n] * 3 + 1, sizeof(double));
        double *FA = (double *)calloc(offA[n] * 3 + 1, sizeof(double)), *AA = (double *)calloc(offA[n] * 3 + 1, sizeof(double));
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; ++i) {
            int ti = type[i];
            double chi = phi[i] - ((oq_ablation & 1) ? 0.0 : phibar);
            double *g = (double *)malloc(sizeof(double) * (size_t)ndes), *ga = (double *)malloc(sizeof(double) * (size_t)ndes);
            for (int q = 0; q < ndes; ++q) {
                g[q] = gU[(size_t)i * ndes + q] + chi * gq[(size_t)i * ndes + q];
                ga[q] = s * gq[(size_t)i * ndes + q];
            }
            /* radial: dq_n/dr_ij = sum_k c_nk f_k'(r) r_hat */
            double f[ORC_MAXB + 1], df[ORC_MAXB + 1];
            for (int p = 0; p < LR[i].n; ++p) {
                const oq_pair *pp = &LR[i].p[p];
                int tj = type[pp->j];
                radial_basis(pp->r, v.rcR, v.bR, f, df);
                double sE = 0.0, sQ = 0.0;
                for (int nn = 0; nn <= v.nR; ++nn) {
                    double dq = 0.0;
                    for (int k = 0; k <= v.bR; ++k) dq += cR_at(&v, ti, tj, nn, k) * df[k];
                    sE += g[nn] * dq;
                    sQ += ga[nn] * dq;
                }
                for (int b = 0; b < 3; ++b) {
                    FR[(offR[i] + p) * 3 + b] = sE * pp->d[b] / pp->r;
                    AR[(offR[i] + p) * 3 + b] = sQ * pp->d[b] / pp->r;
                }
            }
            /* angular: dq_nl/dr_ij = 2 g_n'(r_j) r_hat_j sum_b g_n(r_b) P_l(c_jb)
                                    + 2 g_n(r_j) sum_b g_n(r_b) P_l'(c_jb) (r_hat_b - c_jb r_hat_j)/r_j */
            int m = LA[i].n;
            if (m > 0) {
                int na = v.nA + 1;
                double *ga_n = (double *)malloc(sizeof(double) * (size_t)m * na), *dga_n = (double *)malloc(sizeof(double) * (size_t)m * na);
                for (int a = 0; a < m; ++a) g_angular(&v, ti, type[LA[i].p[a].j], LA[i].p[a].r, ga_n + a * na, dga_n + a * na);
                double P[ORC_MAXL + 1], dP[ORC_MAXL + 1];
                for (int a = 0; a < m; ++a) {
                    const oq_pair *pa = &LA[i].p[a];
                    double ua[3] = {pa->d[0] / pa->r, pa->d[1] / pa->r, pa->d[2] / pa->r};
                    double fE[3] = {0, 0, 0}, fQ[3] = {0, 0, 0};
                    for (int b = 0; b < m; ++b) {
                        const oq_pair *pb = &LA[i].p[b];
                        double ub[3] = {pb->d[0] / pb->r, pb->d[1] / pb->r, pb->d[2] / pb->r};
                        double c = a == b ? 1.0 : ua[0] * ub[0] + ua[1] * ub[1] + ua[2] * ub[2];
                        legendre(c, v.L, P, dP);
                        double dc[3];
                        for (int x = 0; x < 3; ++x) dc[x] = a == b ? 0.0 : (ub[x] - c * ua[x]) / pa->r;
                        for (int l = 1; l <= v.L; ++l)
                            for (int nn = 0; nn < na; ++nn) {
                                int q = ang_index(&v, nn, l);
                                double t1 = 2.0 * dga_n[a * na + nn] * ga_n[b * na + nn] * P[l];
                                double t2 = 2.0 * ga_n[a * na + nn] * ga_n[b * na + nn] * dP[l];
                                for (int x = 0; x < 3; ++x) {
                                    double dD = t1 * ua[x] + t2 * dc[x];
                                    fE[x] += g[q] * dD;
                                    fQ[x] += ga[q] * dD;
                                }
                            }
                    }
                    for (int x = 0; x < 3; ++x) { FA[(offA[i] + a) * 3 + x] = fE[x]; AA[(offA[i] + a) * 3 + x] = fQ[x]; }
                }
                free(ga_n); free(dga_n);
            }
            free(g); free(ga);
        }
        /* assembly: F_i = sum_j (F_ij - F_ji) (Eq. 11) + static; W = -sum F_ij (x) r_ij + static;
           Z_i = q~'_i I + 1/2 sum_j (r_ij (x) a_ij - r_ji (x) a_ji) (Eq. 28) */
        double *F = out->forces, *Z = out->bec, W[9];
        double *Fl = (double *)calloc((size_t)n * 3, sizeof(double)), *Zl = (double *)calloc((size_t)n * 9, sizeof(double));
        for (int t = 0; t < 9; ++t) W[t] = Wst[t];
        for (int i = 0; i < n; ++i) {
            for (int b = 0; b < 3; ++b) Fl[3 * i + b] += Fst[3 * i + b];
            for (int a = 0; a < 3; ++a) Zl[9 * i + 4 * a] += qt[i];
        }
        /* isolated system: Z_k = dP/dr_k with absolute positions (Eq. 27) and the
           corrected charges, q~'_k I + sum_i (r_i - rbar) (x) dq~_i/dr_k */
        double rbar[3] = {0, 0, 0};
        if (!periodic) {
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a) rbar[a] += pos[3 * i + a] / n;
        }
        for (int pass = 0; pass < 2; ++pass) {
            oq_plist *L = pass == 0 ? LR : LA;
            size_t *off = pass == 0 ? offR : offA;
            double *FF = pass == 0 ? FR : FA, *AAp = pass == 0 ? AR : AA;
            for (int i = 0; i < n; ++i)
                for (int p = 0; p < L[i].n; ++p) {
                    const oq_pair *pp = &L[i].p[p];
                    int j = pp->j;
                    const double *fij = FF + (off[i] + p) * 3, *aij = AAp + (off[i] + p) * 3;
                    for (int b = 0; b < 3; ++b) { Fl[3 * i + b] += fij[b]; Fl[3 * j + b] -= fij[b]; }
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) {
                            W[3 * a + b] -= fij[a] * pp->d[b];
                            /* per atom (Eq. 12): W_j += r_ji (x) F_ij */
                            if (Va) Va[9 * j + 3 * a + b] -= pp->d[a] * fij[b];
                            if (periodic) {
                                /* Eq. 28 */
                                double c = 0.5 * pp->d[a] * aij[b];
                                Zl[9 * i + 3 * a + b] += c;
                                Zl[9 * j + 3 * a + b] -= c;
                            } else {
                                /* dq~_i/dr_j = a_ij, dq~_i/dr_i = -sum_j a_ij */
                                double c = (pos[3 * i + a] - rbar[a]) * aij[b];
                                Zl[9 * j + 3 * a + b] += c;
                                Zl[9 * i + 3 * a + b] -= c;
                            }
                        }
                }
        }
        /* external field (Eq. 29): F_i[b] += sum_a E_a Z_i[a][b] */
        if (es->efield[0] != 0.0 || es->efield[1] != 0.0 || es->efield[2] != 0.0)
            for (int i = 0; i < n; ++i)
                for (int b = 0; b < 3; ++b)
                    for (int a = 0; a < 3; ++a) Fl[3 * i + b] += es->efield[a] * Zl[9 * i + 3 * a + b];
        if (F) memcpy(F, Fl, sizeof(double) * 3 * (size_t)n);
        if (Va) memcpy(out->vatom, Va, sizeof(double) * 9 * (size_t)n);
        if (Z) memcpy(Z, Zl, sizeof(double) * 9 * (size_t)n);
        if (out->virial) memcpy(out->virial, W, sizeof(double) * 9);
        free(Fl); free(Zl);
        free(offR); free(offA); free(FR); free(AR); free(FA); free(AA);
    }

    free_lists(n, LR); free_lists(n, LA); free_lists(n, LC);
    free(frac); free(wpos); free(D); free(gU); free(gq); free(U); free(qraw); free(qt); free(qs); free(phi); free(Fst);
    free(Va);
    return 0;
}
