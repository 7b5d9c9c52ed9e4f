/*
 * oracle.c -- plain, slow, FP64 CPU reference for the two-electron repulsion
 * integrals (ERIs) over contracted Cartesian Gaussian shells and for the
 * Coulomb (J) and exchange (K) matrices built from them.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library.
 *
 * What it computes (paper, Section 2.2):
 *   - contracted functions psi_a = sum_k c_ak phi_ak (Eq. 1), phi a primitive
 *     Cartesian Gaussian (x-Ax)^i (y-Ay)^j (z-Az)^k exp(-alpha |r-A|^2);
 *   - contracted ERIs (ab|cd) = sum_klmn c_ak c_bl c_cm c_dn [a_k b_l|c_m d_n]
 *     (Eq. 2) in chemists' notation, int int psi_a(1) psi_b(1) 1/r12
 *     psi_c(2) psi_d(2);
 *   - J_mn = sum_ls (mn|ls) D_ls and K_mn = sum_ls (ml|ns) D_ls, the
 *     two-electron part of the Fock matrix of the SCF loop (Section 2.1);
 *   - the nuclear gradient of E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) at fixed D.
 *
 * The paper names the recurrences it uses on the GPU (HRR and VRR down to an
 * analytic [00|00]) but prints no formula.  The oracle therefore evaluates
 * each primitive integral with the McMurchie-Davidson Hermite expansion, a
 * different exact route: 1-D Hermite coefficients E^{ij}_t per primitive pair,
 * Hermite Coulomb integrals R_{tuv} from the Boys function, and the ket then
 * bra Hermite-to-Cartesian sums.  The Boys function F_m(T) = int_0^1
 * t^{2m} exp(-T t^2) dt is taken from its power series (T < 30) or from
 * erf plus upward recursion (T >= 30), in long double.
 *
 * Component order inside a shell is lexicographic: for l = 2,
 * xx, xy, xz, yy, yz, zz.  Matrices are N x N row-major.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_LSHELL 3           /* shells: l <= 3                     */
#define ORC_LMAX 5             /* l <= 3 plus two (kinetic operator)  */
#define ORC_EDIM (ORC_LMAX + 1)
#define ORC_TDIM (2 * ORC_LMAX + 1)
#define ORC_RDIM (4 * ORC_LMAX + 1)
#define ORC_MAXPRIM 16

static const long double PI_L = 3.141592653589793238462643383279502884L;

typedef struct {
    int natom;
    const double *xyz;
    int nshell;
    const int *shell_atom;
    const int *shell_l;
    const int *shell_nprim;
    const int *shell_prim_off;
    const double *exps;
    const double *coefs;
} orc_basis;

int orc_version(void) { return 1; }

int orc_nthreads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

static int ncart(int l) { return (l + 1) * (l + 2) / 2; }

/* lexicographic Cartesian exponents of component n of angular momentum l */
static void cart_exp(int l, int n, int e[3])
{
    int idx = 0;
    for (int i = l; i >= 0; --i)
        for (int j = l - i; j >= 0; --j) {
            if (idx == n) {
                e[0] = i;
                e[1] = j;
                e[2] = l - i - j;
                return;
            }
            ++idx;
        }
}

static void ao_offsets(const orc_basis *b, int *off)
{
    off[0] = 0;
    for (int s = 0; s < b->nshell; ++s) off[s + 1] = off[s] + ncart(b->shell_l[s]);
}


/* l <= 3 and 1 <= nprim <= ORC_MAXPRIM for every shell */
static int check_basis(const orc_basis *b)
{
    for (int s = 0; s < b->nshell; ++s)
        if (b->shell_l[s] < 0 || b->shell_l[s] > ORC_LSHELL || b->shell_nprim[s] < 1 ||
            b->shell_nprim[s] > ORC_MAXPRIM)
            return -2;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Boys function                                                            */
/* ------------------------------------------------------------------------ */

static void boys_ld(int mmax, long double T, long double *F)
{
    if (T < 30.0L) {
        /* F_m(T) = exp(-T) sum_k (2T)^k / ((2m+1)(2m+3)...(2m+2k+1)),
         * all terms positive; then downward F_m = (2T F_{m+1} + e^-T)/(2m+1) */
        long double term = 1.0L / (2 * mmax + 1), sum = term;
        for (int k = 1; k < 2000; ++k) {
            term *= 2.0L * T / (long double)(2 * mmax + 2 * k + 1);
            sum += term;
            if (term < sum * 1e-22L) break;
        }
        long double e = expl(-T);
        F[mmax] = e * sum;
        for (int m = mmax - 1; m >= 0; --m) F[m] = (2.0L * T * F[m + 1] + e) / (2 * m + 1);
    } else {
        /* F_0 = sqrt(pi/T) erf(sqrt T) / 2, then the upward recursion
         * F_{m+1} = ((2m+1) F_m - e^-T) / (2T), stable for T >> m */
        long double e = expl(-T);
        F[0] = 0.5L * sqrtl(PI_L / T) * erfl(sqrtl(T));
        for (int m = 0; m < mmax; ++m) F[m + 1] = ((2 * m + 1) * F[m] - e) / (2.0L * T);
    }
}

int orc_boys(int mmax, double T, double *F)
{
    if (mmax < 0 || mmax > 40 || !(T >= 0.0)) return -1;
    long double f[41];
    boys_ld(mmax, (long double)T, f);
    for (int m = 0; m <= mmax; ++m) F[m] = (double)f[m];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* McMurchie-Davidson pieces                                                */
/* ------------------------------------------------------------------------ */

/* 1-D Hermite expansion coefficients of the product of two 1-D Gaussian
 * factors (x-A)^i (x-B)^j around P, E^{ij}_t for i <= imax, j <= jmax:
 *   E^{00}_0 = 1,
 *   E^{i+1,j}_t = E^{ij}_{t-1}/(2p) + X_PA E^{ij}_t + (t+1) E^{ij}_{t+1},
 *   E^{i,j+1}_t = E^{ij}_{t-1}/(2p) + X_PB E^{ij}_t + (t+1) E^{ij}_{t+1}.
 * (The exp(-mu X_AB^2) factor is carried in the pair prefactor.) */
static void hermite_E(int imax, int jmax, double p, double XPA, double XPB,
                      double E[ORC_EDIM][ORC_EDIM][ORC_TDIM])
{
    memset(E, 0, sizeof(double) * ORC_EDIM * ORC_EDIM * ORC_TDIM);
    const double h = 0.5 / p;
    E[0][0][0] = 1.0;
    for (int i = 0; i <= imax; ++i) {
        if (i > 0) {
            for (int t = 0; t <= i; ++t) {
                double v = XPA * E[i - 1][0][t];
                if (t > 0) v += h * E[i - 1][0][t - 1];
                if (t + 1 <= i - 1) v += (t + 1) * E[i - 1][0][t + 1];
                E[i][0][t] = v;
            }
        }
        for (int j = 1; j <= jmax; ++j) {
            for (int t = 0; t <= i + j; ++t) {
                double v = 0.0;
                if (t <= i + j - 1) v += XPB * E[i][j - 1][t];
                if (t > 0) v += h * E[i][j - 1][t - 1];
                if (t + 1 <= i + j - 1) v += (t + 1) * E[i][j - 1][t + 1];
                E[i][j][t] = v;
            }
        }
    }
}

/* Hermite Coulomb integrals R^0_{tuv}, t+u+v <= L:
 *   R^n_{000} = (-2 rho)^n F_n(rho |PQ|^2),
 *   R^n_{t+1,u,v} = t R^{n+1}_{t-1,u,v} + X_PQ R^{n+1}_{t,u,v}  (same in u, v).
 * R is stored as R[n][t][u][v] in a (L+1)^4 box. */
typedef struct {
    int L;
    double *R; /* (L+1)^4 */
} herm_R;

#define RIDX(L, n, t, u, v) ((((size_t)(n) * ((L) + 1) + (t)) * ((L) + 1) + (u)) * ((L) + 1) + (v))

static void hermite_R(herm_R *H, double rho, const double PQ[3])
{
    const int L = H->L;
    double *R = H->R;
    const double T = rho * (PQ[0] * PQ[0] + PQ[1] * PQ[1] + PQ[2] * PQ[2]);
    long double F[ORC_RDIM + 1];
    boys_ld(L, (long double)T, F);
    double fac = 1.0;
    for (int n = 0; n <= L; ++n) {
        R[RIDX(L, n, 0, 0, 0)] = fac * (double)F[n];
        fac *= -2.0 * rho;
    }
    for (int s = 1; s <= L; ++s)            /* s = t+u+v */
        for (int n = 0; n <= L - s; ++n)
            for (int t = 0; t <= s; ++t)
                for (int u = 0; u <= s - t; ++u) {
                    int v = s - t - u;
                    double val;
                    if (t > 0) {
                        val = PQ[0] * R[RIDX(L, n + 1, t - 1, u, v)];
                        if (t > 1) val += (t - 1) * R[RIDX(L, n + 1, t - 2, u, v)];
                    } else if (u > 0) {
                        val = PQ[1] * R[RIDX(L, n + 1, t, u - 1, v)];
                        if (u > 1) val += (u - 1) * R[RIDX(L, n + 1, t, u - 2, v)];
                    } else {
                        val = PQ[2] * R[RIDX(L, n + 1, t, u, v - 1)];
                        if (v > 1) val += (v - 1) * R[RIDX(L, n + 1, t, u, v - 2)];
                    }
                    R[RIDX(L, n, t, u, v)] = val;
                }
}

/* A primitive pair: exponents, centres, Hermite tables on three axes. */
typedef struct {
    double p, P[3], pref; /* pref = exp(-ab/p |AB|^2) */
    double E[3][ORC_EDIM][ORC_EDIM][ORC_TDIM];
} prim_pair;

static void make_prim_pair(double a, const double *A, double b, const double *B, int imax, int jmax,
                           prim_pair *pp)
{
    const double p = a + b;
    double AB2 = 0.0;
    pp->p = p;
    for (int x = 0; x < 3; ++x) {
        pp->P[x] = (a * A[x] + b * B[x]) / p;
        AB2 += (A[x] - B[x]) * (A[x] - B[x]);
    }
    pp->pref = exp(-a * b / p * AB2);
    for (int x = 0; x < 3; ++x)
        hermite_E(imax, jmax, p, pp->P[x] - A[x], pp->P[x] - B[x], pp->E[x]);
}

/* Primitive [ab|cd] for explicit Cartesian exponent triples, from a bra pair,
 * a ket pair and the Hermite integrals of that primitive quartet:
 *   [ab|cd] = 2 pi^{5/2} / (p q sqrt(p+q)) * pref_ab * pref_cd
 *             * sum_{tuv} E^{ab}_{tuv} sum_{t'u'v'} (-1)^{t'+u'+v'} E^{cd}_{t'u'v'} R_{t+t',u+u',v+v'} */
static double md_prim(const prim_pair *bra, const prim_pair *ket, const herm_R *H, const int a[3],
                      const int b[3], const int c[3], const int d[3])
{
    const int L = H->L;
    double sum = 0.0;
    for (int t = 0; t <= a[0] + b[0]; ++t) {
        const double ex = bra->E[0][a[0]][b[0]][t];
        if (ex == 0.0) continue;
        for (int u = 0; u <= a[1] + b[1]; ++u) {
            const double ey = bra->E[1][a[1]][b[1]][u];
            if (ey == 0.0) continue;
            for (int v = 0; v <= a[2] + b[2]; ++v) {
                const double ez = bra->E[2][a[2]][b[2]][v];
                if (ez == 0.0) continue;
                double inner = 0.0;
                for (int t2 = 0; t2 <= c[0] + d[0]; ++t2) {
                    const double fx = ket->E[0][c[0]][d[0]][t2];
                    for (int u2 = 0; u2 <= c[1] + d[1]; ++u2) {
                        const double fy = ket->E[1][c[1]][d[1]][u2];
                        for (int v2 = 0; v2 <= c[2] + d[2]; ++v2) {
                            const double fz = ket->E[2][c[2]][d[2]][v2];
                            const double sgn = ((t2 + u2 + v2) & 1) ? -1.0 : 1.0;
                            inner += sgn * fx * fy * fz * H->R[RIDX(L, 0, t + t2, u + u2, v + v2)];
                        }
                    }
                }
                sum += ex * ey * ez * inner;
            }
        }
    }
    const double p = bra->p, q = ket->p;
    const double pre = 2.0 * pow((double)PI_L, 2.5) / (p * q * sqrt(p + q)) * bra->pref * ket->pref;
    return pre * sum;
}

/* Per-thread work area */
typedef struct {
    herm_R H;
    prim_pair *bra, *ket; /* ORC_MAXPRIM^2 each */
} work_t;

static void work_init(work_t *w)
{
    w->H.L = 0;
    w->H.R = (double *)malloc(sizeof(double) * (size_t)ORC_RDIM * ORC_RDIM * ORC_RDIM * ORC_RDIM);
    w->bra = (prim_pair *)malloc(sizeof(prim_pair) * ORC_MAXPRIM * ORC_MAXPRIM);
    w->ket = (prim_pair *)malloc(sizeof(prim_pair) * ORC_MAXPRIM * ORC_MAXPRIM);
}

static void work_free(work_t *w)
{
    free(w->H.R);
    free(w->bra);
    free(w->ket);
}

/* all primitive pairs of shells (S1, S2), with Hermite tables up to l+extra */
static int shell_pairs(const orc_basis *B, int S1, int S2, int extra, prim_pair *out)
{
    const int n1 = B->shell_nprim[S1], n2 = B->shell_nprim[S2];
    const int o1 = B->shell_prim_off[S1], o2 = B->shell_prim_off[S2];
    const double *A = B->xyz + 3 * B->shell_atom[S1];
    const double *C = B->xyz + 3 * B->shell_atom[S2];
    int k = 0;
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n2; ++j)
            make_prim_pair(B->exps[o1 + i], A, B->exps[o2 + j], C, B->shell_l[S1] + extra,
                           B->shell_l[S2] + extra, &out[k++]);
    return k;
}

/* Contracted block (AB|CD), na*nb*nc*nd row-major, Eq. 2 */
static void eri_block(const orc_basis *B, int SA, int SB, int SC, int SD, double *out, work_t *w)
{
    const int la = B->shell_l[SA], lb = B->shell_l[SB], lc = B->shell_l[SC], ld = B->shell_l[SD];
    const int na = ncart(la), nb = ncart(lb), nc = ncart(lc), nd = ncart(ld);
    const int nbra = shell_pairs(B, SA, SB, 0, w->bra);
    const int nket = shell_pairs(B, SC, SD, 0, w->ket);
    const int nA = B->shell_nprim[SA], nB = B->shell_nprim[SB];
    const int nC = B->shell_nprim[SC], nD = B->shell_nprim[SD];
    (void)nA;
    memset(out, 0, sizeof(double) * (size_t)na * nb * nc * nd);
    w->H.L = la + lb + lc + ld;
    int ea[3], eb[3], ec[3], ed[3];
    for (int ib = 0; ib < nbra; ++ib) {
        const int k = ib / nB, l = ib % nB;
        const double cab = B->coefs[B->shell_prim_off[SA] + k] * B->coefs[B->shell_prim_off[SB] + l];
        for (int ik = 0; ik < nket; ++ik) {
            const int m = ik / nD, n = ik % nD;
            (void)nC;
            const double ccd = B->coefs[B->shell_prim_off[SC] + m] * B->coefs[B->shell_prim_off[SD] + n];
            const prim_pair *bra = &w->bra[ib], *ket = &w->ket[ik];
            const double p = bra->p, q = ket->p, rho = p * q / (p + q);
            double PQ[3] = {bra->P[0] - ket->P[0], bra->P[1] - ket->P[1], bra->P[2] - ket->P[2]};
            hermite_R(&w->H, rho, PQ);
            size_t idx = 0;
            for (int ia = 0; ia < na; ++ia) {
                cart_exp(la, ia, ea);
                for (int jb = 0; jb < nb; ++jb) {
                    cart_exp(lb, jb, eb);
                    for (int kc = 0; kc < nc; ++kc) {
                        cart_exp(lc, kc, ec);
                        for (int ld2 = 0; ld2 < nd; ++ld2) {
                            cart_exp(ld, ld2, ed);
                            out[idx++] += cab * ccd * md_prim(bra, ket, &w->H, ea, eb, ec, ed);
                        }
                    }
                }
            }
        }
    }
}

int orc_eri_block(const orc_basis *B, int SA, int SB, int SC, int SD, double *out)
{
    if (check_basis(B)) return -2;
    if (SA < 0 || SB < 0 || SC < 0 || SD < 0 || SA >= B->nshell || SB >= B->nshell ||
        SC >= B->nshell || SD >= B->nshell)
        return -1;
    work_t w;
    work_init(&w);
    eri_block(B, SA, SB, SC, SD, out, &w);
    work_free(&w);
    return 0;
}

/* Full N^4 tensor, row-major (mu nu | la si) */
int orc_eri_tensor(const orc_basis *B, double *out)
{
    if (check_basis(B)) return -2;
    const int ns = B->nshell;
    int *off = (int *)malloc(sizeof(int) * (ns + 1));
    ao_offsets(B, off);
    const size_t N = (size_t)off[ns];
#pragma omp parallel
    {
        work_t w;
        work_init(&w);
        double *blk = (double *)malloc(sizeof(double) * 10 * 10 * 10 * 10);
#pragma omp for schedule(dynamic)
        for (int AB = 0; AB < ns * ns; ++AB) {
            const int SA = AB / ns, SB = AB % ns;
            for (int SC = 0; SC < ns; ++SC)
                for (int SD = 0; SD < ns; ++SD) {
                    eri_block(B, SA, SB, SC, SD, blk, &w);
                    const int na = ncart(B->shell_l[SA]), nb = ncart(B->shell_l[SB]);
                    const int nc = ncart(B->shell_l[SC]), nd = ncart(B->shell_l[SD]);
                    size_t idx = 0;
                    for (int a = 0; a < na; ++a)
                        for (int b = 0; b < nb; ++b)
                            for (int c = 0; c < nc; ++c)
                                for (int d = 0; d < nd; ++d) {
                                    const size_t I = off[SA] + a, J = off[SB] + b, K = off[SC] + c,
                                                 L = off[SD] + d;
                                    out[((I * N + J) * N + K) * N + L] = blk[idx++];
                                }
                }
        }
        free(blk);
        work_free(&w);
    }
    free(off);
    return 0;
}

/* Schwarz factors Q[A][B] = sqrt(max_{a in A, b in B} (ab|ab)), nshell^2 */
int orc_schwarz(const orc_basis *B, double *Q)
{
    if (check_basis(B)) return -2;
    const int ns = B->nshell;
#pragma omp parallel
    {
        work_t w;
        work_init(&w);
        double *blk = (double *)malloc(sizeof(double) * 10 * 10 * 10 * 10);
#pragma omp for schedule(dynamic)
        for (int SA = 0; SA < ns; ++SA)
            for (int SB = 0; SB <= SA; ++SB) {
                eri_block(B, SA, SB, SA, SB, blk, &w);
                const int na = ncart(B->shell_l[SA]), nb = ncart(B->shell_l[SB]);
                double mx = 0.0;
                for (int a = 0; a < na; ++a)
                    for (int b = 0; b < nb; ++b) {
                        const double v = blk[((a * nb + b) * na + a) * nb + b];
                        if (v > mx) mx = v;
                    }
                Q[SA * ns + SB] = Q[SB * ns + SA] = sqrt(mx);
            }
        free(blk);
        work_free(&w);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* J and K                                                                  */
/* ------------------------------------------------------------------------ */

/* Unique shell quartets (AB|CD): A >= B, C >= D, pair(AB) >= pair(CD), with
 * pair(XY) = X(X+1)/2 + Y.  Each unique quartet stands for its eight
 * permutational images; with symmetric D its contribution is
 *   w = (ab|cd) / (s_AB s_CD s_ABCD)   (s = 2 for identical shells / pairs),
 *   Jt_ab += 2 w D_cd,  Jt_cd += 2 w D_ab,
 *   Kt_ac += w D_bd,  Kt_ad += w D_bc,  Kt_bc += w D_ad,  Kt_bd += w D_ac,
 * and J = Jt + Jt^T, K = Kt + Kt^T.  A quartet is skipped when
 * Q_AB Q_CD < tau.  This routine accumulates Jt, Kt over the bra pairs listed
 * in rows[] (pair indices); passing every pair gives the whole matrices. */
int orc_jk_rows(const orc_basis *B, const double *D, double tau, const double *Q, int nrows,
                const int *rows, double *Jt, double *Kt, long long *nquartets)
{
    if (check_basis(B)) return -2;
    const int ns = B->nshell;
    int *off = (int *)malloc(sizeof(int) * (ns + 1));
    ao_offsets(B, off);
    const int N = off[ns];
    const int npair = ns * (ns + 1) / 2;
    int *pA = (int *)malloc(sizeof(int) * npair), *pB = (int *)malloc(sizeof(int) * npair);
    for (int A = 0, k = 0; A < ns; ++A)
        for (int Bs = 0; Bs <= A; ++Bs, ++k) {
            pA[k] = A;
            pB[k] = Bs;
        }
    for (int r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= npair) {
            free(off);
            free(pA);
            free(pB);
            return -1;
        }
    long long count = 0;
#pragma omp parallel reduction(+ : count)
    {
        work_t w;
        work_init(&w);
        double *blk = (double *)malloc(sizeof(double) * 10 * 10 * 10 * 10);
        double *jl = (double *)calloc((size_t)N * N, sizeof(double));
        double *kl = (double *)calloc((size_t)N * N, sizeof(double));
#pragma omp for schedule(dynamic)
        for (int r = 0; r < nrows; ++r) {
            const int ab = rows[r];
            const int SA = pA[ab], SB = pB[ab];
            for (int cd = 0; cd <= ab; ++cd) {
                const int SC = pA[cd], SD = pB[cd];
                if (Q[SA * ns + SB] * Q[SC * ns + SD] < tau) continue;
                ++count;
                eri_block(B, SA, SB, SC, SD, blk, &w);
                double s = 1.0;
                if (SA == SB) s *= 2.0;
                if (SC == SD) s *= 2.0;
                if (ab == cd) s *= 2.0;
                const double wgt = 1.0 / s;
                const int na = ncart(B->shell_l[SA]), nb = ncart(B->shell_l[SB]);
                const int nc = ncart(B->shell_l[SC]), nd = ncart(B->shell_l[SD]);
                size_t idx = 0;
                for (int i = 0; i < na; ++i)
                    for (int j = 0; j < nb; ++j)
                        for (int k = 0; k < nc; ++k)
                            for (int l = 0; l < nd; ++l) {
                                const int a = off[SA] + i, b = off[SB] + j, c = off[SC] + k,
                                          d = off[SD] + l;
                                const double v = wgt * blk[idx++];
                                jl[(size_t)a * N + b] += 2.0 * v * D[(size_t)c * N + d];
                                jl[(size_t)c * N + d] += 2.0 * v * D[(size_t)a * N + b];
                                kl[(size_t)a * N + c] += v * D[(size_t)b * N + d];
                                kl[(size_t)a * N + d] += v * D[(size_t)b * N + c];
                                kl[(size_t)b * N + c] += v * D[(size_t)a * N + d];
                                kl[(size_t)b * N + d] += v * D[(size_t)a * N + c];
                            }
            }
        }
#pragma omp critical
        {
            for (size_t i = 0; i < (size_t)N * N; ++i) {
                Jt[i] += jl[i];
                Kt[i] += kl[i];
            }
        }
        free(jl);
        free(kl);
        free(blk);
        work_free(&w);
    }
    *nquartets = count;
    free(off);
    free(pA);
    free(pB);
    return 0;
}

/* J and K blocks by their plain definitions, one shell pair (A, B) at a time:
 *   J_ab = sum_{C,D} sum_{c in C, d in D} (ab|cd) D_cd   (skip Q_AB Q_CD < tau)
 *   K_ab = sum_{C,D} sum_{c in C, d in D} (ac|bd) D_cd   (skip Q_AC Q_BD < tau)
 * over all shells C, D with no symmetry used.  blk[2*i], blk[2*i+1] = (A, B)
 * of block i; Jb, Kb hold the blocks back to back (na*nb each, row-major). */
int orc_jk_blocks(const orc_basis *B, const double *D, double tau, const double *Q, int nblk,
                  const int *blk, double *Jb, double *Kb)
{
    if (check_basis(B)) return -2;
    const int ns = B->nshell;
    int *off = (int *)malloc(sizeof(int) * (ns + 1));
    ao_offsets(B, off);
    const int N = off[ns];
    size_t *boff = (size_t *)malloc(sizeof(size_t) * (nblk + 1));
    boff[0] = 0;
    for (int i = 0; i < nblk; ++i) {
        if (blk[2 * i] < 0 || blk[2 * i] >= ns || blk[2 * i + 1] < 0 || blk[2 * i + 1] >= ns) {
            free(off);
            free(boff);
            return -1;
        }
        boff[i + 1] = boff[i] + (size_t)ncart(B->shell_l[blk[2 * i]]) * ncart(B->shell_l[blk[2 * i + 1]]);
    }
    memset(Jb, 0, sizeof(double) * boff[nblk]);
    memset(Kb, 0, sizeof(double) * boff[nblk]);
    for (int i = 0; i < nblk; ++i) {
        const int SA = blk[2 * i], SB = blk[2 * i + 1];
        const int na = ncart(B->shell_l[SA]), nb = ncart(B->shell_l[SB]);
        double *jo = Jb + boff[i], *ko = Kb + boff[i];
#pragma omp parallel
        {
            work_t w;
            work_init(&w);
            double *eri = (double *)malloc(sizeof(double) * 10 * 10 * 10 * 10);
            double *jl = (double *)calloc((size_t)na * nb, sizeof(double));
            double *kl = (double *)calloc((size_t)na * nb, sizeof(double));
#pragma omp for schedule(dynamic)
            for (int CD = 0; CD < ns * ns; ++CD) {
                const int SC = CD / ns, SD = CD % ns;
                const int nc = ncart(B->shell_l[SC]), nd = ncart(B->shell_l[SD]);
                if (!(Q[SA * ns + SB] * Q[SC * ns + SD] < tau)) {
                    eri_block(B, SA, SB, SC, SD, eri, &w); /* (ab|cd) */
                    for (int a = 0; a < na; ++a)
                        for (int b = 0; b < nb; ++b) {
                            double s = 0.0;
                            for (int c = 0; c < nc; ++c)
                                for (int d = 0; d < nd; ++d)
                                    s += eri[((a * nb + b) * nc + c) * nd + d] *
                                         D[(size_t)(off[SC] + c) * N + off[SD] + d];
                            jl[a * nb + b] += s;
                        }
                }
                /* K_ab: the quartet (A C | B D), components (a c | b d) */
                if (!(Q[SA * ns + SC] * Q[SB * ns + SD] < tau)) {
                    eri_block(B, SA, SC, SB, SD, eri, &w);
                    for (int a = 0; a < na; ++a)
                        for (int b = 0; b < nb; ++b) {
                            double s = 0.0;
                            for (int c = 0; c < nc; ++c)
                                for (int d = 0; d < nd; ++d)
                                    s += eri[((a * nc + c) * nb + b) * nd + d] *
                                         D[(size_t)(off[SC] + c) * N + off[SD] + d];
                            kl[a * nb + b] += s;
                        }
                }
            }
#pragma omp critical
            {
                for (int k = 0; k < na * nb; ++k) {
                    jo[k] += jl[k];
                    ko[k] += kl[k];
                }
            }
            free(jl);
            free(kl);
            free(eri);
            work_free(&w);
        }
    }
    free(off);
    free(boff);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Overlap (for the normalization check of the input recipe)               */
/* ------------------------------------------------------------------------ */

/* Contracted overlap block <a|b> = sum_kl c_ak c_bl prod_x E^{ij}_0 sqrt(pi/p) */
int orc_overlap_block(const orc_basis *B, int SA, int SB, double *out)
{
    if (check_basis(B)) return -2;
    if (SA < 0 || SB < 0 || SA >= B->nshell || SB >= B->nshell) return -1;
    const int la = B->shell_l[SA], lb = B->shell_l[SB];
    const int na = ncart(la), nb = ncart(lb);
    prim_pair *pp = (prim_pair *)malloc(sizeof(prim_pair) * ORC_MAXPRIM * ORC_MAXPRIM);
    const int np = shell_pairs(B, SA, SB, 0, pp);
    const int nB = B->shell_nprim[SB];
    memset(out, 0, sizeof(double) * na * nb);
    int ea[3], eb[3];
    for (int k = 0; k < np; ++k) {
        const double c = B->coefs[B->shell_prim_off[SA] + k / nB] * B->coefs[B->shell_prim_off[SB] + k % nB];
        const double s1 = sqrt((double)PI_L / pp[k].p);
        for (int a = 0; a < na; ++a) {
            cart_exp(la, a, ea);
            for (int b = 0; b < nb; ++b) {
                cart_exp(lb, b, eb);
                double v = pp[k].pref;
                for (int x = 0; x < 3; ++x) v *= pp[k].E[x][ea[x]][eb[x]][0] * s1;
                out[a * nb + b] += c * v;
            }
        }
    }
    free(pp);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One-electron integrals of the SCF loop (Section 2.1: the Fock matrix is   */
/* the one-electron Hamiltonian plus the two-electron part)                  */
/* ------------------------------------------------------------------------ */

/* Contracted blocks of shells (SA, SB), na*nb row-major each:
 *   S_ab = <a|b>,
 *   T_ab = <a| -1/2 nabla^2 |b>,
 *   V_ab = sum_C -Z_C <a| 1/|r - R_C| |b>   (point nuclei at the atom centres).
 * McMurchie-Davidson: with the 1-D Hermite coefficients E^{ij}_t of each
 * primitive pair and s = sqrt(pi/p) per axis,
 *   overlap factor   S^x_{ij} = E^{ij}_0 s,
 *   kinetic factor   K^x_{ij} = -1/2 [ j(j-1) S^x_{i,j-2} - 2 beta (2j+1) S^x_{ij}
 *                                      + 4 beta^2 S^x_{i,j+2} ]
 *                    (the second derivative of (x-B)^j exp(-beta (x-B)^2)),
 *   T = K^x S^y S^z + S^x K^y S^z + S^x S^y K^z,
 *   V = -Z_C 2 pi / p sum_{tuv} E^x_t E^y_u E^z_v R_{tuv}(p, P - C),
 * each times exp(-alpha beta / p |AB|^2) and the contraction coefficients. */
static void one_e_block(const orc_basis *B, const double *Z, int SA, int SB, double *S, double *T, double *V,
                        prim_pair *pp, herm_R *H)
{
    const int la = B->shell_l[SA], lb = B->shell_l[SB];
    const int na = ncart(la), nb = ncart(lb);
    const int np = shell_pairs(B, SA, SB, 2, pp);
    const int nB = B->shell_nprim[SB];
    memset(S, 0, sizeof(double) * na * nb);
    memset(T, 0, sizeof(double) * na * nb);
    memset(V, 0, sizeof(double) * na * nb);
    H->L = la + lb;
    int ea[3], eb[3];
    for (int k = 0; k < np; ++k) {
        const double c = B->coefs[B->shell_prim_off[SA] + k / nB] * B->coefs[B->shell_prim_off[SB] + k % nB];
        const double beta = B->exps[B->shell_prim_off[SB] + k % nB];
        const prim_pair *q = &pp[k];
        const double s1 = sqrt((double)PI_L / q->p);
        for (int a = 0; a < na; ++a) {
            cart_exp(la, a, ea);
            for (int b = 0; b < nb; ++b) {
                cart_exp(lb, b, eb);
                double sx[3], kx[3];
                for (int x = 0; x < 3; ++x) {
                    const int i = ea[x], j = eb[x];
                    sx[x] = q->E[x][i][j][0] * s1;
                    double d2 = -2.0 * beta * (2 * j + 1) * sx[x] + 4.0 * beta * beta * q->E[x][i][j + 2][0] * s1;
                    if (j >= 2) d2 += j * (j - 1) * q->E[x][i][j - 2][0] * s1;
                    kx[x] = -0.5 * d2;
                }
                S[a * nb + b] += c * q->pref * sx[0] * sx[1] * sx[2];
                T[a * nb + b] += c * q->pref *
                                 (kx[0] * sx[1] * sx[2] + sx[0] * kx[1] * sx[2] + sx[0] * sx[1] * kx[2]);
            }
        }
        for (int C = 0; C < B->natom; ++C) {
            if (Z[C] == 0.0) continue;
            const double PC[3] = {q->P[0] - B->xyz[3 * C], q->P[1] - B->xyz[3 * C + 1], q->P[2] - B->xyz[3 * C + 2]};
            hermite_R(H, q->p, PC);
            const double pre = -Z[C] * 2.0 * (double)PI_L / q->p * q->pref * c;
            for (int a = 0; a < na; ++a) {
                cart_exp(la, a, ea);
                for (int b = 0; b < nb; ++b) {
                    cart_exp(lb, b, eb);
                    double sum = 0.0;
                    for (int t = 0; t <= ea[0] + eb[0]; ++t)
                        for (int u = 0; u <= ea[1] + eb[1]; ++u)
                            for (int v = 0; v <= ea[2] + eb[2]; ++v)
                                sum += q->E[0][ea[0]][eb[0]][t] * q->E[1][ea[1]][eb[1]][u] *
                                       q->E[2][ea[2]][eb[2]][v] * H->R[RIDX(H->L, 0, t, u, v)];
                    V[a * nb + b] += pre * sum;
                }
            }
        }
    }
}

/* Whole N x N matrices S, T, V (row-major), every shell pair (A, B). */
int orc_one_electron(const orc_basis *B, const double *Z, double *S, double *T, double *V)
{
    if (check_basis(B)) return -2;
    const int ns = B->nshell;
    int *off = (int *)malloc(sizeof(int) * (ns + 1));
    ao_offsets(B, off);
    const size_t N = (size_t)off[ns];
#pragma omp parallel
    {
        work_t w;
        work_init(&w);
        double bs[100], bt[100], bv[100];
#pragma omp for schedule(dynamic)
        for (int AB = 0; AB < ns * ns; ++AB) {
            const int SA = AB / ns, SB = AB % ns;
            one_e_block(B, Z, SA, SB, bs, bt, bv, w.bra, &w.H);
            const int na = ncart(B->shell_l[SA]), nb = ncart(B->shell_l[SB]);
            for (int a = 0; a < na; ++a)
                for (int b = 0; b < nb; ++b) {
                    const size_t i = (size_t)(off[SA] + a) * N + off[SB] + b;
                    S[i] = bs[a * nb + b];
                    T[i] = bt[a * nb + b];
                    V[i] = bv[a * nb + b];
                }
        }
        work_free(&w);
    }
    free(off);
    return 0;
}

/* Repulsion of the point nuclei, sum_{A<B} Z_A Z_B / |R_A - R_B|; a centre
 * without charge (Z = 0, a basis-only centre) adds nothing, also where it
 * coincides with another atom. */
double orc_nuclear_repulsion(int natom, const double *xyz, const double *Z)
{
    double e = 0.0;
    for (int a = 0; a < natom; ++a)
        for (int b = 0; b < a; ++b) {
            if (Z[a] == 0.0 || Z[b] == 0.0) continue;
            const double dx = xyz[3 * a] - xyz[3 * b], dy = xyz[3 * a + 1] - xyz[3 * b + 1],
                         dz = xyz[3 * a + 2] - xyz[3 * b + 2];
            e += Z[a] * Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
        }
    return e;
}

/* ------------------------------------------------------------------------ */
/* Nuclear gradient of E2 at fixed density                                  */
/* ------------------------------------------------------------------------ */

/* E2 = 1/2 Tr(DJ) - 1/4 Tr(DK) = sum_{abcd} (ab|cd) [D_ab D_cd / 2 - D_ac D_bd / 4].
 * The basis functions move with their atoms; a primitive's centre derivative
 * is d phi_a / dA_i = 2 alpha phi_{a+1_i} - a_i phi_{a-1_i}.  Summing the
 * four centre derivatives of every (ab|cd) over all shell quartets (no
 * permutational symmetry used) gives grad[atom][i] = dE2/dR_{atom,i}. */
int orc_grad_e2(const orc_basis *B, const double *D, double *grad)
{
    const int ns = B->nshell;
    int *off = (int *)malloc(sizeof(int) * (ns + 1));
    ao_offsets(B, off);
    const int N = off[ns];
    const int na_ = B->natom;
    for (int s = 0; s < ns; ++s)
        if (B->shell_l[s] > ORC_LSHELL || B->shell_nprim[s] > ORC_MAXPRIM) {
            free(off);
            return -2;
        }
    memset(grad, 0, sizeof(double) * 3 * na_);
#pragma omp parallel
    {
        work_t w;
        work_init(&w);
        double *gl = (double *)calloc((size_t)3 * na_, sizeof(double));
#pragma omp for schedule(dynamic)
        for (int AB = 0; AB < ns * ns; ++AB) {
            const int S[2] = {AB / ns, AB % ns};
            for (int SC = 0; SC < ns; ++SC)
                for (int SD = 0; SD < ns; ++SD) {
                    const int sh[4] = {S[0], S[1], SC, SD};
                    int l[4], n[4];
                    for (int k = 0; k < 4; ++k) {
                        l[k] = B->shell_l[sh[k]];
                        n[k] = ncart(l[k]);
                    }
                    const int nbra = shell_pairs(B, sh[0], sh[1], 1, w.bra);
                    const int nket = shell_pairs(B, sh[2], sh[3], 1, w.ket);
                    const int nB = B->shell_nprim[sh[1]], nD = B->shell_nprim[sh[3]];
                    w.H.L = l[0] + l[1] + l[2] + l[3] + 1;
                    for (int ib = 0; ib < nbra; ++ib)
                        for (int ik = 0; ik < nket; ++ik) {
                            const int pk[4] = {ib / nB, ib % nB, ik / nD, ik % nD};
                            double cprod = 1.0, alpha[4];
                            for (int k = 0; k < 4; ++k) {
                                cprod *= B->coefs[B->shell_prim_off[sh[k]] + pk[k]];
                                alpha[k] = B->exps[B->shell_prim_off[sh[k]] + pk[k]];
                            }
                            const prim_pair *bra = &w.bra[ib], *ket = &w.ket[ik];
                            const double p = bra->p, q = ket->p, rho = p * q / (p + q);
                            double PQ[3] = {bra->P[0] - ket->P[0], bra->P[1] - ket->P[1],
                                            bra->P[2] - ket->P[2]};
                            hermite_R(&w.H, rho, PQ);
                            int e[4][3];
                            for (int i0 = 0; i0 < n[0]; ++i0)
                                for (int i1 = 0; i1 < n[1]; ++i1)
                                    for (int i2 = 0; i2 < n[2]; ++i2)
                                        for (int i3 = 0; i3 < n[3]; ++i3) {
                                            const int idx[4] = {i0, i1, i2, i3};
                                            for (int k = 0; k < 4; ++k) cart_exp(l[k], idx[k], e[k]);
                                            const int a = off[sh[0]] + i0, b = off[sh[1]] + i1,
                                                      c = off[sh[2]] + i2, d = off[sh[3]] + i3;
                                            const double wD =
                                                0.5 * D[(size_t)a * N + b] * D[(size_t)c * N + d] -
                                                0.25 * D[(size_t)a * N + c] * D[(size_t)b * N + d];
                                            if (wD == 0.0) continue;
                                            for (int k = 0; k < 4; ++k)
                                                for (int x = 0; x < 3; ++x) {
                                                    int ee[4][3];
                                                    memcpy(ee, e, sizeof(ee));
                                                    ee[k][x] += 1;
                                                    double dv = 2.0 * alpha[k] *
                                                                md_prim(bra, ket, &w.H, ee[0], ee[1], ee[2], ee[3]);
                                                    if (e[k][x] > 0) {
                                                        memcpy(ee, e, sizeof(ee));
                                                        ee[k][x] -= 1;
                                                        dv -= e[k][x] *
                                                              md_prim(bra, ket, &w.H, ee[0], ee[1], ee[2], ee[3]);
                                                    }
                                                    gl[3 * B->shell_atom[sh[k]] + x] += cprod * wD * dv;
                                                }
                                        }
                        }
                }
        }
#pragma omp critical
        {
            for (int i = 0; i < 3 * na_; ++i) grad[i] += gl[i];
        }
        free(gl);
        work_free(&w);
    }
    free(off);
    return 0;
}
