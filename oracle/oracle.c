/*
 * FP64 CPU oracle for nuclear two-point correlators (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library. It shares no code with the GPU
 * library. Every routine is a plain transcription of a definition:
 *
 *  - Wick's theorem for the quark fields (Sec. 3.1, the expansion before
 *    Eq. 2.8): <q..q qbar..qbar> = sum over bijections sigma of sgn(sigma)
 *    prod_q S(chi_q, chi'_sigma(q)), with contractions between different
 *    flavors vanishing. sgn is the sign of sigma as a permutation of quark
 *    positions (so the flavor-grouping factor eta of Eq. 2.8 is included).
 *  - Zero-momentum nucleon sinks (Sec. 2.1, Eqs. 2.4-2.6 and the A-nucleon
 *    form of App. D): every nucleon a is summed over its own site x_a.
 *  - Baryon block (Eq. 2.4 / App. D): B_k[i1,i2,i3] = sum_x sum_j w_k(j)
 *    S_f1(x)[j1,i1] S_f2(x)[j2,i2] S_f3(x)[j3,i3].
 *
 * Arrays: a propagator at one time slice is S[V][12][12] complex (sink index
 * j is the row, source index i the column). Complex numbers are interleaved
 * (re, im) doubles. Kinds: flav[3*K], nw[K], woff[K], wj[3*total],
 * wre[total], wim[total]. Patterns: kind[n*A], c[2*n].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

/* Neumaier compensated accumulator for one complex value. */
typedef struct { double sr, cr, si, ci; } acc_t;

static void nadd(double *s, double *c, double x)
{
    double t = *s + x;
    if (fabs(*s) >= fabs(x)) *c += (*s - t) + x; else *c += (x - t) + *s;
    *s = t;
}

static void acc_add(acc_t *a, cplx z) { nadd(&a->sr, &a->cr, creal(z)); nadd(&a->si, &a->ci, cimag(z)); }
static cplx acc_val(const acc_t *a) { return (a->sr + a->cr) + I * (a->si + a->ci); }

static const cplx *site(const cplx *S, int64_t x) { return S + x * 144; }

/* ------------------------------------------------------------------------- */
/* Blocks                                                                     */
/* ------------------------------------------------------------------------- */

/* Raw block of one kind (the block formula written out). B[i1*144+i2*12+i3]. */
void oracle_block_raw(int64_t V, const double *Su_, const double *Sd_, const int32_t *flav,
                      int32_t nw, const int32_t *wj, const double *wre, const double *wim,
                      double *B_)
{
    const cplx *S[2] = {(const cplx *)Su_, (const cplx *)Sd_};
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    acc_t *part = calloc((size_t)nth * 1728, sizeof(acc_t));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        acc_t *acc = part + (size_t)tid * 1728;
#pragma omp for schedule(static)
        for (int64_t x = 0; x < V; ++x) {
            const cplx *s1 = site(S[flav[0]], x), *s2 = site(S[flav[1]], x), *s3 = site(S[flav[2]], x);
            for (int n = 0; n < nw; ++n) {
                cplx w = wre[n] + I * wim[n];
                const cplx *r1 = s1 + 12 * wj[3 * n], *r2 = s2 + 12 * wj[3 * n + 1], *r3 = s3 + 12 * wj[3 * n + 2];
                for (int i1 = 0; i1 < 12; ++i1)
                    for (int i2 = 0; i2 < 12; ++i2) {
                        cplx a = w * r1[i1] * r2[i2];
                        for (int i3 = 0; i3 < 12; ++i3) acc_add(&acc[i1 * 144 + i2 * 12 + i3], a * r3[i3]);
                    }
            }
        }
    }
    cplx *B = (cplx *)B_;
    for (int e = 0; e < 1728; ++e) {
        acc_t tot = {0, 0, 0, 0};
        for (int t = 0; t < nth; ++t) acc_add(&tot, acc_val(&part[(size_t)t * 1728 + e]));
        B[e] = acc_val(&tot);
    }
    free(part);
}

/* The block as Eq. 2.4 writes it, antisymmetrised in the two same-flavor
 * source slots (here slots 1 and 3, which must share a flavor):
 * B[i1,i2,i3] = sum_x sum_j w(j) [S_f(j1,i1) S_f(j3,i3) - S_f(j3,i1) S_f(j1,i3)] S_g(j2,i2). */
void oracle_block_eq24(int64_t V, const double *Su_, const double *Sd_, const int32_t *flav,
                       int32_t nw, const int32_t *wj, const double *wre, const double *wim,
                       double *B_)
{
    const cplx *S[2] = {(const cplx *)Su_, (const cplx *)Sd_};
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    acc_t *part = calloc((size_t)nth * 1728, sizeof(acc_t));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        acc_t *acc = part + (size_t)tid * 1728;
#pragma omp for schedule(static)
        for (int64_t x = 0; x < V; ++x) {
            const cplx *sf = site(S[flav[0]], x), *sg = site(S[flav[1]], x);
            for (int n = 0; n < nw; ++n) {
                cplx w = wre[n] + I * wim[n];
                const cplx *a = sf + 12 * wj[3 * n], *b = sg + 12 * wj[3 * n + 1], *c = sf + 12 * wj[3 * n + 2];
                for (int i1 = 0; i1 < 12; ++i1)
                    for (int i3 = 0; i3 < 12; ++i3) {
                        cplx uu = a[i1] * c[i3] - c[i1] * a[i3];
                        for (int i2 = 0; i2 < 12; ++i2) acc_add(&acc[i1 * 144 + i2 * 12 + i3], w * uu * b[i2]);
                    }
            }
        }
    }
    cplx *B = (cplx *)B_;
    for (int e = 0; e < 1728; ++e) {
        acc_t tot = {0, 0, 0, 0};
        for (int t = 0; t < nth; ++t) acc_add(&tot, acc_val(&part[(size_t)t * 1728 + e]));
        B[e] = acc_val(&tot);
    }
    free(part);
}

/* ------------------------------------------------------------------------- */
/* Helpers for operators                                                      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int32_t K;
    const int32_t *flav, *nw, *woff, *wj;
    const double *wre, *wim;
} kinds_t;

/* Flavor listing of a pattern (3A entries, nucleon by nucleon). */
static void listing(const kinds_t *ks, int A, const int32_t *pk, int *f)
{
    for (int a = 0; a < A; ++a)
        for (int s = 0; s < 3; ++s) f[3 * a + s] = ks->flav[3 * pk[a] + s];
}

static int perm_parity(const int *p, int n)
{
    int inv = 0;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) inv += p[i] > p[j];
    return inv & 1;
}

/* All flavor-preserving bijections sink position -> source position and their
 * signs. Returns the count; sig is [count][n], sgn is [count]. */
static int next_perm(int *a, int n)
{
    int i = n - 2;
    while (i >= 0 && a[i] >= a[i + 1]) --i;
    if (i < 0) return 0;
    int j = n - 1;
    while (a[j] <= a[i]) --j;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = n - 1; l < r; ++l, --r) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

static int bijections(const int *f, const int *g, int n, int **sig_out, int **sgn_out)
{
    int qu[16], qd[16], ru[16], rd[16], nu = 0, nd = 0, mu = 0, md = 0;
    for (int q = 0; q < n; ++q) { if (f[q] == 0) qu[nu++] = q; else qd[nd++] = q; }
    for (int r = 0; r < n; ++r) { if (g[r] == 0) ru[mu++] = r; else rd[md++] = r; }
    *sig_out = NULL; *sgn_out = NULL;
    if (nu != mu || nd != md) return 0;
    long cnt = 1;
    for (int i = 2; i <= nu; ++i) cnt *= i;
    for (int i = 2; i <= nd; ++i) cnt *= i;
    int *sig = malloc(sizeof(int) * cnt * n), *sgn = malloc(sizeof(int) * cnt);
    int pu[16], pd[16], k = 0;
    for (int i = 0; i < nu; ++i) pu[i] = i;
    do {
        for (int i = 0; i < nd; ++i) pd[i] = i;
        do {
            int *s = sig + (long)k * n;
            for (int i = 0; i < nu; ++i) s[qu[i]] = ru[pu[i]];
            for (int i = 0; i < nd; ++i) s[qd[i]] = rd[pd[i]];
            sgn[k] = perm_parity(s, n) ? -1 : 1;
            ++k;
        } while (next_perm(pd, nd));
    } while (next_perm(pu, nu));
    *sig_out = sig; *sgn_out = sgn;
    return k;
}

/* Expand the nonzero weight entries of a product of A kinds: returns count,
 * idx [count][3A] and weight [count]. */
static long expand(const kinds_t *ks, int A, const int32_t *pk, int **idx_out, cplx **w_out)
{
    long cnt = 1;
    for (int a = 0; a < A; ++a) cnt *= ks->nw[pk[a]];
    int *idx = malloc(sizeof(int) * (cnt ? cnt : 1) * 3 * A);
    cplx *w = malloc(sizeof(cplx) * (cnt ? cnt : 1));
    int ctr[16] = {0};
    for (long n = 0; n < cnt; ++n) {
        cplx prod = 1.0;
        for (int a = 0; a < A; ++a) {
            int k = pk[a], e = ks->woff[k] + ctr[a];
            for (int s = 0; s < 3; ++s) idx[n * 3 * A + 3 * a + s] = ks->wj[3 * e + s];
            prod *= ks->wre[e] + I * ks->wim[e];
        }
        w[n] = prod;
        for (int a = A - 1; a >= 0; --a) {
            if (++ctr[a] < ks->nw[pk[a]]) break;
            ctr[a] = 0;
        }
    }
    *idx_out = idx; *w_out = w;
    return cnt;
}

/* ------------------------------------------------------------------------- */
/* Route 1: the definition, quark by quark, on a small lattice.               */
/*                                                                            */
/* mode 0: sum over every flavor-preserving bijection of all 3A positions     */
/*         with its full sign.                                                */
/* mode 1: the same sum, flavor by flavor (Eqs. 2.8-2.9): eta times the       */
/*         Leibniz sums over the u positions and over the d positions (the    */
/*         determinants of M^u and M^d), eta being the full sign of the       */
/*         order-preserving bijection.                                        */
/* ------------------------------------------------------------------------- */
static int all_perms(int n, int **out, int **sgn_out)
{
    long cnt = 1;
    for (int i = 2; i <= n; ++i) cnt *= i;
    int *p = malloc(sizeof(int) * cnt * (n ? n : 1)), *sg = malloc(sizeof(int) * cnt), a[16];
    for (int i = 0; i < n; ++i) a[i] = i;
    long k = 0;
    do {
        for (int i = 0; i < n; ++i) p[k * n + i] = a[i];
        sg[k] = perm_parity(a, n) ? -1 : 1;
        ++k;
    } while (next_perm(a, n));
    *out = p; *sgn_out = sg;
    return (int)k;
}

long oracle_count_bijections(int32_t n, const int32_t *f, const int32_t *g)
{
    int ff[48], gg[48], *sig, *sgn;
    for (int i = 0; i < n; ++i) { ff[i] = f[i]; gg[i] = g[i]; }
    int k = bijections(ff, gg, n, &sig, &sgn);
    free(sig); free(sgn);
    return k;
}

void oracle_bruteforce(int32_t A, int64_t V, const double *Su_, const double *Sd_,
                       int32_t K, const int32_t *flav, const int32_t *nw, const int32_t *woff,
                       const int32_t *wj, const double *wre, const double *wim,
                       int32_t n_snk, const int32_t *snk_kind, const double *snk_c,
                       int32_t n_src, const int32_t *src_kind, const double *src_c,
                       int32_t mode, double *out)
{
    const cplx *S[2] = {(const cplx *)Su_, (const cplx *)Sd_};
    kinds_t ks = {K, flav, nw, woff, wj, wre, wim};
    const int n = 3 * A;
    long nx = 1;
    for (int a = 0; a < A; ++a) nx *= V;
    acc_t total = {0, 0, 0, 0}, mag = {0, 0, 0, 0};
    for (int s = 0; s < n_snk; ++s) {
        int f[48];
        listing(&ks, A, snk_kind + s * A, f);
        int *J; cplx *wJ;
        long nJ = expand(&ks, A, snk_kind + s * A, &J, &wJ);
        cplx cs = snk_c[2 * s] + I * snk_c[2 * s + 1];
        for (int sp = 0; sp < n_src; ++sp) {
            int g[48];
            listing(&ks, A, src_kind + sp * A, g);
            int qu[48], qd[48], ru[48], rd[48], nu = 0, nd = 0, mu = 0, md = 0;
            for (int q = 0; q < n; ++q) { if (f[q] == 0) qu[nu++] = q; else qd[nd++] = q; }
            for (int r = 0; r < n; ++r) { if (g[r] == 0) ru[mu++] = r; else rd[md++] = r; }
            if (nu != mu || nd != md) continue;
            int *sig = NULL, *sgn = NULL, nsig = 0;
            int *pu = NULL, *su = NULL, *pd = NULL, *sd = NULL, npu = 0, npd = 0, eta = 1;
            if (mode == 0) {
                nsig = bijections(f, g, n, &sig, &sgn);
            } else {
                int s0[48];
                for (int i = 0; i < nu; ++i) s0[qu[i]] = ru[i];
                for (int i = 0; i < nd; ++i) s0[qd[i]] = rd[i];
                eta = perm_parity(s0, n) ? -1 : 1;
                npu = all_perms(nu, &pu, &su);
                npd = all_perms(nd, &pd, &sd);
            }
            int *Iix; cplx *wI;
            long nI = expand(&ks, A, src_kind + sp * A, &Iix, &wI);
            cplx csp = src_c[2 * sp] + I * src_c[2 * sp + 1];
            int nth = 1;
#ifdef _OPENMP
            nth = omp_get_max_threads();
#endif
            acc_t *part = calloc(2 * nth, sizeof(acc_t));
#pragma omp parallel
            {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
                const cplx *row[48];
#pragma omp for schedule(dynamic)
                for (long xt = 0; xt < nx; ++xt) {
                    int64_t xs[16];
                    long r = xt;
                    for (int a = 0; a < A; ++a) { xs[a] = r % V; r /= V; }
                    for (long j = 0; j < nJ; ++j) {
                        for (int q = 0; q < n; ++q)
                            row[q] = site(S[f[q]], xs[q / 3]) + 12 * J[j * n + q];
                        for (long i = 0; i < nI; ++i) {
                            const int *Ii = Iix + i * n;
                            cplx sum = 0;
                            double amag = 0;
                            if (mode == 0) {
                                for (int k = 0; k < nsig; ++k) {
                                    const int *sg = sig + (long)k * n;
                                    cplx prod = sgn[k];
                                    for (int q = 0; q < n; ++q) prod *= row[q][Ii[sg[q]]];
                                    sum += prod;
                                    amag += cabs(prod);
                                }
                            } else {
                                cplx du = 0, dd = 0;
                                for (int k = 0; k < npu; ++k) {
                                    cplx prod = su[k];
                                    for (int c = 0; c < nu; ++c) prod *= row[qu[c]][Ii[ru[pu[k * nu + c]]]];
                                    du += prod;
                                }
                                for (int k = 0; k < npd; ++k) {
                                    cplx prod = sd[k];
                                    for (int c = 0; c < nd; ++c) prod *= row[qd[c]][Ii[rd[pd[k * nd + c]]]];
                                    dd += prod;
                                }
                                sum = eta * du * dd;
                                amag = cabs(sum);
                            }
                            cplx coef = cs * csp * wJ[j] * wI[i];
                            acc_add(&part[2 * tid], coef * sum);
                            acc_add(&part[2 * tid + 1], cabs(coef) * amag);
                        }
                    }
                }
            }
            for (int t = 0; t < nth; ++t) {
                acc_add(&total, acc_val(&part[2 * t]));
                acc_add(&mag, acc_val(&part[2 * t + 1]));
            }
            free(part); free(Iix); free(wI); free(sig); free(sgn);
            free(pu); free(su); free(pd); free(sd);
        }
        free(J); free(wJ);
    }
    cplx c = acc_val(&total);
    out[0] = creal(c); out[1] = cimag(c);
    out[2] = creal(acc_val(&mag));
}

/* ------------------------------------------------------------------------- */
/* Route 2: blocks, every source index tuple and every bijection (Eq. 2.6).   */
/* B is [K][1728] raw blocks of one time slice.                               */
/* ------------------------------------------------------------------------- */
void oracle_sum_full(int32_t A, const double *B_,
                     int32_t K, const int32_t *flav, const int32_t *nw, const int32_t *woff,
                     const int32_t *wj, const double *wre, const double *wim,
                     int32_t n_snk, const int32_t *snk_kind, const double *snk_c,
                     int32_t n_src, const int32_t *src_kind, const double *src_c,
                     double *out)
{
    const cplx *B = (const cplx *)B_;
    kinds_t ks = {K, flav, nw, woff, wj, wre, wim};
    const int n = 3 * A;
    acc_t total = {0, 0, 0, 0};
    for (int s = 0; s < n_snk; ++s) {
        int f[48];
        const int32_t *pk = snk_kind + s * A;
        listing(&ks, A, pk, f);
        cplx cs = snk_c[2 * s] + I * snk_c[2 * s + 1];
        for (int sp = 0; sp < n_src; ++sp) {
            int g[48];
            listing(&ks, A, src_kind + sp * A, g);
            int *sig, *sgn;
            int nsig = bijections(f, g, n, &sig, &sgn);
            if (!nsig) continue;
            int *Iix; cplx *wI;
            long nI = expand(&ks, A, src_kind + sp * A, &Iix, &wI);
            cplx csp = src_c[2 * sp] + I * src_c[2 * sp + 1];
            int nth = 1;
#ifdef _OPENMP
            nth = omp_get_max_threads();
#endif
            acc_t *part = calloc(nth, sizeof(acc_t));
#pragma omp parallel
            {
                int tid = 0;
#ifdef _OPENMP
                tid = omp_get_thread_num();
#endif
#pragma omp for schedule(dynamic, 16)
                for (long i = 0; i < nI; ++i) {
                    const int *Ii = Iix + i * n;
                    cplx sum = 0;
                    for (int k = 0; k < nsig; ++k) {
                        const int *sg = sig + (long)k * n;
                        cplx prod = sgn[k];
                        for (int a = 0; a < A; ++a) {
                            int e = Ii[sg[3 * a]] * 144 + Ii[sg[3 * a + 1]] * 12 + Ii[sg[3 * a + 2]];
                            prod *= B[(long)pk[a] * 1728 + e];
                        }
                        sum += prod;
                    }
                    acc_add(&part[tid], cs * csp * wI[i] * sum);
                }
            }
            for (int t = 0; t < nth; ++t) acc_add(&total, acc_val(&part[t]));
            free(part); free(Iix); free(wI); free(sig); free(sgn);
        }
    }
    cplx c = acc_val(&total);
    out[0] = creal(c); out[1] = cimag(c);
}

/* ------------------------------------------------------------------------- */
/* Route 3: antisymmetrised source (method A of Sec. 3.3) + a dynamic         */
/* programme over the used source positions (Laplace-style expansion).        */
/*                                                                            */
/* Every source index tuple I with pairwise different same-flavor indices is  */
/* mapped to its canonical ordering: all u indices ascending, then all d      */
/* indices ascending; W'[(U,D)] collects c' * w'(I) * sgn(map). The sink      */
/* blocks then take canonical positions in sink order; the sign of the whole  */
/* bijection is the parity of its inversions, added one position at a time.  */
/* ------------------------------------------------------------------------- */
typedef struct { uint64_t key; cplx w; } grp_t;

static int grp_cmp(const void *a, const void *b)
{
    uint64_t x = ((const grp_t *)a)->key, y = ((const grp_t *)b)->key;
    return x < y ? -1 : x > y;
}

/* Build the antisymmetrised source groups. Returns the count; key packs the
 * canonical index list (4 bits each, u's then d's). */
static long source_groups(const kinds_t *ks, int A, int32_t n_src, const int32_t *src_kind,
                          const double *src_c, int n_u_want, grp_t **out)
{
    const int n = 3 * A;
    long cap = 0, m = 0;
    grp_t *all = NULL;
    for (int sp = 0; sp < n_src; ++sp) {
        int g[48];
        listing(ks, A, src_kind + sp * A, g);
        int nu = 0;
        for (int r = 0; r < n; ++r) nu += g[r] == 0;
        if (nu != n_u_want) continue;
        int *Iix; cplx *wI;
        long nI = expand(ks, A, src_kind + sp * A, &Iix, &wI);
        cplx csp = src_c[2 * sp] + I * src_c[2 * sp + 1];
        if (m + nI > cap) { cap = 2 * (m + nI); all = realloc(all, sizeof(grp_t) * cap); }
        for (long i = 0; i < nI; ++i) {
            const int *Ii = Iix + i * n;
            int pos[48], ok = 1;
            /* canonical position of each listed quark */
            for (int r = 0; r < n && ok; ++r) {
                int rank = 0, base = g[r] == 0 ? 0 : nu;
                for (int r2 = 0; r2 < n; ++r2) {
                    if (r2 == r || g[r2] != g[r]) continue;
                    if (Ii[r2] == Ii[r]) { ok = 0; break; }   /* Pauli: repeated index */
                    rank += Ii[r2] < Ii[r];
                }
                pos[r] = base + rank;
            }
            if (!ok) continue;
            int canon[48];
            for (int r = 0; r < n; ++r) canon[pos[r]] = Ii[r];
            uint64_t key = 0;
            for (int p = 0; p < n; ++p) key = (key << 4) | (uint64_t)canon[p];
            all[m].key = key;
            all[m].w = csp * wI[i] * (perm_parity(pos, n) ? -1.0 : 1.0);
            ++m;
        }
        free(Iix); free(wI);
    }
    qsort(all, m, sizeof(grp_t), grp_cmp);
    long k = 0;
    for (long i = 0; i < m; ) {
        long j = i;
        cplx w = 0;
        while (j < m && all[j].key == all[i].key) w += all[j++].w;
        if (w != 0) { all[k].key = all[i].key; all[k].w = w; ++k; }
        i = j;
    }
    *out = all;
    return k;
}

long oracle_source_group_count(int32_t A, int32_t K, const int32_t *flav, const int32_t *nw,
                               const int32_t *woff, const int32_t *wj, const double *wre,
                               const double *wim, int32_t n_src, const int32_t *src_kind,
                               const double *src_c, int32_t n_u)
{
    kinds_t ks = {K, flav, nw, woff, wj, wre, wim};
    grp_t *gr;
    long ng = source_groups(&ks, A, n_src, src_kind, src_c, n_u, &gr);
    free(gr);
    return ng;
}

void oracle_sum_dp(int32_t A, const double *B_,
                   int32_t K, const int32_t *flav, const int32_t *nw, const int32_t *woff,
                   const int32_t *wj, const double *wre, const double *wim,
                   int32_t n_snk, const int32_t *snk_kind, const double *snk_c,
                   int32_t n_src, const int32_t *src_kind, const double *src_c,
                   double *out)
{
    const cplx *B = (const cplx *)B_;
    kinds_t ks = {K, flav, nw, woff, wj, wre, wim};
    const int n = 3 * A;
    int f0[48], nu = 0;
    listing(&ks, A, snk_kind, f0);
    for (int q = 0; q < n; ++q) nu += f0[q] == 0;
    grp_t *gr;
    long ng = source_groups(&ks, A, n_src, src_kind, src_c, nu, &gr);
    const long nstate = 1L << n;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    acc_t *part = calloc(nth, sizeof(acc_t));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        cplx *cur = malloc(sizeof(cplx) * nstate), *nxt = malloc(sizeof(cplx) * nstate);
        uint8_t *live = malloc(nstate), *nlive = malloc(nstate);
#pragma omp for schedule(dynamic)
        for (long gi = 0; gi < ng; ++gi) {
            int val[48];
            uint64_t key = gr[gi].key;
            for (int p = n - 1; p >= 0; --p) { val[p] = key & 15; key >>= 4; }
            for (int s = 0; s < n_snk; ++s) {
                const int32_t *pk = snk_kind + s * A;
                int f[48], cu = 0;
                listing(&ks, A, pk, f);
                for (int q = 0; q < n; ++q) cu += f[q] == 0;
                if (cu != nu) continue;
                memset(live, 0, nstate);
                cur[0] = 1.0; live[0] = 1;
                for (int a = 0; a < A; ++a) {
                    memset(nlive, 0, nstate);
                    const cplx *Bk = B + (long)pk[a] * 1728;
                    for (long m = 0; m < nstate; ++m) {
                        if (!live[m]) continue;
                        /* choose a canonical position for each of the block's three slots */
                        for (int p1 = 0; p1 < n; ++p1) {
                            if ((m >> p1) & 1) continue;
                            if ((p1 < nu) != (f[3 * a] == 0)) continue;
                            long m1 = m | (1L << p1);
                            int s1 = __builtin_popcountl(m >> p1);
                            for (int p2 = 0; p2 < n; ++p2) {
                                if ((m1 >> p2) & 1) continue;
                                if ((p2 < nu) != (f[3 * a + 1] == 0)) continue;
                                long m2 = m1 | (1L << p2);
                                int s2 = __builtin_popcountl(m1 >> p2);
                                for (int p3 = 0; p3 < n; ++p3) {
                                    if ((m2 >> p3) & 1) continue;
                                    if ((p3 < nu) != (f[3 * a + 2] == 0)) continue;
                                    long m3 = m2 | (1L << p3);
                                    int s3 = __builtin_popcountl(m2 >> p3);
                                    cplx b = Bk[val[p1] * 144 + val[p2] * 12 + val[p3]];
                                    cplx v = cur[m] * b;
                                    if ((s1 + s2 + s3) & 1) v = -v;
                                    if (!nlive[m3]) { nxt[m3] = v; nlive[m3] = 1; }
                                    else nxt[m3] += v;
                                }
                            }
                        }
                    }
                    cplx *tc = cur; cur = nxt; nxt = tc;
                    uint8_t *tl = live; live = nlive; nlive = tl;
                }
                long full = nstate - 1;
                if (live[full]) {
                    cplx cs = snk_c[2 * s] + I * snk_c[2 * s + 1];
                    acc_add(&part[tid], cs * gr[gi].w * cur[full]);
                }
            }
        }
        free(cur); free(nxt); free(live); free(nlive);
    }
    acc_t total = {0, 0, 0, 0};
    for (int t = 0; t < nth; ++t) acc_add(&total, acc_val(&part[t]));
    free(part); free(gr);
    cplx c = acc_val(&total);
    out[0] = creal(c); out[1] = cimag(c);
}

/* ------------------------------------------------------------------------- */
/* Route 4: the list of block-form terms (Eq. 2.6 / App. D with the source    */
/* antisymmetrised as in method A of Sec. 3.3), one entry per canonical slot  */
/* assignment, not merged.                                                    */
/*                                                                            */
/* For every source group (U, D) and sink pattern s, every flavor-preserving  */
/* assignment sigma of the canonical positions to the sink slots is a term    */
/* c_s * W'(U,D) * sgn(sigma) * prod_a Braw_{k_a}[i1, i2, i3]. The assignment */
/* that swaps a nucleon's two same-flavor slots has the opposite sign, so the */
/* 2^A assignments of one class add up to one product of blocks of Eq. 2.4,   */
/* Beq[i1,i2,i3] = Braw[i1,i2,i3] - Braw[i3,i2,i1], taken at the member with  */
/* i1 < i3 in every nucleon. That member is emitted: entries                  */
/* ent[A] = k*1728 + i1*144 + i2*12 + i3 (sink order) and its coefficient.    */
/* With ent == NULL only the count is returned. Kinds must have the same      */
/* flavor in slots 1 and 3.                                                   */
/* ------------------------------------------------------------------------- */
long oracle_term_list(int32_t A, int32_t K, const int32_t *flav, const int32_t *nw, const int32_t *woff,
                      const int32_t *wj, const double *wre, const double *wim,
                      int32_t n_snk, const int32_t *snk_kind, const double *snk_c,
                      int32_t n_src, const int32_t *src_kind, const double *src_c,
                      int32_t *ent, double *coef)
{
    kinds_t ks = {K, flav, nw, woff, wj, wre, wim};
    const int n = 3 * A;
    int f0[48], nu = 0;
    listing(&ks, A, snk_kind, f0);
    for (int q = 0; q < n; ++q) nu += f0[q] == 0;
    grp_t *gr;
    long ng = source_groups(&ks, A, n_src, src_kind, src_c, nu, &gr);
    int gcanon[48];
    for (int p = 0; p < n; ++p) gcanon[p] = p < nu ? 0 : 1;
    long cnt = 0;
    for (int s = 0; s < n_snk; ++s) {
        const int32_t *pk = snk_kind + s * A;
        int f[48], cu = 0;
        listing(&ks, A, pk, f);
        for (int q = 0; q < n; ++q) cu += f[q] == 0;
        if (cu != nu) continue;
        int *sig, *sgn;
        int nsig = bijections(f, gcanon, n, &sig, &sgn);
        cplx cs = snk_c[2 * s] + I * snk_c[2 * s + 1];
        for (long gi = 0; gi < ng; ++gi) {
            int val[48];
            uint64_t key = gr[gi].key;
            for (int p = n - 1; p >= 0; --p) { val[p] = key & 15; key >>= 4; }
            for (int b = 0; b < nsig; ++b) {
                const int *sg = sig + (long)b * n;
                int canon = 1;
                for (int a = 0; a < A && canon; ++a) canon = val[sg[3 * a]] < val[sg[3 * a + 2]];
                if (!canon) continue;
                if (ent) {
                    for (int a = 0; a < A; ++a)
                        ent[cnt * A + a] = pk[a] * 1728 + val[sg[3 * a]] * 144 + val[sg[3 * a + 1]] * 12 +
                                           val[sg[3 * a + 2]];
                    cplx c = cs * gr[gi].w * (double)sgn[b];
                    coef[2 * cnt] = creal(c);
                    coef[2 * cnt + 1] = cimag(c);
                }
                ++cnt;
            }
        }
        free(sig); free(sgn);
    }
    free(gr);
    return cnt;
}

/* The antisymmetrised source groups themselves (method A of Sec. 3.3):
 * canonical index lists (n values each: u's ascending, then d's ascending)
 * and weights W'(U, D). With vals == NULL only the count is returned. */
long oracle_source_groups(int32_t A, int32_t K, const int32_t *flav, const int32_t *nw, const int32_t *woff,
                          const int32_t *wj, const double *wre, const double *wim, int32_t n_src,
                          const int32_t *src_kind, const double *src_c, int32_t n_u, int32_t *vals, double *w)
{
    kinds_t ks = {K, flav, nw, woff, wj, wre, wim};
    grp_t *gr;
    long ng = source_groups(&ks, A, n_src, src_kind, src_c, n_u, &gr);
    const int n = 3 * A;
    if (vals)
        for (long g = 0; g < ng; ++g) {
            uint64_t key = gr[g].key;
            for (int p = n - 1; p >= 0; --p) { vals[g * n + p] = (int32_t)(key & 15); key >>= 4; }
            w[2 * g] = creal(gr[g].w);
            w[2 * g + 1] = cimag(gr[g].w);
        }
    free(gr);
    return ng;
}

/* A flat table evaluated on given blocks, on all threads (the same-table CPU
 * reference): out = sum_n coef_n prod_a B[kidx[a][n]] for each of n_sets
 * block sets of K792 complex entries (kidx[A][N] as uint16, coef [N][2]). */
void oracle_table_sum(int32_t A, int64_t N, const uint16_t *kidx, const double *coef_, int32_t n_sets,
                      int64_t set_len, const double *B_, double *out)
{
    const cplx *coef = (const cplx *)coef_, *B = (const cplx *)B_;
    for (int s = 0; s < n_sets; ++s) {
        const cplx *Bs = B + (int64_t)s * set_len;
        double sr = 0, si = 0;
#pragma omp parallel for reduction(+ : sr, si) schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            cplx p = coef[n];
            for (int a = 0; a < A; ++a) p *= Bs[kidx[(int64_t)a * N + n]];
            sr += creal(p);
            si += cimag(p);
        }
        out[2 * s] = sr;
        out[2 * s + 1] = si;
    }
}

/* Number of OpenMP threads the oracle's parallel loops use. */
int32_t oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
