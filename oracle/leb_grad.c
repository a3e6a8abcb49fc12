/*
 * leb_grad.c -- oracle gradient of the path-based Hessian bound.
 *
 * TEST INFRASTRUCTURE (same rules as leb_oracle.c; shares no code with the
 * GPU library).  The paper differentiates its bounds for gradient-based
 * refinement of the nominal point (section IV.D, Table II) and for the
 * linearization-error penalty (eq. linearization_error_cost_penalty).
 *
 * Target: L = sum_{unit, row} g_hi r_hi + g_lo r_lo, differentiated with
 * respect to z, v, sigma, mu of the exact-arithmetic Theorem 1 formula of
 * leb_oracle.c (same canonical expressions, same prefix boxes; rounding
 * treated as the identity).  Method: forward-mode dual numbers, one input
 * direction at a time, evaluating only the rows that direction reaches.
 *
 * Selections (min/max of candidate products, interval square of an
 * interval containing 0, box clamps, sin/cos extrema) follow the
 * candidates' order lo*lo, lo*hi, hi*lo, hi*hi and take the first on a
 * tie.  The smallest relative gap between a selected and a rejected
 * candidate seen in a unit is reported as its "margin": finite-difference
 * checks are meaningful only where it is well above the step.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double v, d; } dd;
typedef struct { dd lo, hi; } ivd;

typedef struct {
    int32_t kind, nx, nu, n_units;
    double dt, m, g, arm, inertia, k_spring, rest_len;
    const double* Q;
    double J[3];
} orc_dyn;

enum { ORC_CHAIN = 4 };

static dd D(double v, double d) { dd r = {v, d}; return r; }
static dd dadd(dd a, dd b) { return D(a.v + b.v, a.d + b.d); }
static dd dmul(dd a, dd b) { return D(a.v * b.v, a.d * b.v + a.v * b.d); }
static dd dscale(double k, dd a) { return D(k * a.v, k * a.d); }

static void gap(double* margin, double a, double b) {
    double s = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
    if (s == 0.0) return;                         /* both exactly 0: same value, no kink in value */
    double g = fabs(a - b) / s;
    if (g < *margin) *margin = g;
}

/* first-min / first-max over candidates in order */
static dd dmin_n(const dd* c, int n, double* margin) {
    int best = 0;
    for (int i = 1; i < n; ++i) if (c[i].v < c[best].v) best = i;
    for (int i = 0; i < n; ++i) if (i != best && c[i].d != c[best].d) gap(margin, c[i].v, c[best].v);
    return c[best];
}
static dd dmax_n(const dd* c, int n, double* margin) {
    int best = 0;
    for (int i = 1; i < n; ++i) if (c[i].v > c[best].v) best = i;
    for (int i = 0; i < n; ++i) if (i != best && c[i].d != c[best].d) gap(margin, c[i].v, c[best].v);
    return c[best];
}

static ivd I(dd lo, dd hi) { ivd r = {lo, hi}; return r; }
static ivd ipt(dd x) { return I(x, x); }
static ivd iadd(ivd a, ivd b) { return I(dadd(a.lo, b.lo), dadd(a.hi, b.hi)); }
static ivd ineg(ivd a) { return I(dscale(-1.0, a.hi), dscale(-1.0, a.lo)); }
static ivd isub(ivd a, ivd b) { return iadd(a, ineg(b)); }
static ivd imul(ivd a, ivd b, double* mg) {
    dd c[4] = {dmul(a.lo, b.lo), dmul(a.lo, b.hi), dmul(a.hi, b.lo), dmul(a.hi, b.hi)};
    return I(dmin_n(c, 4, mg), dmax_n(c, 4, mg));
}
static ivd iscale(double k, ivd a, double* mg) { return imul(ipt(D(k, 0.0)), a, mg); }
/* distance of x from a kink at 0, relative to a scale */
static void kink(double* margin, double x, double scale) {
    if (scale <= 0.0) return;
    double g = fabs(x) / scale;
    if (g < *margin) *margin = g;
}
static ivd isq(ivd a, double* mg) {
    double w = a.hi.v - a.lo.v;
    /* the branch switches when an endpoint crosses 0: a kink only if it moves */
    if (w > 0.0 && a.lo.d != 0.0) kink(mg, a.lo.v, w);
    if (w > 0.0 && a.hi.d != 0.0) kink(mg, a.hi.v, w);
    if (a.lo.v >= 0) return I(dmul(a.lo, a.lo), dmul(a.hi, a.hi));
    if (a.hi.v <= 0) return I(dmul(a.hi, a.hi), dmul(a.lo, a.lo));
    dd c[2] = {dmul(a.lo, a.lo), dmul(a.hi, a.hi)};
    return I(D(0.0, 0.0), dmax_n(c, 2, mg));
}
static ivd isqrt(ivd a) {
    double s1 = sqrt(a.lo.v), s2 = sqrt(a.hi.v);
    return I(D(s1, a.lo.d / (2.0 * s1)), D(s2, a.hi.d / (2.0 * s2)));
}
static ivd irecip(ivd a) {
    return I(D(1.0 / a.hi.v, -a.hi.d / (a.hi.v * a.hi.v)), D(1.0 / a.lo.v, -a.lo.d / (a.lo.v * a.lo.v)));
}

static const double PI_ = 3.14159265358979323846;

/* distance (relative to 1) from the interval to the nearest point x0 + 2 pi m */
static void crit_gap(double a, double b, double frac, double* mg) {
    double x0 = frac * PI_;
    double m1 = round((a - x0) / (2 * PI_)), m2 = round((b - x0) / (2 * PI_));
    double g1 = fabs(a - (x0 + 2 * PI_ * m1)), g2 = fabs(b - (x0 + 2 * PI_ * m2));
    double g = g1 < g2 ? g1 : g2;
    if (g < *mg) *mg = g;
}
static int contains_crit(double a, double b, double frac) {
    double x0 = frac * PI_;
    double m = ceil((a - x0) / (2 * PI_));
    return x0 + 2 * PI_ * m <= b;
}
static ivd isin(ivd a, double* mg) {
    dd s1 = D(sin(a.lo.v), cos(a.lo.v) * a.lo.d), s2 = D(sin(a.hi.v), cos(a.hi.v) * a.hi.d);
    dd c[2] = {s1, s2};
    dd lo = dmin_n(c, 2, mg), hi = dmax_n(c, 2, mg);
    crit_gap(a.lo.v, a.hi.v, 0.5, mg);
    crit_gap(a.lo.v, a.hi.v, -0.5, mg);
    if (contains_crit(a.lo.v, a.hi.v, 0.5)) hi = D(1.0, 0.0);
    if (contains_crit(a.lo.v, a.hi.v, -0.5)) lo = D(-1.0, 0.0);
    return I(lo, hi);
}
static ivd icos(ivd a, double* mg) {
    dd c1 = D(cos(a.lo.v), -sin(a.lo.v) * a.lo.d), c2 = D(cos(a.hi.v), -sin(a.hi.v) * a.hi.d);
    dd c[2] = {c1, c2};
    dd lo = dmin_n(c, 2, mg), hi = dmax_n(c, 2, mg);
    crit_gap(a.lo.v, a.hi.v, 0.0, mg);
    crit_gap(a.lo.v, a.hi.v, 1.0, mg);
    if (contains_crit(a.lo.v, a.hi.v, 0.0)) hi = D(1.0, 0.0);
    if (contains_crit(a.lo.v, a.hi.v, 1.0)) lo = D(-1.0, 0.0);
    return I(lo, hi);
}

/* ----------------------------------------------------- chain dynamics */

static int c_px(int i) { return 6 * i; }
static int c_pz(int i) { return 6 * i + 1; }
static int c_th(int i) { return 6 * i + 2; }
static int c_u(const orc_dyn* d, int i, int a) { return d->nx + 2 * i + a; }
static int node_of_pos(int k, int U) { return (k < 6 * U && (k % 6) < 2) ? k / 6 : -1; }

/* G of leb_oracle.c (same expressions), dual version */
static ivd spring_hess(const orc_dyn* d, int comp, int a, int b, ivd dx, ivd dz, double* mg) {
    double kL = d->k_spring * d->rest_len;
    ivd a2 = isq(dx, mg), b2 = isq(dz, mg);
    ivd s2 = iadd(a2, b2);
    ivd r = isqrt(s2);
    ivd q = irecip(imul(isq(s2, mg), r, mg));
    int nz = (a == 1) + (b == 1);
    ivd two_a = iscale(2.0, a2, mg), two_b = iscale(2.0, b2, mg);
    if (comp == 0) {
        if (nz == 0) return imul(imul(iscale(3.0 * kL, dx, mg), b2, mg), q, mg);
        if (nz == 1) return imul(imul(iscale(-kL, dz, mg), isub(two_a, b2), mg), q, mg);
        return imul(imul(iscale(kL, dx, mg), isub(a2, two_b), mg), q, mg);
    }
    if (nz == 2) return imul(imul(iscale(3.0 * kL, dz, mg), a2, mg), q, mg);
    if (nz == 1) return imul(imul(iscale(-kL, dx, mg), isub(two_b, a2), mg), q, mg);
    return imul(imul(iscale(kL, dz, mg), isub(b2, two_a), mg), q, mg);
}

/* entry (k >= j) of row l over box X; returns 0 for a structural zero */
static int chain_entry(const orc_dyn* d, int l, int k, int j, const ivd* X, ivd* out, double* mg) {
    int U = d->n_units, nx = d->nx;
    if (l >= nx) return 0;
    int i = l / 6, rc = l % 6;
    if (rc != 3 && rc != 4) return 0;
    int comp = rc - 3;
    double c = d->dt / d->m;
    int th = c_th(i), u1 = c_u(d, i, 0), u2 = c_u(d, i, 1);
    if ((k == th || k == u1 || k == u2) && j == th) {
        ivd Th = X[th];
        if (k == th) {
            ivd S = iadd(X[u1], X[u2]);
            if (comp == 0) *out = imul(iscale(c, S, mg), isin(Th, mg), mg);
            else *out = imul(iscale(-c, S, mg), icos(Th, mg), mg);
        } else {
            if (comp == 0) *out = iscale(-c, icos(Th, mg), mg);
            else *out = iscale(-c, isin(Th, mg), mg);
        }
        return 1;
    }
    int nk = node_of_pos(k, U), nj = node_of_pos(j, U);
    if (nk < 0 || nj < 0) return 0;
    int found = 0;
    ivd acc;
    for (int s = i - 1; s <= i; ++s) {
        if (s < 0 || s + 1 >= U) continue;
        if (!((nk == s || nk == s + 1) && (nj == s || nj == s + 1))) continue;
        ivd dx = iadd(isub(ipt(D(d->rest_len, 0.0)), X[c_px(s)]), X[c_px(s + 1)]);
        ivd dz = isub(X[c_pz(s + 1)], X[c_pz(s)]);
        int ak = (k % 6 == 1), aj = (j % 6 == 1);
        ivd G = spring_hess(d, comp, ak, aj, dx, dz, mg);
        double sk = (nk == s) ? -1.0 : 1.0, sj = (nj == s) ? -1.0 : 1.0;
        double row = (i == s) ? 1.0 : -1.0;
        ivd t = iscale(row * sk * sj * c, G, mg);
        acc = found ? iadd(acc, t) : t;
        found = 1;
    }
    if (!found) return 0;
    *out = acc;
    return 1;
}

/* Dual bound of one row: PBH sum over the row's candidate entries */
static ivd row_bound(const orc_dyn* d, int l, const dd* nom, const ivd* Dl, const ivd* X, int n, double* mg,
                     ivd* P) {
    int U = d->n_units, i = l / 6;
    int co[16], nc = 0;
    co[nc++] = c_th(i); co[nc++] = c_u(d, i, 0); co[nc++] = c_u(d, i, 1);
    for (int m = i - 1; m <= i + 1; ++m)
        if (m >= 0 && m < U) { co[nc++] = c_px(m); co[nc++] = c_pz(m); }
    ivd R = ipt(D(0.0, 0.0));
    for (int a = 0; a < nc; ++a)
        for (int b = 0; b < nc; ++b) {
            int k = co[a], j = co[b];
            if (k < j) continue;
            for (int q = 0; q < n; ++q) P[q] = (q <= j) ? X[q] : ipt(nom[q]);
            ivd H;
            if (!chain_entry(d, l, k, j, P, &H, mg)) continue;
            ivd T;
            if (k == j) T = imul(iscale(0.5, H, mg), isq(Dl[k], mg), mg);
            else T = imul(H, imul(Dl[j], Dl[k], mg), mg);
            R = iadd(R, T);
        }
    return R;
}

/* rows reached by coordinate c (chain): nonlinear rows of nearby nodes */
static int rows_of(const orc_dyn* d, int c, int* rows) {
    int U = d->n_units, cnt = 0;
    int node, lo, hi;
    if (c < d->nx) {
        node = c / 6;
        int t = c % 6;
        if (t == 2) { lo = hi = node; }
        else if (t < 2) { lo = node - 1; hi = node + 1; }
        else return 0;
    } else {
        node = (c - d->nx) / 2;
        lo = hi = node;
    }
    for (int m = lo; m <= hi; ++m)
        if (m >= 0 && m < U) { rows[cnt++] = 6 * m + 3; rows[cnt++] = 6 * m + 4; }
    return cnt;
}

#define MAXN 2048

/* Gradient of L with respect to z, v, sigma, mu (gmu may be NULL).
 * g_lo, g_hi [units][nx]; margin [units] (nullable). Rows whose bound is
 * not finite are skipped (contribute nothing). */
int orc_leb_grad(const orc_dyn* d, long units, const double* z, const double* v, const double* mu,
                 const double* sigma, const double* g_lo, const double* g_hi, double* gz, double* gv,
                 double* gmu, double* gsigma, double* margin, int nthreads) {
    if (!d || d->kind != ORC_CHAIN) return -1;
    int n = d->nx + d->nu;
    if (n > MAXN) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (long u = 0; u < units; ++u) {
        double nomv[MAXN], m_[MAXN], s_[MAXN];
        dd* nom = (dd*)malloc(sizeof(dd) * n);
        ivd* Dl = (ivd*)malloc(sizeof(ivd) * n);
        ivd* X = (ivd*)malloc(sizeof(ivd) * n);
        ivd* P = (ivd*)malloc(sizeof(ivd) * n);
        double mg = INFINITY;
        for (int q = 0; q < d->nx; ++q) nomv[q] = z[u * d->nx + q];
        for (int q = 0; q < d->nu; ++q) nomv[d->nx + q] = v[u * d->nu + q];
        for (int q = 0; q < n; ++q) { m_[q] = mu ? mu[u * n + q] : 0.0; s_[q] = sigma[u * n + q]; }
        for (int dir = 0; dir < 3 * n; ++dir) {
            int c = dir % n, kind = dir / n;           /* 0 nominal, 1 sigma, 2 mu */
            if (kind == 2 && !gmu) continue;
            for (int q = 0; q < n; ++q) {
                double t_nom = (kind == 0 && q == c) ? 1.0 : 0.0;
                double t_s = (kind == 1 && q == c) ? 1.0 : 0.0;
                double t_m = (kind == 2 && q == c) ? 1.0 : 0.0;
                nom[q] = D(nomv[q], t_nom);
                /* Delta_lo = min(mu - sigma, 0), Delta_hi = max(mu + sigma, 0): first candidate on a tie */
                double a = m_[q] - s_[q], b = m_[q] + s_[q];
                if (q == c && kind > 0) { kink(&mg, a, s_[q] + fabs(m_[q])); kink(&mg, b, s_[q] + fabs(m_[q])); }
                dd lo = a <= 0.0 ? D(a, t_m - t_s) : D(0.0, 0.0);
                dd hi = b >= 0.0 ? D(b, t_m + t_s) : D(0.0, 0.0);
                Dl[q] = I(lo, hi);
                X[q] = I(dadd(nom[q], lo), dadd(nom[q], hi));
            }
            int rows[8];
            int nr = rows_of(d, c, rows);
            double acc = 0.0;
            for (int r = 0; r < nr; ++r) {
                int l = rows[r];
                ivd R = row_bound(d, l, nom, Dl, X, n, &mg, P);
                if (!isfinite(R.lo.v) || !isfinite(R.hi.v)) continue;
                acc += g_lo[u * d->nx + l] * R.lo.d + g_hi[u * d->nx + l] * R.hi.d;
            }
            if (kind == 0) {
                if (c < d->nx) gz[u * d->nx + c] = acc;
                else gv[u * d->nu + c - d->nx] = acc;
            } else if (kind == 1) gsigma[u * n + c] = acc;
            else gmu[u * n + c] = acc;
        }
        if (margin) margin[u] = mg;
        free(nom); free(Dl); free(X); free(P);
    }
    return 0;
}
