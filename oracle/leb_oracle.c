/*
 * leb_oracle.c -- plain, slow FP64 CPU oracle for linearization-error bounds.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant with the GPU library; both take their inputs
 * from the seeded generators.
 *
 * What it computes (paper: "GPU-Parallel Linearization Error Bounds ...",
 * section IV.A):
 *   - the path-based Hessian (PBH) enclosure of Theorem 1 (eq.
 *     path_based_hessian): for output l,
 *       R_l = sum_{j<k} [H_l,kj](X^(j)) (Delta_j . Delta_k)
 *           + 1/2 sum_k [H_l,kk](X^(k)) Delta_k^2,
 *     with prefix boxes X^(p) (coordinates 1..p free, the rest pinned at
 *     the nominal point), section IV.A "coordinate-wise path";
 *   - the expanded interval Hessian (eq. expanded_interval_hessian): the
 *     same sum with every entry over the full box X;
 *   - the classic interval quadratic form (eq. interval_quadratic_form):
 *     1/2 Delta^T [H](X) Delta, evaluated as [H] Delta first, then the
 *     interval dot product with Delta;
 *   - the true remainder r(a; a~) = f(a) - f(a~) - J(a~)(a - a~)
 *     (eq. linear_error_def) at sample points, for violation checks.
 *
 * Arithmetic: every +, -, *, /, sqrt is rounded to the enclosing FP64
 * number in the needed direction (exactly, via error-free transformations),
 * so exact results stay exact.  sin and cos come from the C library and
 * are widened by 4 ulps, above the library's documented 1-ulp bound.
 *
 * Readings where the paper leaves a choice (listed in the design notes):
 *   - coordinate order alpha = [x; u]; chains stack node blocks;
 *   - box X = hull({a~} U [a~+mu-sigma, a~+mu+sigma]) so that a~ is in X
 *     (Theorem 1 needs a~ in X); Delta = X - a~;
 *   - Delta_k^2 is the interval square (never negative);
 *   - terms are [H] (Delta_j Delta_k): the Delta product first;
 *   - several contributions to one Hessian entry are summed as intervals
 *     before the product with the Delta product;
 *   - an entry whose enclosure needs division by an interval containing 0
 *     makes its output row [-inf, +inf] and sets the UNBOUNDED flag;
 *   - a non-finite input or a negative radius is invalid: every row of the
 *     unit becomes [-inf, +inf] and the BAD_INPUT flag is set.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- types */

typedef struct { double lo, hi; } iv;

enum { ORC_LINEAR = 0, ORC_QUADRATIC = 1, ORC_SIN1D = 2, ORC_SINCOS2D = 3, ORC_CHAIN = 4, ORC_SATELLITE = 5,
       ORC_QUAD3D = 6 };
enum { ORC_PATH = 0, ORC_EXPAND = 1, ORC_CLASSIC = 2 };
enum { ORC_FLAG_UNBOUNDED = 1u, ORC_FLAG_BAD_INPUT = 2u, ORC_FLAG_HULL = 4u };

typedef struct {
    int32_t kind;          /* ORC_* */
    int32_t nx, nu;        /* state and input sizes */
    int32_t n_units;       /* chain: number of planar quadrotors */
    double dt, m, g, arm, inertia, k_spring, rest_len;
    const double* Q;       /* quadratic: [nx][n][n] symmetric Hessians */
    double J[3];           /* satellite: inertia diag(I_S); 3-D quadrotor: Jx, Jy, Jz */
} orc_dyn;

/* ------------------------------------------------ directed FP64 rounding */

static double dn(double x) { return nextafter(x, -INFINITY); }
static double up(double x) { return nextafter(x, INFINITY); }

/* a + b rounded down / up: TwoSum gives the exact error of the RN sum. */
static double add_rd(double a, double b) {
    double s = a + b;
    if (!isfinite(s)) return s;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return e < 0 ? dn(s) : s;
}
static double add_ru(double a, double b) {
    double s = a + b;
    if (!isfinite(s)) return s;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return e > 0 ? up(s) : s;
}
/* a * b rounded down / up: fma gives the exact error; below 2^-960 the
 * error may be lost to underflow, so step outward unconditionally. */
static double mul_rd(double a, double b) {
    if (a == 0.0 || b == 0.0) return 0.0;
    double p = a * b;
    if (!isfinite(p)) return p;
    if (fabs(p) < 0x1p-960) return dn(p);
    double e = fma(a, b, -p);
    return e < 0 ? dn(p) : p;
}
static double mul_ru(double a, double b) {
    if (a == 0.0 || b == 0.0) return 0.0;
    double p = a * b;
    if (!isfinite(p)) return p;
    if (fabs(p) < 0x1p-960) return up(p);
    double e = fma(a, b, -p);
    return e > 0 ? up(p) : p;
}
/* a / b (b != 0): the remainder a - q b is exact; its sign over b's sign
 * tells on which side of q the true quotient lies.  Quotients below 2^-960
 * (possibly underflowed) step outward unconditionally. */
static double div_rd(double a, double b) {
    double q = a / b;
    if (a == 0.0 || !isfinite(q)) return q;
    if (fabs(q) < 0x1p-960) return dn(q);
    double r = fma(-q, b, a);
    return (r != 0 && ((r < 0) != (b < 0))) ? dn(q) : q;
}
static double div_ru(double a, double b) {
    double q = a / b;
    if (a == 0.0 || !isfinite(q)) return q;
    if (fabs(q) < 0x1p-960) return up(q);
    double r = fma(-q, b, a);
    return (r != 0 && ((r < 0) == (b < 0))) ? up(q) : q;
}
static double sqrt_rd(double x) { double s = sqrt(x); return fma(-s, s, x) < 0 ? dn(s) : s; }
static double sqrt_ru(double x) { double s = sqrt(x); return fma(-s, s, x) > 0 ? up(s) : s; }

/* ------------------------------------------------------------- intervals */

static iv ipt(double x) { iv r = {x, x}; return r; }
static iv imk(double lo, double hi) { iv r = {lo, hi}; return r; }
static iv iadd(iv a, iv b) { return imk(add_rd(a.lo, b.lo), add_ru(a.hi, b.hi)); }
static iv ineg(iv a) { return imk(-a.hi, -a.lo); }
static iv isub(iv a, iv b) { return iadd(a, ineg(b)); }
static double min4(double a, double b, double c, double d) { double x = a < b ? a : b, y = c < d ? c : d; return x < y ? x : y; }
static double max4(double a, double b, double c, double d) { double x = a > b ? a : b, y = c > d ? c : d; return x > y ? x : y; }
/* set product {x*y : x in a, y in b} (notation section: Delta . Delta^) */
static iv imul(iv a, iv b) {
    return imk(min4(mul_rd(a.lo, b.lo), mul_rd(a.lo, b.hi), mul_rd(a.hi, b.lo), mul_rd(a.hi, b.hi)),
               max4(mul_ru(a.lo, b.lo), mul_ru(a.lo, b.hi), mul_ru(a.hi, b.lo), mul_ru(a.hi, b.hi)));
}
static iv iscale(double k, iv a) { return imul(ipt(k), a); }
/* interval square: the range of x^2, never negative */
static iv isq(iv a) {
    if (a.lo >= 0) return imk(mul_rd(a.lo, a.lo), mul_ru(a.hi, a.hi));
    if (a.hi <= 0) return imk(mul_rd(a.hi, a.hi), mul_ru(a.lo, a.lo));
    double m = -a.lo > a.hi ? -a.lo : a.hi;
    return imk(0.0, mul_ru(m, m));
}
static iv isqrt(iv a) { return imk(sqrt_rd(a.lo), sqrt_ru(a.hi)); }      /* a.lo >= 0 */
static iv irecip(iv a) { return imk(div_rd(1.0, a.hi), div_ru(1.0, a.lo)); } /* a.lo > 0 */

/* pi enclosure: M_PI is the FP64 number just below pi */
static const double PI_LO = 3.141592653589793115997963468544185161590576171875;
static const double PI_HI = 3.141592653589793560087173318606801331043243408203125;

static double wide_dn(double x, int k) { while (k--) x = dn(x); return x; }
static double wide_up(double x, int k) { while (k--) x = up(x); return x; }

/* may the interval a contain x0 + 2 pi m for some integer m?  x0 = frac * pi
 * (frac in {0, 1/2, 1, -1/2}); computed with an outward pi enclosure so the
 * answer errs towards "yes". */
static int may_contain_critical(iv a, double frac) {
    iv pi = imk(PI_LO, PI_HI);
    iv x0 = iscale(frac, pi);
    iv twopi = iscale(2.0, pi);
    iv t_lo = isub(ipt(a.lo), x0);
    iv t_hi = isub(ipt(a.hi), x0);
    /* smallest possible (a.lo - x0)/2pi and largest possible (a.hi - x0)/2pi */
    double lo = t_lo.lo >= 0 ? div_rd(t_lo.lo, twopi.hi) : div_rd(t_lo.lo, twopi.lo);
    double hi = t_hi.hi >= 0 ? div_ru(t_hi.hi, twopi.lo) : div_ru(t_hi.hi, twopi.hi);
    return floor(hi) >= ceil(lo);
}

/* interval sine / cosine: hull of the endpoint values (each widened by 4
 * ulps), plus +1 / -1 whenever a maximum / minimum may lie inside. */
static iv isin(iv a) {
    if (a.hi - a.lo >= 2.0 * PI_LO) return imk(-1.0, 1.0);
    double s1 = sin(a.lo), s2 = sin(a.hi);
    double lo = wide_dn(s1 < s2 ? s1 : s2, 4), hi = wide_up(s1 > s2 ? s1 : s2, 4);
    if (may_contain_critical(a, 0.5)) hi = 1.0;
    if (may_contain_critical(a, -0.5)) lo = -1.0;
    if (lo < -1.0) lo = -1.0;
    if (hi > 1.0) hi = 1.0;
    return imk(lo, hi);
}
static iv icos(iv a) {
    if (a.hi - a.lo >= 2.0 * PI_LO) return imk(-1.0, 1.0);
    double c1 = cos(a.lo), c2 = cos(a.hi);
    double lo = wide_dn(c1 < c2 ? c1 : c2, 4), hi = wide_up(c1 > c2 ? c1 : c2, 4);
    if (may_contain_critical(a, 0.0)) hi = 1.0;
    if (may_contain_critical(a, 1.0)) lo = -1.0;
    if (lo < -1.0) lo = -1.0;
    if (hi > 1.0) hi = 1.0;
    return imk(lo, hi);
}

/* ------------------------------------------------------------ dynamics */

static int dyn_n(const orc_dyn* d) { return d->nx + d->nu; }

/* chain coordinate indices (0-based) */
static int c_px(int i) { return 6 * i; }
static int c_pz(int i) { return 6 * i + 1; }
static int c_th(int i) { return 6 * i + 2; }
static int c_u(const orc_dyn* d, int i, int a) { return d->nx + 2 * i + a; }
static int node_of_pos(int k, int U) { return (k < 6 * U && (k % 6) < 2) ? k / 6 : -1; }

/* Second derivative of the spring force component `comp` (0: F_x, 1: F_z)
 * with respect to the separation coordinates (a, b in {0: dx, 1: dz}),
 * for the spring force F = k (|d| - L0) d/|d|.  Only -k L0 d/|d| has a
 * non-zero Hessian.  Natural interval extension of:
 *   a2 = dx^2, b2 = dz^2, s2 = a2 + b2, r = sqrt(s2), q = 1/(s2^2 r)
 *   F_x: G_xx = 3kL0 dx b2 q,  G_xz = -kL0 dz (2 a2 - b2) q,  G_zz = kL0 dx (a2 - 2 b2) q
 *   F_z: G_zz = 3kL0 dz a2 q,  G_xz = -kL0 dx (2 b2 - a2) q,  G_xx = kL0 dz (b2 - 2 a2) q
 * Returns 0 when |d| may be 0 (unbounded). */
static int spring_hess(const orc_dyn* d, int comp, int a, int b, iv dx, iv dz, iv* out) {
    double kL = d->k_spring * d->rest_len;
    iv a2 = isq(dx), b2 = isq(dz);
    iv s2 = iadd(a2, b2);
    if (s2.lo <= 0.0) return 0;
    iv r = isqrt(s2);
    iv q = irecip(imul(isq(s2), r));
    int nz = (a == 1) + (b == 1);           /* number of dz derivatives */
    iv g;
    if (comp == 0) {
        if (nz == 0)      g = imul(imul(imul(ipt(3.0 * kL), dx), b2), q);
        else if (nz == 1) g = imul(imul(imul(ipt(-kL), dz), isub(iscale(2.0, a2), b2)), q);
        else              g = imul(imul(imul(ipt(kL), dx), isub(a2, iscale(2.0, b2))), q);
    } else {
        if (nz == 2)      g = imul(imul(imul(ipt(3.0 * kL), dz), a2), q);
        else if (nz == 1) g = imul(imul(imul(ipt(-kL), dx), isub(iscale(2.0, b2), a2)), q);
        else              g = imul(imul(imul(ipt(kL), dz), isub(b2, iscale(2.0, a2))), q);
    }
    *out = g;
    return 1;
}

/* Enclosure of the Hessian entry H_{l,kj} (k >= j) of the chain dynamics
 * over the box X (n intervals; pinned coordinates are points).
 * Returns 0 for a structural zero, 1 for a non-zero entry, -1 when
 * unbounded.  Forward Euler: f = x + dt xdot, so only the velocity rows
 * vx_i, vz_i carry curvature:
 *   vx_i+ : -(dt/m)(u1+u2) sin(theta_i) + (dt/m)(F_x(i,i+1) - F_x(i-1,i))
 *   vz_i+ :  (dt/m)(u1+u2) cos(theta_i) + (dt/m)(F_z(i,i+1) - F_z(i-1,i))
 * The spring (s, s+1) sees d = (L0 + px_{s+1} - px_s, pz_{s+1} - pz_s). */
static int chain_entry(const orc_dyn* d, int l, int k, int j, const iv* X, iv* out) {
    int U = d->n_units, nx = d->nx;
    if (l >= nx) return 0;
    int i = l / 6, rc = l % 6;
    if (rc != 3 && rc != 4) return 0;
    int comp = rc - 3;                      /* 0: vx row, 1: vz row */
    iv c = imk(div_rd(d->dt, d->m), div_ru(d->dt, d->m));
    int th = c_th(i), u1 = c_u(d, i, 0), u2 = c_u(d, i, 1);

    /* attitude / thrust block */
    if ((k == th || k == u1 || k == u2) && j == th) {
        iv Th = X[th];
        if (k == th) {
            iv S = iadd(X[u1], X[u2]);
            if (comp == 0) *out = imul(imul(c, S), isin(Th));                 /*  c S sin */
            else           *out = imul(imul(ineg(c), S), icos(Th));           /* -c S cos */
        } else {
            if (comp == 0) *out = imul(ineg(c), icos(Th));                    /* -c cos */
            else           *out = imul(ineg(c), isin(Th));                    /* -c sin */
        }
        return 1;
    }
    /* spring block: both coordinates are positions */
    int nk = node_of_pos(k, U), nj = node_of_pos(j, U);
    if (nk < 0 || nj < 0) return 0;
    int found = 0;
    iv acc = ipt(0.0);
    for (int s = i - 1; s <= i; ++s) {
        if (s < 0 || s + 1 >= U) continue;
        if (!((nk == s || nk == s + 1) && (nj == s || nj == s + 1))) continue;
        iv dx = iadd(isub(ipt(d->rest_len), X[c_px(s)]), X[c_px(s + 1)]);
        iv dz = isub(X[c_pz(s + 1)], X[c_pz(s)]);
        int ak = (k % 6 == 1), aj = (j % 6 == 1);     /* 0: x, 1: z coordinate */
        iv G;
        if (!spring_hess(d, comp, ak, aj, dx, dz, &G)) return -1;
        double sk = (nk == s) ? -1.0 : 1.0, sj = (nj == s) ? -1.0 : 1.0;
        double row = (i == s) ? 1.0 : -1.0;           /* force on the first node is +F */
        iv coef = iscale(row * sk * sj, c);
        acc = found ? iadd(acc, imul(coef, G)) : imul(coef, G);
        found = 1;
    }
    if (!found) return 0;
    *out = acc;
    return 1;
}

static int quad_entry(const orc_dyn* d, int l, int k, int j, iv* out) {
    int n = dyn_n(d);
    double q = d->Q[((size_t)l * n + k) * n + j];
    if (q == 0.0) return 0;
    *out = ipt(q);
    return 1;
}

/* f = sin(a1) (1-D) ; f1 = sin a1 cos a2, f2 = cos a1 sin a2 (2-D) */
static int sincos_entry(const orc_dyn* d, int l, int k, int j, const iv* X, iv* out) {
    if (d->kind == ORC_SIN1D) { *out = ineg(isin(X[0])); return 1; }
    iv s1 = isin(X[0]), c1 = icos(X[0]), s2 = isin(X[1]), c2 = icos(X[1]);
    if (l == 0) {
        if (k == j) *out = ineg(imul(s1, c2));            /* d11 = d22 = -sin a1 cos a2 */
        else        *out = ineg(imul(c1, s2));            /* d21 = -cos a1 sin a2 */
    } else {
        if (k == j) *out = ineg(imul(c1, s2));            /* d11 = d22 = -cos a1 sin a2 */
        else        *out = ineg(imul(s1, c2));            /* d21 = -sin a1 cos a2 */
    }
    return 1;
}

/* Satellite (appendix, dynamical system definitions): a = (q0..q3, w1..w3,
 * v1..v3), f = x + dt xdot with qdot = zeta(w) q (zeta carries the 1/2) and
 * wdot = I^-1 (v - w x (I w)), I = diag(J).  Every second derivative is a
 * constant: qdot_r is bilinear in (w, q) with coefficients +-1/2, and
 *   wdot_1 = ... - (I3 - I2)/I1 w2 w3,  wdot_2 = ... - (I1 - I3)/I2 w1 w3,
 *   wdot_3 = ... - (I2 - I1)/I3 w1 w2. */
static const signed char SAT_Q[4][3][3] = {          /* row r of qdot: (w index 1..3, q index, sign) */
    {{1, 1, -1}, {2, 2, -1}, {3, 3, -1}},
    {{1, 0, 1}, {3, 2, 1}, {2, 3, -1}},
    {{2, 0, 1}, {3, 1, -1}, {1, 3, 1}},
    {{3, 0, 1}, {2, 1, 1}, {1, 2, -1}}};

static iv sat_euler_coef(const orc_dyn* d, int row) {       /* -(I_b - I_c)/I_a times dt, row = a - 1 */
    static const int B[3] = {2, 0, 1}, C[3] = {1, 2, 0};
    iv num = isub(ipt(d->J[B[row]]), ipt(d->J[C[row]]));
    return imul(ipt(-d->dt), imul(num, irecip(ipt(d->J[row]))));
}

static int sat_entry(const orc_dyn* d, int l, int k, int j, iv* out) {
    if (l < 4) {
        for (int t = 0; t < 3; ++t) {
            int w = 3 + SAT_Q[l][t][0], q = SAT_Q[l][t][1];
            if (k == w && j == q) { *out = ipt(0.5 * SAT_Q[l][t][2] * d->dt); return 1; }
        }
        return 0;
    }
    if (l < 7) {
        static const int K[3] = {6, 6, 5}, Jn[3] = {5, 4, 4};
        if (k == K[l - 4] && j == Jn[l - 4]) { *out = sat_euler_coef(d, l - 4); return 1; }
    }
    return 0;
}

/* 3-D quadrotor (appendix): a = (px, py, pz, phi, theta, psi, vx, vy, vz, p,
 * q, r, T, tau_phi, tau_theta, tau_psi), f = x + dt xdot.  Curvature sits in
 *   phidot   = p + A tan(theta),       A = q sin(phi) + r cos(phi)
 *   thetadot = B,                      B = q cos(phi) - r sin(phi)
 *   psidot   = A sec(theta)
 *   v dot    = (T/m) (Rx, Ry, Rz) - (0, 0, g), with
 *     Rx = cpsi stheta cphi + spsi sphi,  Ry = spsi stheta cphi - cpsi sphi,
 *     Rz = ctheta cphi
 *   pdot = (Jy - Jz)/Jx q r, qdot = (Jz - Jx)/Jy p r, rdot = (Jx - Jy)/Jz p q.
 * Entries (k >= j) are natural interval extensions of the second
 * derivatives written with A and B kept whole, sec = 1/cos(theta),
 * tan = sin(theta) sec (a cos(theta) interval that is not positive makes
 * the entry unbounded); each entry is multiplied by dt. */
enum { Q3_PHI = 3, Q3_TH = 4, Q3_PSI = 5, Q3_P = 9, Q3_Q = 10, Q3_R = 11, Q3_T = 12 };

/* rows phidot, thetadot, psidot: the structurally non-zero entries (k >= j) */
static int q3_att_entry(int l, int k, int j) {
    if (j == Q3_PHI) return k == Q3_PHI || k == Q3_Q || k == Q3_R || (l != 4 && k == Q3_TH);
    if (j == Q3_TH) return l != 4 && (k == Q3_TH || k == Q3_Q || k == Q3_R);
    return 0;
}

static int quad3d_entry(const orc_dyn* d, int l, int k, int j, const iv* X, iv* out) {
    iv H;
    if (l >= 3 && l <= 5) {
        if (!q3_att_entry(l, k, j)) return 0;
        iv sf = isin(X[Q3_PHI]), cf = icos(X[Q3_PHI]);
        iv A = iadd(imul(X[Q3_Q], sf), imul(X[Q3_R], cf));
        iv B = isub(imul(X[Q3_Q], cf), imul(X[Q3_R], sf));
        iv sec = ipt(0.0), tn = ipt(0.0), sec2 = ipt(0.0);
        if (l != 4) {
            iv st = isin(X[Q3_TH]), ct = icos(X[Q3_TH]);
            if (ct.lo <= 0.0) return -1;            /* sec, tan unbounded */
            sec = irecip(ct);
            tn = imul(st, sec);
            sec2 = isq(sec);
        }
        if (l == 3) {
            if (k == Q3_PHI && j == Q3_PHI) H = ineg(imul(A, tn));
            else if (k == Q3_TH && j == Q3_PHI) H = imul(B, sec2);
            else if (k == Q3_Q && j == Q3_PHI) H = imul(cf, tn);
            else if (k == Q3_R && j == Q3_PHI) H = ineg(imul(sf, tn));
            else if (k == Q3_TH) H = imul(iscale(2.0, A), imul(sec2, tn));
            else if (k == Q3_Q) H = imul(sf, sec2);
            else H = imul(cf, sec2);
        } else if (l == 4) {
            if (k == Q3_PHI) H = ineg(B);
            else if (k == Q3_Q) H = ineg(sf);
            else H = ineg(cf);
        } else {
            if (k == Q3_PHI && j == Q3_PHI) H = ineg(imul(A, sec));
            else if (k == Q3_TH && j == Q3_PHI) H = imul(B, imul(sec, tn));
            else if (k == Q3_Q && j == Q3_PHI) H = imul(cf, sec);
            else if (k == Q3_R && j == Q3_PHI) H = ineg(imul(sf, sec));
            else if (k == Q3_TH) H = imul(A, imul(sec, iadd(isq(tn), sec2)));
            else if (k == Q3_Q) H = imul(sf, imul(sec, tn));
            else H = imul(cf, imul(sec, tn));
        }
    } else if (l >= 6 && l <= 8) {
        int a = (k == Q3_PHI || k == Q3_TH || k == Q3_PSI) ? k : (k == Q3_T ? Q3_T : -1);
        int b = (j == Q3_PHI || j == Q3_TH || j == Q3_PSI) ? j : -1;
        if (a < 0 || b < 0) return 0;
        iv sf = isin(X[Q3_PHI]), cf = icos(X[Q3_PHI]);
        iv st = isin(X[Q3_TH]), ct = icos(X[Q3_TH]);
        iv sp = isin(X[Q3_PSI]), cp = icos(X[Q3_PSI]);
        iv im = imk(div_rd(1.0, d->m), div_ru(1.0, d->m));
        iv D;                        /* the derivative of R in (a, b); a = T: the first derivative in b */
        int r = l - 6;               /* 0: Rx, 1: Ry, 2: Rz */
        if (a == Q3_T) {
            if (r == 0) {
                if (b == Q3_PHI) D = isub(imul(sp, cf), imul(imul(cp, st), sf));
                else if (b == Q3_TH) D = imul(imul(cp, ct), cf);
                else D = isub(imul(cp, sf), imul(imul(sp, st), cf));
            } else if (r == 1) {
                if (b == Q3_PHI) D = ineg(iadd(imul(imul(sp, st), sf), imul(cp, cf)));
                else if (b == Q3_TH) D = imul(imul(sp, ct), cf);
                else D = iadd(imul(imul(cp, st), cf), imul(sp, sf));
            } else {
                if (b == Q3_PHI) D = ineg(imul(ct, sf));
                else if (b == Q3_TH) D = ineg(imul(st, cf));
                else return 0;
            }
            H = imul(im, D);
        } else {
            if (r == 0) {
                if (a == Q3_PHI) D = ineg(iadd(imul(imul(cp, st), cf), imul(sp, sf)));          /* (phi, phi) */
                else if (a == Q3_TH && b == Q3_PHI) D = ineg(imul(imul(cp, ct), sf));
                else if (a == Q3_TH) D = ineg(imul(imul(cp, st), cf));                          /* (theta, theta) */
                else if (b == Q3_PHI) D = iadd(imul(imul(sp, st), sf), imul(cp, cf));           /* (psi, phi) */
                else if (b == Q3_TH) D = ineg(imul(imul(sp, ct), cf));                          /* (psi, theta) */
                else D = ineg(iadd(imul(imul(cp, st), cf), imul(sp, sf)));                      /* (psi, psi) */
            } else if (r == 1) {
                if (a == Q3_PHI) D = isub(imul(cp, sf), imul(imul(sp, st), cf));
                else if (a == Q3_TH && b == Q3_PHI) D = ineg(imul(imul(sp, ct), sf));
                else if (a == Q3_TH) D = ineg(imul(imul(sp, st), cf));
                else if (b == Q3_PHI) D = isub(imul(sp, cf), imul(imul(cp, st), sf));
                else if (b == Q3_TH) D = imul(imul(cp, ct), cf);
                else D = isub(imul(cp, sf), imul(imul(sp, st), cf));
            } else {
                if (a == Q3_PHI) D = ineg(imul(ct, cf));
                else if (a == Q3_TH && b == Q3_PHI) D = imul(st, sf);
                else if (a == Q3_TH) D = ineg(imul(ct, cf));
                else return 0;
            }
            H = imul(imul(im, X[Q3_T]), D);
        }
    } else if (l >= 9 && l <= 11) {
        static const int K[3] = {Q3_R, Q3_R, Q3_Q}, Jn[3] = {Q3_Q, Q3_P, Q3_P};
        static const int NA[3] = {1, 2, 0}, NB[3] = {2, 0, 1};
        int i = l - 9;
        if (k != K[i] || j != Jn[i]) return 0;
        H = imul(isub(ipt(d->J[NA[i]]), ipt(d->J[NB[i]])), irecip(ipt(d->J[i])));
    } else {
        return 0;
    }
    *out = imul(ipt(d->dt), H);
    return 1;
}

static int hess_entry(const orc_dyn* d, int l, int k, int j, const iv* X, iv* out) {
    switch (d->kind) {
    case ORC_LINEAR: return 0;
    case ORC_QUADRATIC: return quad_entry(d, l, k, j, out);
    case ORC_SIN1D: case ORC_SINCOS2D: return sincos_entry(d, l, k, j, X, out);
    case ORC_CHAIN: return chain_entry(d, l, k, j, X, out);
    case ORC_SATELLITE: return sat_entry(d, l, k, j, out);
    case ORC_QUAD3D: return quad3d_entry(d, l, k, j, X, out);
    }
    return 0;
}

/* Candidate entries (k >= j) of row l: every pair that the dynamics can
 * couple.  All other entries of the row are structurally zero. */
static int row_candidates(const orc_dyn* d, int l, int* ks, int* js, int cap) {
    int n = dyn_n(d), cnt = 0;
    if (d->kind == ORC_CHAIN) {
        if (l % 6 != 3 && l % 6 != 4) return 0;
        int i = l / 6, U = d->n_units;
        int co[16], nc = 0;
        co[nc++] = c_th(i); co[nc++] = c_u(d, i, 0); co[nc++] = c_u(d, i, 1);
        for (int m = i - 1; m <= i + 1; ++m)
            if (m >= 0 && m < U) { co[nc++] = c_px(m); co[nc++] = c_pz(m); }
        for (int a = 0; a < nc; ++a)
            for (int b = 0; b < nc; ++b)
                if (co[a] >= co[b] && cnt < cap) { ks[cnt] = co[a]; js[cnt] = co[b]; ++cnt; }
        return cnt;
    }
    for (int k = 0; k < n; ++k)
        for (int j = 0; j <= k; ++j)
            if (cnt < cap) { ks[cnt] = k; js[cnt] = j; ++cnt; }
    return cnt;
}

/* ----------------------------------------------------------- one unit */

#define MAXN 4096
#define MAXCAND 4096

/* Box and displacement of one unit: Delta_i = [min(mu_i - sigma_i, 0),
 * max(mu_i + sigma_i, 0)] (the hull with the nominal point, so a~ in X),
 * X_i = a~_i + Delta_i. */
static unsigned unit_box(int n, const double* nom, const double* mu, const double* sg, iv* D, iv* X) {
    unsigned fl = 0;
    for (int i = 0; i < n; ++i) {
        double m = mu ? mu[i] : 0.0;
        if (!isfinite(nom[i]) || !isfinite(m) || !isfinite(sg[i]) || !(sg[i] >= 0.0)) fl |= ORC_FLAG_BAD_INPUT;
        if (fabs(m) > sg[i]) fl |= ORC_FLAG_HULL;
        double lo = add_rd(m, -sg[i]), hi = add_ru(m, sg[i]);
        D[i] = imk(lo < 0 ? lo : 0.0, hi > 0 ? hi : 0.0);
        X[i] = imk(add_rd(nom[i], D[i].lo), add_ru(nom[i], D[i].hi));
    }
    return fl;
}

/* prefix box X^(p): coordinates 0..p free (0-based), the rest at a~ */
static void prefix_box(int n, int p, const double* nom, const iv* X, iv* P) {
    for (int i = 0; i < n; ++i) P[i] = (i <= p) ? X[i] : ipt(nom[i]);
}

static unsigned unit_bound(const orc_dyn* d, int mode, const double* nom, const double* mu,
                           const double* sg, double* lo, double* hi) {
    int n = dyn_n(d);
    iv* D = (iv*)malloc(sizeof(iv) * n);
    iv* X = (iv*)malloc(sizeof(iv) * n);
    iv* P = (iv*)malloc(sizeof(iv) * n);
    int* ks = (int*)malloc(sizeof(int) * MAXCAND);
    int* js = (int*)malloc(sizeof(int) * MAXCAND);
    iv* H = (iv*)malloc(sizeof(iv) * MAXCAND);
    int* nzf = (int*)malloc(sizeof(int) * MAXCAND);
    iv* v = (iv*)malloc(sizeof(iv) * n);
    unsigned fl = unit_box(n, nom, mu, sg, D, X);
    for (int l = 0; l < d->nx; ++l) {
        if (fl & ORC_FLAG_BAD_INPUT) { lo[l] = -INFINITY; hi[l] = INFINITY; continue; }
        int nc = row_candidates(d, l, ks, js, MAXCAND);
        int unbounded = 0;
        for (int c = 0; c < nc; ++c) {
            int k = ks[c], j = js[c];
            if (mode == ORC_PATH) prefix_box(n, j, nom, X, P);   /* j <= k: prefix of the smaller index */
            else memcpy(P, X, sizeof(iv) * n);
            int r = hess_entry(d, l, k, j, P, &H[c]);
            if (r < 0) unbounded = 1;
            nzf[c] = r > 0;
        }
        if (unbounded) { lo[l] = -INFINITY; hi[l] = INFINITY; fl |= ORC_FLAG_UNBOUNDED; continue; }
        iv R = ipt(0.0);
        if (mode == ORC_CLASSIC) {
            /* v = [H](X) Delta over the full symmetric matrix, then 1/2 Delta^T v */
            for (int a = 0; a < n; ++a) v[a] = ipt(0.0);
            int any = 0;
            for (int c = 0; c < nc; ++c) {
                if (!nzf[c]) continue;
                int k = ks[c], j = js[c];
                v[k] = iadd(v[k], imul(H[c], D[j]));
                if (k != j) v[j] = iadd(v[j], imul(H[c], D[k]));
                any = 1;
            }
            if (any) {
                for (int a = 0; a < n; ++a) R = iadd(R, imul(D[a], v[a]));
                R = iscale(0.5, R);
            }
        } else {
            for (int c = 0; c < nc; ++c) {
                if (!nzf[c]) continue;
                int k = ks[c], j = js[c];
                iv T = (k == j) ? imul(iscale(0.5, H[c]), isq(D[k])) : imul(H[c], imul(D[j], D[k]));
                R = iadd(R, T);
            }
        }
        lo[l] = R.lo;
        hi[l] = R.hi;
    }
    free(D); free(X); free(P); free(ks); free(js); free(H); free(nzf); free(v);
    return fl;
}

/* Bounds for `units` independent (nominal, box) units.
 * z [units][nx], v [units][nu], mu (nullable) and sigma [units][n];
 * lo, hi [units][nx]; flags [units] (nullable).  Returns 0, or -1 on bad
 * arguments. */
int orc_leb(const orc_dyn* d, int mode, long units, const double* z, const double* v,
            const double* mu, const double* sigma, double* lo, double* hi, uint32_t* flags,
            int nthreads) {
    int n = dyn_n(d);
    if (!d || n <= 0 || n > MAXN || units < 0 || mode < 0 || mode > 2) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (long u = 0; u < units; ++u) {
        double nom[MAXN];
        for (int i = 0; i < d->nx; ++i) nom[i] = z[u * d->nx + i];
        for (int i = 0; i < d->nu; ++i) nom[d->nx + i] = v[u * d->nu + i];
        unsigned fl = unit_bound(d, mode, nom, mu ? mu + u * n : NULL, sigma + u * n,
                                 lo + u * d->nx, hi + u * d->nx);
        if (flags) flags[u] = fl;
    }
    return 0;
}

/* Single Hessian-entry enclosure over a caller-given box (tests). */
int orc_hess_entry(const orc_dyn* d, int l, int k, int j, const double* box_lo,
                   const double* box_hi, double* out_lo, double* out_hi) {
    int n = dyn_n(d);
    iv X[MAXN];
    for (int i = 0; i < n; ++i) X[i] = imk(box_lo[i], box_hi[i]);
    iv H = ipt(0.0);
    int r = hess_entry(d, l, k, j, X, &H);
    *out_lo = H.lo;
    *out_hi = H.hi;
    return r;
}

int orc_isin(double lo, double hi, double* out) { iv r = isin(imk(lo, hi)); out[0] = r.lo; out[1] = r.hi; return 0; }
int orc_icos(double lo, double hi, double* out) { iv r = icos(imk(lo, hi)); out[0] = r.lo; out[1] = r.hi; return 0; }

/* ------------------------------------------------- true remainder */

/* Nonlinear part N_l of f_l (f = affine + N), its gradient at a point and
 * the sum of magnitudes of its summands (for the rounding allowance). */
static void spring_force(const orc_dyn* d, double dx, double dz, double* F, double* dF) {
    /* F = k (r - L0) d / r ; dF[2*a+b] = dF_a / dd_b */
    double k = d->k_spring, L = d->rest_len;
    double r2 = dx * dx + dz * dz, r = sqrt(r2), r3 = r2 * r;
    F[0] = k * (r - L) * dx / r;
    F[1] = k * (r - L) * dz / r;
    dF[0] = k - k * L * dz * dz / r3;
    dF[1] = k * L * dx * dz / r3;
    dF[2] = k * L * dx * dz / r3;
    dF[3] = k - k * L * dx * dx / r3;
}

/* value, gradient (dense, n) and summand magnitude of N_l at point a */
static void chain_nonlin(const orc_dyn* d, int l, const double* a, double* val, double* grad, double* mag) {
    int n = dyn_n(d), U = d->n_units;
    int i = l / 6, comp = l % 6 - 3;
    double c = d->dt / d->m;
    if (grad) memset(grad, 0, sizeof(double) * n);
    *val = 0.0; *mag = 0.0;
    if (comp != 0 && comp != 1) return;
    double th = a[c_th(i)], S = a[c_u(d, i, 0)] + a[c_u(d, i, 1)];
    double t = comp == 0 ? -c * S * sin(th) : c * S * cos(th);
    *val += t; *mag += fabs(t);
    if (grad) {
        grad[c_th(i)] = comp == 0 ? -c * S * cos(th) : -c * S * sin(th);
        double gu = comp == 0 ? -c * sin(th) : c * cos(th);
        grad[c_u(d, i, 0)] = gu;
        grad[c_u(d, i, 1)] = gu;
    }
    for (int s = i - 1; s <= i; ++s) {
        if (s < 0 || s + 1 >= U) continue;
        double dx = d->rest_len + a[c_px(s + 1)] - a[c_px(s)];
        double dz = a[c_pz(s + 1)] - a[c_pz(s)];
        double F[2], dF[4];
        spring_force(d, dx, dz, F, dF);
        double row = (i == s) ? 1.0 : -1.0;
        double tv = row * c * F[comp];
        *val += tv; *mag += fabs(tv) + fabs(c * d->k_spring * (fabs(dx) + fabs(dz)));
        if (grad) {
            /* dd/dpx_s = (-1,0), dd/dpx_{s+1} = (1,0), same for pz */
            grad[c_px(s)]     += row * c * -dF[comp * 2 + 0];
            grad[c_px(s + 1)] += row * c *  dF[comp * 2 + 0];
            grad[c_pz(s)]     += row * c * -dF[comp * 2 + 1];
            grad[c_pz(s + 1)] += row * c *  dF[comp * 2 + 1];
        }
    }
}

static void test_nonlin(const orc_dyn* d, int l, const double* a, double* val, double* grad, double* mag) {
    int n = dyn_n(d);
    if (grad) memset(grad, 0, sizeof(double) * n);
    *val = 0.0; *mag = 0.0;
    switch (d->kind) {
    case ORC_LINEAR: return;
    case ORC_QUADRATIC: {
        const double* Q = d->Q + (size_t)l * n * n;
        for (int k = 0; k < n; ++k)
            for (int j = 0; j < n; ++j) {
                double t = 0.5 * Q[k * n + j] * a[k] * a[j];
                *val += t; *mag += fabs(t);
                if (grad) grad[k] += Q[k * n + j] * a[j];
            }
        return;
    }
    case ORC_SIN1D:
        *val = sin(a[0]); *mag = fabs(*val);
        if (grad) grad[0] = cos(a[0]);
        return;
    case ORC_SATELLITE:
        if (l < 4) {
            for (int t = 0; t < 3; ++t) {
                int w = 3 + SAT_Q[l][t][0], q = SAT_Q[l][t][1];
                double c = 0.5 * SAT_Q[l][t][2] * d->dt;
                double tv = c * a[w] * a[q];
                *val += tv; *mag += fabs(tv);
                if (grad) { grad[w] += c * a[q]; grad[q] += c * a[w]; }
            }
        } else if (l < 7) {
            static const int K[3] = {6, 6, 5}, Jn[3] = {5, 4, 4}, B[3] = {2, 0, 1}, C[3] = {1, 2, 0};
            int r = l - 4;
            double c = -d->dt * (d->J[B[r]] - d->J[C[r]]) / d->J[r];
            *val = c * a[K[r]] * a[Jn[r]]; *mag = fabs(*val);
            if (grad) { grad[K[r]] = c * a[Jn[r]]; grad[Jn[r]] = c * a[K[r]]; }
        }
        return;
    case ORC_QUAD3D: {
        double dt = d->dt;
        if (l >= 3 && l <= 5) {
            double sf = sin(a[Q3_PHI]), cf = cos(a[Q3_PHI]), st = sin(a[Q3_TH]), ct = cos(a[Q3_TH]);
            double q = a[Q3_Q], r = a[Q3_R];
            double A = q * sf + r * cf, B = q * cf - r * sf, Am = fabs(q * sf) + fabs(r * cf);
            if (l == 4) {
                *val = dt * B; *mag = dt * (fabs(q * cf) + fabs(r * sf));
                if (grad) { grad[Q3_PHI] = -dt * A; grad[Q3_Q] = dt * cf; grad[Q3_R] = -dt * sf; }
            } else if (l == 3) {
                double tn = st / ct;
                *val = dt * A * tn; *mag = dt * Am * fabs(tn);
                if (grad) {
                    grad[Q3_PHI] = dt * B * tn; grad[Q3_TH] = dt * A / (ct * ct);
                    grad[Q3_Q] = dt * sf * tn; grad[Q3_R] = dt * cf * tn;
                }
            } else {
                *val = dt * A / ct; *mag = dt * Am / fabs(ct);
                if (grad) {
                    grad[Q3_PHI] = dt * B / ct; grad[Q3_TH] = dt * A * st / (ct * ct);
                    grad[Q3_Q] = dt * sf / ct; grad[Q3_R] = dt * cf / ct;
                }
            }
        } else if (l >= 6 && l <= 8) {
            double sf = sin(a[Q3_PHI]), cf = cos(a[Q3_PHI]), st = sin(a[Q3_TH]), ct = cos(a[Q3_TH]);
            double sp = sin(a[Q3_PSI]), cp = cos(a[Q3_PSI]);
            double R, Rf, Rt, Rp, Rm;
            if (l == 6) {
                R = cp * st * cf + sp * sf; Rm = fabs(cp * st * cf) + fabs(sp * sf);
                Rf = sp * cf - cp * st * sf; Rt = cp * ct * cf; Rp = cp * sf - sp * st * cf;
            } else if (l == 7) {
                R = sp * st * cf - cp * sf; Rm = fabs(sp * st * cf) + fabs(cp * sf);
                Rf = -(sp * st * sf + cp * cf); Rt = sp * ct * cf; Rp = cp * st * cf + sp * sf;
            } else {
                R = ct * cf; Rm = fabs(R);
                Rf = -ct * sf; Rt = -st * cf; Rp = 0.0;
            }
            double c = dt * a[Q3_T] / d->m;
            *val = c * R; *mag = fabs(c) * Rm;
            if (grad) {
                grad[Q3_T] = dt * R / d->m;
                grad[Q3_PHI] = c * Rf; grad[Q3_TH] = c * Rt; grad[Q3_PSI] = c * Rp;
            }
        } else if (l >= 9 && l <= 11) {
            static const int K[3] = {Q3_R, Q3_R, Q3_Q}, Jn[3] = {Q3_Q, Q3_P, Q3_P};
            static const int NA[3] = {1, 2, 0}, NB[3] = {2, 0, 1};
            int i = l - 9;
            double c = dt * (d->J[NA[i]] - d->J[NB[i]]) / d->J[i];
            *val = c * a[K[i]] * a[Jn[i]]; *mag = fabs(*val);
            if (grad) { grad[K[i]] = c * a[Jn[i]]; grad[Jn[i]] = c * a[K[i]]; }
        }
        return;
    }
    case ORC_SINCOS2D:
        if (l == 0) {
            *val = sin(a[0]) * cos(a[1]);
            if (grad) { grad[0] = cos(a[0]) * cos(a[1]); grad[1] = -sin(a[0]) * sin(a[1]); }
        } else {
            *val = cos(a[0]) * sin(a[1]);
            if (grad) { grad[0] = -sin(a[0]) * sin(a[1]); grad[1] = cos(a[0]) * cos(a[1]); }
        }
        *mag = fabs(*val) + 1.0;
        return;
    }
}

/* r_l(a; a~) = N_l(a) - N_l(a~) - grad N_l(a~) . (a - a~) for samples
 * pts [S][n] of units unit_of [S] with nominals nom [units][n].
 * eps [S][nx] receives a bound on the FP64 evaluation error of r. */
int orc_remainder(const orc_dyn* d, long S, const int64_t* unit_of, const double* nom,
                  const double* pts, double* r, double* eps, int nthreads) {
    int n = dyn_n(d);
    if (n > MAXN) return -1;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
    for (long s = 0; s < S; ++s) {
        const double* a = pts + s * n;
        const double* at = nom + unit_of[s] * n;
        double grad[MAXN];
        for (int l = 0; l < d->nx; ++l) {
            double v1, v0, m1, m0;
            if (d->kind == ORC_CHAIN) {
                if (l % 6 != 3 && l % 6 != 4) { r[s * d->nx + l] = 0.0; eps[s * d->nx + l] = 0.0; continue; }
                chain_nonlin(d, l, a, &v1, NULL, &m1);
                chain_nonlin(d, l, at, &v0, grad, &m0);
            } else {
                test_nonlin(d, l, a, &v1, NULL, &m1);
                test_nonlin(d, l, at, &v0, grad, &m0);
            }
            double lin = 0.0, lm = 0.0;
            for (int k = 0; k < n; ++k) { double t = grad[k] * (a[k] - at[k]); lin += t; lm += fabs(t); }
            r[s * d->nx + l] = (v1 - v0) - lin;
            eps[s * d->nx + l] = 64.0 * 0x1p-53 * (m1 + m0 + lm + fabs(v1) + fabs(v0));
        }
    }
    return 0;
}

/* Nonlinear-part gradient (dense Jacobian rows of N) at one point: for
 * finite-difference pins of the Hessian entries. */
int orc_nonlin(const orc_dyn* d, int l, const double* a, double* val, double* grad) {
    double mag;
    if (d->kind == ORC_CHAIN) chain_nonlin(d, l, a, val, grad, &mag);
    else test_nonlin(d, l, a, val, grad, &mag);
    return 0;
}

/* ------------------------------------------- dynamics and linearization */

/* Affine part of the discretised chain dynamics (explicit Euler, x+ = x +
 * dt xdot): row l of its Jacobian in a = [x; u] is written to row[n] and its
 * constant term returned.  Per node i: px+ = px + dt vx, pz+ = pz + dt vz,
 * theta+ = theta + dt omega, vx+ = vx (+ N), vz+ = vz - dt g (+ N),
 * omega+ = omega + dt (u1 - u2) arm / inertia.  The remaining terms of the
 * velocity rows (thrust and springs) are the nonlinear part N above. */
static double chain_affine_row(const orc_dyn* d, int l, double* row) {
    int n = dyn_n(d), i = l / 6, comp = l % 6;
    memset(row, 0, sizeof(double) * n);
    row[l] = 1.0;
    double cst = 0.0;
    switch (comp) {
    case 0: case 1: case 2: row[6 * i + comp + 3] = d->dt; break;
    case 4: cst = -d->dt * d->g; break;
    case 5: row[c_u(d, i, 0)] = d->dt * d->arm / d->inertia;
            row[c_u(d, i, 1)] = -d->dt * d->arm / d->inertia; break;
    }
    return cst;
}

/* f(x, u) of the discretised dynamics at `units` points: the affine part
 * (chain only; the test kinds have none) plus N.  f [units][nx]. */
int orc_step(const orc_dyn* d, long units, const double* z, const double* v, double* f) {
    int n = dyn_n(d);
    if (n > MAXN || d->kind == ORC_LINEAR) return -1;
    for (long u = 0; u < units; ++u) {
        double a[MAXN], row[MAXN];
        for (int i = 0; i < d->nx; ++i) a[i] = z[u * d->nx + i];
        for (int i = 0; i < d->nu; ++i) a[d->nx + i] = v[u * d->nu + i];
        for (int l = 0; l < d->nx; ++l) {
            double val, mag, aff = 0.0;
            if (d->kind == ORC_CHAIN) {
                aff = chain_affine_row(d, l, row);
                for (int k = 0; k < n; ++k) aff += row[k] * a[k];
                chain_nonlin(d, l, a, &val, NULL, &mag);
            } else {
                test_nonlin(d, l, a, &val, NULL, &mag);
            }
            f[u * d->nx + l] = aff + val;
        }
    }
    return 0;
}

/* Jacobians A = df/dx [units][nx][nx] and B = df/du [units][nx][nu] at the
 * nominal points (eq. linearizations): affine rows plus grad N. */
int orc_jacobian(const orc_dyn* d, long units, const double* z, const double* v, double* A, double* B) {
    int n = dyn_n(d);
    if (n > MAXN || d->kind == ORC_LINEAR) return -1;
    for (long u = 0; u < units; ++u) {
        double a[MAXN], row[MAXN], grad[MAXN];
        for (int i = 0; i < d->nx; ++i) a[i] = z[u * d->nx + i];
        for (int i = 0; i < d->nu; ++i) a[d->nx + i] = v[u * d->nu + i];
        for (int l = 0; l < d->nx; ++l) {
            double val, mag;
            if (d->kind == ORC_CHAIN) {
                chain_affine_row(d, l, row);
                chain_nonlin(d, l, a, &val, grad, &mag);
            } else {
                memset(row, 0, sizeof(double) * n);
                test_nonlin(d, l, a, &val, grad, &mag);
            }
            for (int k = 0; k < d->nx; ++k) A[(u * d->nx + l) * d->nx + k] = row[k] + grad[k];
            for (int k = 0; k < d->nu; ++k) B[(u * d->nx + l) * d->nu + k] = row[d->nx + k] + grad[d->nx + k];
        }
    }
    return 0;
}
