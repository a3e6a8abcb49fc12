// smalldyn.hip -- interval-Hessian bounds of small analytic systems (one
// thread per unit): the closed-form test dynamics (LINEAR, QUADRATIC,
// SINCOS), the satellite and the 3-D quadrotor of the dynamics appendix,
// each in the three forms the paper compares (section IV.A):
//   PATH     Theorem 1: sum_{j<k} [H_kj](X^(j)) (Delta_j Delta_k)
//                       + 1/2 sum_k [H_kk](X^(k)) Delta_k^2, prefix boxes X^(p)
//   EXPAND   eq. expanded_interval_hessian: the same sum, every entry over X
//   CLASSIC  eq. interval_quadratic_form: 1/2 Delta^T ([H](X) Delta)
// and the random-sampling under-approximation of the remainder (the
// comparison of the tightness study): min and max of r(a; a~) over
// caller-given points of the box.
//
// Arithmetic as in the chain kernel: the displacement intervals and the
// Hessian entries in outward-rounded FP32, every entry times an FP64 point
// factor (dt, a quadratic coefficient), the terms summed in FP64.  Every
// term contains 0 (each has a displacement factor that does), so the FP64
// sums do not cancel and one relative widening covers their rounding.  A
// term whose displacement factor is exactly [0, 0] contributes exactly 0.
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "leb.h"
#include "leb_internal.hpp"
#include "pbh_common.hpp"
#include "pbh_node.hpp"

namespace leb {

constexpr int SD_MAX_N = 64;     // QUADRATIC: nx + nu
constexpr int SD_MAX_CAND = 9;   // structural entries of one row (3-D quadrotor: velocity rows)

struct SmallArgs {
    const double *z, *v, *mu, *sigma, *Q;
    double *r_lo, *r_hi, *c_bar, *rho_bar;
    uint32_t* flags;
    double pad;
    int64_t units;
    int nx, nu, kind;
    double dt, m, J[3];
};

__device__ __forceinline__ double sd_nom(const SmallArgs& A, int64_t u, int i) {
    return i < A.nx ? A.z[u * A.nx + i] : A.v[u * A.nu + (i - A.nx)];
}
__device__ __forceinline__ fiv sd_disp(const SmallArgs& A, int64_t u, int i) {
    const int n = A.nx + A.nu;
    const IV<float> d = disp_interval(A.mu ? A.mu[u * n + i] : 0.0, A.sigma[u * n + i]);
    return mk(d.lo, d.hi);
}
__device__ __forceinline__ bool sd_zero(fiv d) { return d.lo == 0.0f && d.hi == 0.0f; }

// Coordinate i of the prefix box X^(p) (coordinates 0..p free, the rest at
// the nominal), FP64 endpoints rounded outward.
__device__ __forceinline__ void sd_coord(const SmallArgs& A, int64_t u, int i, int p, double* lo, double* hi) {
    const double a = sd_nom(A, u, i);
    if (i > p) { *lo = a; *hi = a; return; }
    const fiv d = sd_disp(A, u, i);
    const double l = a + (double)d.lo, h = a + (double)d.hi;
    *lo = l - fabs(l) * 0x1p-52;
    *hi = h + fabs(h) * 0x1p-52;
}
__device__ __forceinline__ fiv sd_coord32(const SmallArgs& A, int64_t u, int i, int p) {
    double lo, hi;
    sd_coord(A, u, i, p, &lo, &hi);
    return mk(rd32(lo), ru32(hi));
}
__device__ __forceinline__ SinCos sd_trig(const SmallArgs& A, int64_t u, int i, int p) {
    double lo, hi;
    sd_coord(A, u, i, p, &lo, &hi);
    SinCos r;
    isincos(lo, hi, &r);
    return r;
}

// --------------------------------------------------------------- entries
//
// An entry is kappa * H: kappa an FP64 point, H an FP32 interval (unit when
// `unit` is set, so that a point coefficient is applied once, in FP64).
struct Entry {
    fiv H;
    double kappa;
    bool unit;
};

// Satellite: qdot_r = sum over (w_b, q_c) of +-1/2 w_b q_c (zeta carries the
// 1/2); wdot_1 = ... - (I3 - I2)/I1 w2 w3 and cyclically.  a = (q0..q3, w1..w3, v1..v3).
__constant__ signed char kSatQ[4][3][3] = {
    {{1, 1, -1}, {2, 2, -1}, {3, 3, -1}},
    {{1, 0, 1}, {3, 2, 1}, {2, 3, -1}},
    {{2, 0, 1}, {3, 1, -1}, {1, 3, 1}},
    {{3, 0, 1}, {2, 1, 1}, {1, 2, -1}}};

__device__ __forceinline__ double sat_euler(const SmallArgs& A, int r) {    // -(I_b - I_c)/I_a dt, a = r
    const int b = r == 0 ? 2 : (r == 1 ? 0 : 1), c = r == 0 ? 1 : (r == 1 ? 2 : 0);
    return -A.dt * (A.J[b] - A.J[c]) / A.J[r];
}

// 3-D quadrotor: a = (px, py, pz, phi, theta, psi, vx, vy, vz, p, q, r, T, tau x3)
enum { QD_PHI = 3, QD_TH = 4, QD_PSI = 5, QD_P = 9, QD_Q = 10, QD_R = 11, QD_T = 12 };

// The structurally non-zero entries (k, j), k >= j, of row l.
__device__ int sd_candidates(const SmallArgs& A, int l, int* ks, int* js) {
    int c = 0;
    auto put = [&](int k, int j) { ks[c] = k; js[c] = j; ++c; };
    if (A.kind == LEB_DYN_SINCOS) {
        put(0, 0);
        if (A.nx == 2) { put(1, 0); put(1, 1); }
    } else if (A.kind == LEB_DYN_SATELLITE) {
        if (l < 4)
            for (int t = 0; t < 3; ++t) put(3 + kSatQ[l][t][0], kSatQ[l][t][1]);
        else if (l == 4) put(6, 5);
        else if (l == 5) put(6, 4);
        else if (l == 6) put(5, 4);
    } else if (A.kind == LEB_DYN_QUAD3D) {
        if (l >= 3 && l <= 5) {
            put(QD_PHI, QD_PHI); put(QD_Q, QD_PHI); put(QD_R, QD_PHI);
            if (l != 4) { put(QD_TH, QD_PHI); put(QD_TH, QD_TH); put(QD_Q, QD_TH); put(QD_R, QD_TH); }
        } else if (l >= 6 && l <= 8) {
            put(QD_PHI, QD_PHI); put(QD_TH, QD_PHI); put(QD_TH, QD_TH);
            put(QD_T, QD_PHI); put(QD_T, QD_TH);
            if (l != 8) { put(QD_PSI, QD_PHI); put(QD_PSI, QD_TH); put(QD_PSI, QD_PSI); put(QD_T, QD_PSI); }
        } else if (l == 9) put(QD_R, QD_Q);
        else if (l == 10) put(QD_R, QD_P);
        else if (l == 11) put(QD_Q, QD_P);
    }
    return c;
}

// The 3-D quadrotor's entries see phi over its interval (every entry's prefix
// includes phi), theta, psi, q, r, T either at the nominal ([0]) or over their
// intervals ([1]): computed once per unit and row.
struct Q3Cache {
    SinCos phi, th[2], psi[2];
    fiv q[2], r[2], T[2];
};

__device__ void q3_cache(const SmallArgs& A, int64_t u, int l, Q3Cache& C) {
    const int full = A.nx + A.nu - 1;
    if (l < 3 || l > 8) return;
    C.phi = sd_trig(A, u, QD_PHI, full);
    C.th[0] = sd_trig(A, u, QD_TH, QD_TH - 1);
    C.th[1] = sd_trig(A, u, QD_TH, full);
    if (l >= 6) {
        C.psi[0] = sd_trig(A, u, QD_PSI, QD_PSI - 1);
        C.psi[1] = sd_trig(A, u, QD_PSI, full);
    }
#pragma unroll
    for (int b = 0; b < 2; ++b) {
        const int p = b ? full : 0;
        C.q[b] = sd_coord32(A, u, QD_Q, p);
        C.r[b] = sd_coord32(A, u, QD_R, p);
        C.T[b] = sd_coord32(A, u, QD_T, p);
    }
}

// Entry (k, j) of row l over the prefix box X^(p): 1 (written to e), -1 unbounded.
__device__ int sd_entry(const SmallArgs& A, int64_t u, int l, int k, int j, int p, const Q3Cache& C, Entry& e) {
    e.unit = false;
    e.kappa = 1.0;
    if (A.kind == LEB_DYN_SINCOS) {
        // f = sin a1 (1-D); f1 = sin a1 cos a2, f2 = cos a1 sin a2 (2-D)
        const SinCos t0 = sd_trig(A, u, 0, p);
        if (A.nx == 1) { e.H = neg(t0.s); return 1; }
        const SinCos t1 = sd_trig(A, u, 1, p);
        const bool diag = k == j;
        if (l == 0) e.H = neg(diag ? mul(t0.s, t1.c) : mul(t0.c, t1.s));
        else e.H = neg(diag ? mul(t0.c, t1.s) : mul(t0.s, t1.c));
        return 1;
    }
    if (A.kind == LEB_DYN_SATELLITE) {
        e.unit = true;
        e.H = mk(1.0f, 1.0f);
        if (l < 4) {
            for (int t = 0; t < 3; ++t)
                if (k == 3 + kSatQ[l][t][0] && j == kSatQ[l][t][1]) e.kappa = 0.5 * kSatQ[l][t][2] * A.dt;
        } else {
            e.kappa = sat_euler(A, l - 4);
        }
        return 1;
    }
    // LEB_DYN_QUAD3D
    e.kappa = A.dt;
    if (l >= 9) {
        const int i = l - 9;
        const int na = i == 0 ? 1 : (i == 1 ? 2 : 0), nb = i == 0 ? 2 : (i == 1 ? 0 : 1);
        e.unit = true;
        e.H = mk(1.0f, 1.0f);
        e.kappa = A.dt * (A.J[na] - A.J[nb]) / A.J[i];
        return 1;
    }
    const fiv sf = C.phi.s, cf = C.phi.c;
    if (l <= 5) {
        const fiv q = C.q[p >= QD_Q], r = C.r[p >= QD_R];
        const fiv Aa = add(mul(q, sf), mul(r, cf));          // A = q sin(phi) + r cos(phi)
        const fiv Bb = sub(mul(q, cf), mul(r, sf));          // B = q cos(phi) - r sin(phi)
        if (l == 4) {
            e.H = k == QD_PHI ? neg(Bb) : (k == QD_Q ? neg(sf) : neg(cf));
            return 1;
        }
        const SinCos& tt = C.th[p >= QD_TH];
        if (!(tt.c.lo > 0.0f)) return -1;                    // sec, tan unbounded
        const fiv sec = rcp_pos(tt.c);
        const fiv tn = mul(tt.s, sec);
        const fiv sec2 = mul_nn(sec, sec);
        if (l == 3) {
            if (j == QD_PHI) {
                if (k == QD_PHI) e.H = neg(mul(Aa, tn));
                else if (k == QD_TH) e.H = mul(Bb, sec2);
                else if (k == QD_Q) e.H = mul(cf, tn);
                else e.H = neg(mul(sf, tn));
            } else {
                if (k == QD_TH) e.H = mul(mk(2.0f * Aa.lo, 2.0f * Aa.hi), mul(sec2, tn));
                else if (k == QD_Q) e.H = mul(sf, sec2);
                else e.H = mul(cf, sec2);
            }
        } else {
            const fiv st = mul(sec, tn);
            if (j == QD_PHI) {
                if (k == QD_PHI) e.H = neg(mul(Aa, sec));
                else if (k == QD_TH) e.H = mul(Bb, st);
                else if (k == QD_Q) e.H = mul(cf, sec);
                else e.H = neg(mul(sf, sec));
            } else {
                if (k == QD_TH) e.H = mul(Aa, mul(sec, add(sq(tn), sec2)));
                else if (k == QD_Q) e.H = mul(sf, st);
                else e.H = mul(cf, st);
            }
        }
        return 1;
    }
    // velocity rows: (T/m) R with R = Rx, Ry, Rz
    const SinCos& tt = C.th[p >= QD_TH];
    const SinCos& tp = C.psi[p >= QD_PSI];
    const fiv st = tt.s, ct = tt.c, sp = tp.s, cp = tp.c;
    const int r = l - 6;
    fiv D;
    if (k == QD_T) {                 // (T, b): (1/m) dR/db
        if (r == 0) {
            if (j == QD_PHI) D = sub(mul(sp, cf), mul(mul(cp, st), sf));
            else if (j == QD_TH) D = mul(mul(cp, ct), cf);
            else D = sub(mul(cp, sf), mul(mul(sp, st), cf));
        } else if (r == 1) {
            if (j == QD_PHI) D = neg(add(mul(mul(sp, st), sf), mul(cp, cf)));
            else if (j == QD_TH) D = mul(mul(sp, ct), cf);
            else D = add(mul(mul(cp, st), cf), mul(sp, sf));
        } else {
            D = j == QD_PHI ? neg(mul(ct, sf)) : neg(mul(st, cf));
        }
        e.H = D;
        e.kappa = A.dt / A.m;
        return 1;
    }
    if (r == 0) {
        if (k == QD_PHI) D = neg(add(mul(mul(cp, st), cf), mul(sp, sf)));
        else if (k == QD_TH && j == QD_PHI) D = neg(mul(mul(cp, ct), sf));
        else if (k == QD_TH) D = neg(mul(mul(cp, st), cf));
        else if (j == QD_PHI) D = add(mul(mul(sp, st), sf), mul(cp, cf));
        else if (j == QD_TH) D = neg(mul(mul(sp, ct), cf));
        else D = neg(add(mul(mul(cp, st), cf), mul(sp, sf)));
    } else if (r == 1) {
        if (k == QD_PHI) D = sub(mul(cp, sf), mul(mul(sp, st), cf));
        else if (k == QD_TH && j == QD_PHI) D = neg(mul(mul(sp, ct), sf));
        else if (k == QD_TH) D = neg(mul(mul(sp, st), cf));
        else if (j == QD_PHI) D = sub(mul(sp, cf), mul(mul(cp, st), sf));
        else if (j == QD_TH) D = mul(mul(cp, ct), cf);
        else D = sub(mul(cp, sf), mul(mul(sp, st), cf));
    } else {
        if (k == QD_PHI) D = neg(mul(ct, cf));
        else if (j == QD_PHI) D = mul(st, sf);
        else D = neg(mul(ct, cf));
    }
    e.H = mul(C.T[p >= QD_T], D);
    e.kappa = A.dt / A.m;
    return 1;
}

// kappa * H * P into acc (P contains 0)
__device__ __forceinline__ void sd_acc(div_& acc, const Entry& e, double scale, fiv P) {
    acc_any(acc, scale * e.kappa, e.unit ? P : mul_z(e.H, P));
}

// One thread per (unit, row): the rows of a unit are G consecutive lanes
// (G a power of two >= nx, so a group never straddles a wave); the unit's
// flags are OR-ed over its group.
template <int MODE>
__global__ void __launch_bounds__(256) small_dyn_kernel(SmallArgs A, int G) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t u = q / G;
    const int lane_row = (int)(q - u * G);
    const bool active = u < A.units && lane_row < A.nx;
    const int n = A.nx + A.nu;
    const int full = n - 1;          // X^(n-1) = X
    uint32_t fl = 0, fl_row = 0;
    if (active)
        for (int i = 0; i < n; ++i) {
            const double a = sd_nom(A, u, i), m = A.mu ? A.mu[u * n + i] : 0.0, s = A.sigma[u * n + i];
            if (!isfinite(a) || !isfinite(m) || !isfinite(s) || !(s >= 0.0)) fl |= LEB_FLAG_BAD_INPUT;
            if (fabs(m) > s) fl |= LEB_FLAG_HULL_EXTENDED;
        }
    // LINEAR (G = 1): one thread writes every row of its unit
    const int l_end = A.kind == LEB_DYN_LINEAR ? A.nx : lane_row + 1;
    for (int l = lane_row; active && l < l_end; ++l) {
        div_ vk[MODE == LEB_IH_CLASSIC ? SD_MAX_N : 1];
        div_ acc{0.0, 0.0};
        int terms = 0;
        bool unbounded = false;
        if (!(fl & LEB_FLAG_BAD_INPUT) && A.kind != LEB_DYN_LINEAR) {
            if (MODE == LEB_IH_CLASSIC)
                for (int i = 0; i < n; ++i) vk[i] = div_{0.0, 0.0};
            // one entry (k, j), k >= j: the PATH / EXPAND term, or its CLASSIC contributions
            auto visit = [&](int k, int j, const Entry& e) {
                const fiv dk = sd_disp(A, u, k), dj = sd_disp(A, u, j);
                if (MODE == LEB_IH_CLASSIC) {
                    // v = [H] Delta over the symmetric matrix: row k gets H Delta_j, row j gets H Delta_k
                    if (!sd_zero(dj)) { sd_acc(vk[k], e, 1.0, dj); ++terms; }
                    if (k != j && !sd_zero(dk)) { sd_acc(vk[j], e, 1.0, dk); ++terms; }
                } else {
                    if (sd_zero(dk) || sd_zero(dj)) return;
                    if (j < k) sd_acc(acc, e, 1.0, mul_zz(dj, dk));
                    else sd_acc(acc, e, 0.5, sq_z(dk));
                    ++terms;
                }
            };
            if (A.kind == LEB_DYN_QUADRATIC) {
                const double* Ql = A.Q + (size_t)l * n * n;
                for (int k = 0; k < n && !unbounded; ++k)
                    for (int j = 0; j <= k; ++j) {
                        const double qv = Ql[k * n + j];
                        if (!isfinite(qv)) { unbounded = true; break; }
                        if (qv == 0.0) continue;
                        Entry e;
                        e.unit = true; e.H = mk(1.0f, 1.0f); e.kappa = qv;
                        visit(k, j, e);
                    }
            } else {
                Q3Cache C;
                if (A.kind == LEB_DYN_QUAD3D) q3_cache(A, u, l, C);
                int ks[SD_MAX_CAND], js[SD_MAX_CAND];
                const int nc = sd_candidates(A, l, ks, js);
                for (int c = 0; c < nc && !unbounded; ++c) {
                    Entry e;
                    const int p = MODE == LEB_IH_PATH ? js[c] : full;   // prefix of the smaller index
                    if (sd_entry(A, u, l, ks[c], js[c], p, C, e) < 0) { unbounded = true; break; }
                    visit(ks[c], js[c], e);
                }
            }
            if (MODE == LEB_IH_CLASSIC && !unbounded) {
                // 1/2 Delta^T v: both factors contain 0, so each product does too
                for (int i = 0; i < n; ++i) {
                    const fiv d = sd_disp(A, u, i);
                    if (sd_zero(d)) continue;
                    const double p1 = (double)d.lo * vk[i].hi, p2 = (double)d.hi * vk[i].lo;
                    const double p3 = (double)d.lo * vk[i].lo, p4 = (double)d.hi * vk[i].hi;
                    acc.lo += 0.5 * fmin(p1, p2);
                    acc.hi += 0.5 * fmax(p3, p4);
                }
            }
        }
        double lo, hi;
        if (fl & LEB_FLAG_BAD_INPUT) {
            lo = -INFINITY; hi = INFINITY;
        } else if (unbounded) {
            lo = -INFINITY; hi = INFINITY;
            fl_row = LEB_FLAG_UNBOUNDED;
        } else {
            // at most a few thousand same-sign FP64 roundings of 2^-53 each, relative to the sum
            lo = acc.lo - fabs(acc.lo) * 0x1p-40;
            hi = acc.hi + fabs(acc.hi) * 0x1p-40;
            if (terms == 0) { lo = 0.0; hi = 0.0; }
        }
        const int64_t o = u * A.nx + l;
        if (A.r_lo) { A.r_lo[o] = lo; A.r_hi[o] = hi; }
        if (A.c_bar) row_zono(lo, hi, A.pad, &A.c_bar[o], &A.rho_bar[o]);
    }
    // every lane takes part in the exchange; inactive lanes contribute 0
    uint32_t f = fl | fl_row;
    for (int off = 1; off < G; off <<= 1) f |= (uint32_t)__shfl_xor((int)f, off);
    if (active && lane_row == 0 && A.flags) A.flags[u] = f;
}

// --------------------------------------------------- sampled remainder
//
// r_l(a; a~) = N_l(a) - N_l(a~) - grad N_l(a~) . (a - a~), N the non-affine
// part of the dynamics, in FP64; QUADRATIC uses its exact form 1/2 d^T Q_l d.

constexpr int SD_SAMPLE_N = 16;      // nx + nu of the sampled kinds

// value of N_l at a (and, when g is given, its gradient, written to g[0..SD_SAMPLE_N-1])
__device__ __forceinline__ double sd_nonlin(const SmallArgs& A, const double (&a)[SD_SAMPLE_N], int l,
                                            double (*g)[SD_SAMPLE_N]) {
    if (g) {
#pragma unroll
        for (int i = 0; i < SD_SAMPLE_N; ++i) (*g)[i] = 0.0;
    }
    if (A.kind == LEB_DYN_SINCOS) {
        if (A.nx == 1) {
            if (g) (*g)[0] = cos(a[0]);
            return sin(a[0]);
        }
        const double s0 = sin(a[0]), c0 = cos(a[0]), s1 = sin(a[1]), c1 = cos(a[1]);
        if (l == 0) {
            if (g) { (*g)[0] = c0 * c1; (*g)[1] = -s0 * s1; }
            return s0 * c1;
        }
        if (g) { (*g)[0] = -s0 * s1; (*g)[1] = c0 * c1; }
        return c0 * s1;
    }
    if (A.kind == LEB_DYN_SATELLITE) {
        if (l < 4) {
            double val = 0.0;
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int w = 3 + kSatQ[l][t][0], q = kSatQ[l][t][1];
                const double c = 0.5 * kSatQ[l][t][2] * A.dt;
                val += c * a[w] * a[q];
                if (g) { (*g)[w] += c * a[q]; (*g)[q] += c * a[w]; }
            }
            return val;
        }
        const int r = l - 4;
        const int ka = r == 2 ? 5 : 6, kb = r == 0 ? 5 : 4;
        const double c = sat_euler(A, r);
        if (g) { (*g)[ka] = c * a[kb]; (*g)[kb] = c * a[ka]; }
        return c * a[ka] * a[kb];
    }
    // LEB_DYN_QUAD3D
    const double dt = A.dt;
    if (l <= 2) return 0.0;
    if (l >= 9) {
        const int i = l - 9;
        const int na = i == 0 ? 1 : (i == 1 ? 2 : 0), nb = i == 0 ? 2 : (i == 1 ? 0 : 1);
        const int ka = i == 2 ? QD_Q : QD_R, kb = i == 0 ? QD_Q : QD_P;
        const double c = dt * (A.J[na] - A.J[nb]) / A.J[i];
        if (g) { (*g)[ka] = c * a[kb]; (*g)[kb] = c * a[ka]; }
        return c * a[ka] * a[kb];
    }
    const double sf = sin(a[QD_PHI]), cf = cos(a[QD_PHI]), st = sin(a[QD_TH]), ct = cos(a[QD_TH]);
    if (l <= 5) {
        const double q = a[QD_Q], r = a[QD_R];
        const double Aa = q * sf + r * cf, Bb = q * cf - r * sf;
        if (l == 4) {
            if (g) { (*g)[QD_PHI] = -dt * Aa; (*g)[QD_Q] = dt * cf; (*g)[QD_R] = -dt * sf; }
            return dt * Bb;
        }
        if (l == 3) {
            const double tn = st / ct;
            if (g) {
                (*g)[QD_PHI] = dt * Bb * tn; (*g)[QD_TH] = dt * Aa / (ct * ct);
                (*g)[QD_Q] = dt * sf * tn; (*g)[QD_R] = dt * cf * tn;
            }
            return dt * Aa * tn;
        }
        if (g) {
            (*g)[QD_PHI] = dt * Bb / ct; (*g)[QD_TH] = dt * Aa * st / (ct * ct);
            (*g)[QD_Q] = dt * sf / ct; (*g)[QD_R] = dt * cf / ct;
        }
        return dt * Aa / ct;
    }
    const double sp = sin(a[QD_PSI]), cp = cos(a[QD_PSI]);
    double R, Rf, Rt, Rp;
    if (l == 6) {
        R = cp * st * cf + sp * sf;
        Rf = sp * cf - cp * st * sf; Rt = cp * ct * cf; Rp = cp * sf - sp * st * cf;
    } else if (l == 7) {
        R = sp * st * cf - cp * sf;
        Rf = -(sp * st * sf + cp * cf); Rt = sp * ct * cf; Rp = cp * st * cf + sp * sf;
    } else {
        R = ct * cf;
        Rf = -ct * sf; Rt = -st * cf; Rp = 0.0;
    }
    const double c = dt * a[QD_T] / A.m;
    if (g) { (*g)[QD_T] = dt * R / A.m; (*g)[QD_PHI] = c * Rf; (*g)[QD_TH] = c * Rt; (*g)[QD_PSI] = c * Rp; }
    return c * R;
}

// N_l(a) for every row l < nx at once (each trigonometric value computed once)
__device__ __forceinline__ void sd_nonlin_all(const SmallArgs& A, const double (&a)[SD_SAMPLE_N],
                                              double (&N)[SD_SAMPLE_N]) {
#pragma unroll
    for (int l = 0; l < SD_SAMPLE_N; ++l) N[l] = 0.0;
    if (A.kind == LEB_DYN_SINCOS) {
        if (A.nx == 1) { N[0] = sin(a[0]); return; }
        const double s0 = sin(a[0]), c0 = cos(a[0]), s1 = sin(a[1]), c1 = cos(a[1]);
        N[0] = s0 * c1;
        N[1] = c0 * s1;
        return;
    }
    if (A.kind == LEB_DYN_SATELLITE) {
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
            for (int t = 0; t < 3; ++t)
                N[l] += 0.5 * kSatQ[l][t][2] * A.dt * a[3 + kSatQ[l][t][0]] * a[kSatQ[l][t][1]];
        N[4] = sat_euler(A, 0) * a[6] * a[5];
        N[5] = sat_euler(A, 1) * a[6] * a[4];
        N[6] = sat_euler(A, 2) * a[5] * a[4];
        return;
    }
    // LEB_DYN_QUAD3D
    const double dt = A.dt;
    const double sf = sin(a[QD_PHI]), cf = cos(a[QD_PHI]), st = sin(a[QD_TH]), ct = cos(a[QD_TH]);
    const double sp = sin(a[QD_PSI]), cp = cos(a[QD_PSI]);
    const double q = a[QD_Q], r = a[QD_R];
    const double Aa = q * sf + r * cf, Bb = q * cf - r * sf;
    N[3] = dt * Aa * (st / ct);
    N[4] = dt * Bb;
    N[5] = dt * Aa / ct;
    const double c = dt * a[QD_T] / A.m;
    N[6] = c * (cp * st * cf + sp * sf);
    N[7] = c * (sp * st * cf - cp * sf);
    N[8] = c * (ct * cf);
    N[9] = dt * (A.J[1] - A.J[2]) / A.J[0] * a[QD_R] * a[QD_Q];
    N[10] = dt * (A.J[2] - A.J[0]) / A.J[1] * a[QD_R] * a[QD_P];
    N[11] = dt * (A.J[0] - A.J[1]) / A.J[2] * a[QD_Q] * a[QD_P];
}

struct SampleArgs {
    SmallArgs S;
    const double* t;      // [K][n] in [-1, 1]
    int K;
    double *s_lo, *s_hi;  // [units][nx]
};

// One workgroup per unit: the nominal's values and gradients in LDS, each
// thread a stride of the samples with every row's running minimum and
// maximum in registers, combined across the wave and then the four waves.
// The nominal itself counts as a sample (r = 0).
__global__ void __launch_bounds__(256) sample_rem_kernel(SampleArgs P) {
    const SmallArgs& A = P.S;
    const int64_t u = blockIdx.x;
    const int n = A.nx + A.nu, nx = A.nx;
    __shared__ double sf0[SD_SAMPLE_N], sg0[SD_SAMPLE_N][SD_SAMPLE_N];
    __shared__ double wlo[4][SD_SAMPLE_N], whi[4][SD_SAMPLE_N];
    double a0[SD_SAMPLE_N], ctr[SD_SAMPLE_N], sg[SD_SAMPLE_N];
#pragma unroll
    for (int i = 0; i < SD_SAMPLE_N; ++i) {
        a0[i] = i < n ? sd_nom(A, u, i) : 0.0;
        ctr[i] = i < n ? a0[i] + (A.mu ? A.mu[u * n + i] : 0.0) : 0.0;
        sg[i] = i < n ? A.sigma[u * n + i] : 0.0;
    }
    if ((int)threadIdx.x < SD_SAMPLE_N) {
        const int l = threadIdx.x;
        double g[SD_SAMPLE_N];
        double f = 0.0;
        if (l < nx && A.kind != LEB_DYN_QUADRATIC) f = sd_nonlin(A, a0, l, &g);
        else {
#pragma unroll
            for (int i = 0; i < SD_SAMPLE_N; ++i) g[i] = 0.0;
        }
        sf0[l] = f;
#pragma unroll
        for (int i = 0; i < SD_SAMPLE_N; ++i) sg0[l][i] = g[i];
    }
    __syncthreads();
    double lo[SD_SAMPLE_N], hi[SD_SAMPLE_N];
#pragma unroll
    for (int l = 0; l < SD_SAMPLE_N; ++l) { lo[l] = 0.0; hi[l] = 0.0; }
    for (int s = threadIdx.x; s < P.K; s += blockDim.x) {
        double a[SD_SAMPLE_N], d[SD_SAMPLE_N], r[SD_SAMPLE_N];
#pragma unroll
        for (int i = 0; i < SD_SAMPLE_N; ++i) {
            a[i] = i < n ? ctr[i] + P.t[(int64_t)s * n + i] * sg[i] : 0.0;
            d[i] = a[i] - a0[i];
        }
        if (A.kind == LEB_DYN_QUADRATIC) {
            for (int l = 0; l < nx; ++l) {
                const double* Ql = A.Q + (size_t)l * n * n;
                double acc = 0.0;
                for (int k = 0; k < n; ++k) {
                    double row = 0.5 * Ql[k * n + k] * d[k];
                    for (int j = 0; j < k; ++j) row += Ql[k * n + j] * d[j];
                    acc += row * d[k];
                }
                lo[l] = fmin(lo[l], acc);
                hi[l] = fmax(hi[l], acc);
            }
            continue;
        }
        sd_nonlin_all(A, a, r);
#pragma unroll
        for (int l = 0; l < SD_SAMPLE_N; ++l) {
            if (l >= nx) break;
            double lin = 0.0;
#pragma unroll
            for (int i = 0; i < SD_SAMPLE_N; ++i) lin += sg0[l][i] * d[i];
            const double rv = (r[l] - sf0[l]) - lin;
            lo[l] = fmin(lo[l], rv);
            hi[l] = fmax(hi[l], rv);
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int l = 0; l < SD_SAMPLE_N; ++l) {
        double x = lo[l], y = hi[l];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            x = fmin(x, __shfl_xor(x, off));
            y = fmax(y, __shfl_xor(y, off));
        }
        if ((threadIdx.x & 63) == 0) { wlo[w][l] = x; whi[w][l] = y; }
    }
    __syncthreads();
    if ((int)threadIdx.x < nx) {
        const int l = threadIdx.x;
        P.s_lo[u * nx + l] = fmin(fmin(wlo[0][l], wlo[1][l]), fmin(wlo[2][l], wlo[3][l]));
        P.s_hi[u * nx + l] = fmax(fmax(whi[0][l], whi[1][l]), fmax(whi[2][l], whi[3][l]));
    }
}

static SmallArgs small_args(const leb_dynamics* dyn, int64_t units, const double* z, const double* v,
                            const double* mu, const double* sigma) {
    SmallArgs A;
    A.z = z; A.v = v; A.mu = mu; A.sigma = sigma; A.Q = dyn->coeffs;
    A.r_lo = A.r_hi = A.c_bar = A.rho_bar = nullptr;
    A.flags = nullptr; A.pad = 0.0;
    A.units = units; A.nx = dyn->nx; A.nu = dyn->nu; A.kind = dyn->kind;
    A.dt = dyn->dt; A.m = dyn->m;
    for (int i = 0; i < 3; ++i) A.J[i] = dyn->J[i];
    return A;
}

int launch_small_dyn(const leb_dynamics* dyn, int mode, int64_t units, const double* z, const double* v,
                     const double* mu, const double* sigma, double* r_lo, double* r_hi, double* c_bar,
                     double* rho_bar, double pad, uint32_t* flags, hipStream_t s) {
    int G = 1;
    while (G < dyn->nx) G <<= 1;     // nx <= 64 for every kind but LINEAR
    if (G > 64) G = 64;
    if (dyn->kind == LEB_DYN_LINEAR) G = 1;
    const int64_t threads = units * (dyn->kind == LEB_DYN_LINEAR ? 1 : G);
    if ((threads + 255) / 256 > 0x7fffffff) return LEB_EINVAL;
    SmallArgs A = small_args(dyn, units, z, v, mu, sigma);
    A.r_lo = r_lo; A.r_hi = r_hi; A.c_bar = c_bar; A.rho_bar = rho_bar; A.flags = flags; A.pad = pad;
    const dim3 g((unsigned)((threads + 255) / 256)), b(256);
    if (mode == LEB_IH_PATH) hipLaunchKernelGGL(small_dyn_kernel<LEB_IH_PATH>, g, b, 0, s, A, G);
    else if (mode == LEB_IH_EXPAND) hipLaunchKernelGGL(small_dyn_kernel<LEB_IH_EXPAND>, g, b, 0, s, A, G);
    else hipLaunchKernelGGL(small_dyn_kernel<LEB_IH_CLASSIC>, g, b, 0, s, A, G);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}

}  // namespace leb

using namespace leb;

static int small_kind(const leb_dynamics* dyn) {
    return dyn->kind == LEB_DYN_LINEAR || dyn->kind == LEB_DYN_QUADRATIC || dyn->kind == LEB_DYN_SINCOS ||
           dyn->kind == LEB_DYN_SATELLITE || dyn->kind == LEB_DYN_QUAD3D;
}

extern "C" int leb_interval_hessian_bound(const leb_dynamics* dyn, int32_t mode, int32_t batch, int32_t N,
                                          const double* z, const double* v, const double* mu, const double* sigma,
                                          double* r_lo, double* r_hi, uint32_t* flags, void* stream) {
    int rc = check_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (mode != LEB_IH_PATH && mode != LEB_IH_EXPAND && mode != LEB_IH_CLASSIC) return LEB_EINVAL;
    if (!small_kind(dyn)) return LEB_ENOTSUP;
    if (batch < 0 || N < 0) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    const int64_t nx = dyn->nx, nu = dyn->nu;
    if (!r_lo || !r_hi || (nx > 0 && !z) || (nu > 0 && !v) || !sigma) return LEB_EINVAL;
    const void* ptrs[] = {z, v, mu, sigma, r_lo, r_hi};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    if (flags && (reinterpret_cast<uintptr_t>(flags) & 3u)) return LEB_EINVAL;
    if (units * (nx + nu) > ((int64_t)1 << 46)) return LEB_EINVAL;
    return launch_small_dyn(dyn, mode, units, z, v, mu, sigma, r_lo, r_hi, nullptr, nullptr, 0.0, flags,
                            (hipStream_t)stream);
}

extern "C" int leb_sample_remainder(const leb_dynamics* dyn, int32_t batch, int32_t N, const double* z,
                                    const double* v, const double* mu, const double* sigma, int32_t K,
                                    const double* t, double* s_lo, double* s_hi, void* stream) {
    int rc = check_dynamics(dyn);
    if (rc != LEB_OK) return rc;
    if (!small_kind(dyn) || dyn->kind == LEB_DYN_LINEAR || dyn->nx + dyn->nu > SD_SAMPLE_N) return LEB_ENOTSUP;
    if (batch < 0 || N < 0 || K < 0) return LEB_EINVAL;
    const int64_t units = (int64_t)batch * N;
    if (units == 0) return LEB_OK;
    if (units > 0x7fffffff) return LEB_EINVAL;
    if (!z || (dyn->nu > 0 && !v) || !sigma || !s_lo || !s_hi || (K > 0 && !t)) return LEB_EINVAL;
    const void* ptrs[] = {z, v, mu, sigma, t, s_lo, s_hi};
    for (const void* p : ptrs)
        if (p && !aligned8(p)) return LEB_EINVAL;
    SampleArgs P;
    P.S = small_args(dyn, units, z, v, mu, sigma);
    P.t = t; P.K = K; P.s_lo = s_lo; P.s_hi = s_hi;
    hipLaunchKernelGGL(sample_rem_kernel, dim3((unsigned)units), dim3(256), 0, (hipStream_t)stream, P);
    return hipGetLastError() == hipSuccess ? LEB_OK : LEB_EDEVICE;
}
