/*
 * crp_oracle.c -- plain FP64 CPU reference for charged-particle propagation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code,
 * header, table or constant with the GPU library: every coefficient and
 * constant below is written here from its published definition.
 *
 * What it computes (paper: "Cosmic ray propagation with CRPropa 3"):
 *   - the 3D mode, in which charged nuclei are deflected by a magnetic field
 *     (section 2), sampled on a regular periodic vector grid (section 3.2);
 *   - one particle at a time, advanced by steps whose length is the lowest
 *     bid among all participants (section 3.1, bidding system): the error
 *     controlled integrator, the step limits, the distance to the observer
 *     sphere and the remaining trajectory length;
 *   - the step is the largest one that keeps the user's accuracy (section 3.1);
 *   - no energy losses, as for galactic propagation (section 3.3);
 *   - propagation ends when it is "completed or aborted" (section 3.1) at an
 *     observer sphere or at a maximum trajectory length.
 *
 * The paper names no integrator, interpolation, error norm or controller.
 * The readings taken (all listed with their reasons in the design notes):
 *   - equation of motion in path length s: dx/ds = u, du/ds = kappa u x B(x),
 *     kappa = Z*K/E, K = c * 1e-13 T/nG * 1 Mpc (positions in Mpc, B in nG,
 *     E in eV; beta = 1, the mass number does not enter);
 *   - Cash-Karp embedded Runge-Kutta 5(4) (Cash & Karp 1990, ACM TOMS 16:201),
 *     propagating the 5th-order solution;
 *   - trilinear interpolation on the periodic grid, x then y then z;
 *   - error = max(|delta_u|, |delta_x|/h) / tol; accept when <= 1 or h <= h_min;
 *   - step controller with safety 0.9, growth <= 5, shrink >= 0.1, exponents
 *     -1/5 (grow) and -1/4 (shrink) (Numerical Recipes section 16.2; Hairer,
 *     Norsett & Wanner II.4);
 *   - event location of the sphere crossing by the Illinois variant of
 *     regula falsi (Dowell & Jarratt 1971) on the Cash-Karp step map, keeping
 *     the bracket end outside the sphere as the crossing point;
 *   - an optional reflective box (section 4 uses reflective boundaries): the
 *     distance to its nearest face bids like the sphere distance, and a step
 *     that ends outside is mirrored on the face (x -> 2 face - x, the
 *     direction component negated) after the sphere test;
 *   - an optional modulation grid (section 3.2, modulated grids) multiplying
 *     the vector grid's value, interpolated the same way;
 *   - backtracking (section 3.3): the input is a particle's state where it
 *     was observed; it is propagated as its antiparticle (charge -Z) with the
 *     direction reversed, and the direction reached is reversed again, so
 *     that input and output directions are the physical particle's.
 *
 * Arithmetic is IEEE FP64, round to nearest even, compiled with
 * -ffp-contract=off; fused multiply-adds appear only where fma() is written.
 * The fifth root in the controller is a fixed Newton iteration rather than
 * pow(), so that the result does not depend on a math library.
 *
 * Parity pins: see the oracle tests (closed-form helix, straight line,
 * affine-field interpolation, order conditions, brute-force integration,
 * invariants, stop semantics; the controller's fixed point, shrink chain and
 * growth cap against 40-digit evaluations of the error estimate for the
 * linear motion in a uniform field; derivatives against forward mode,
 * central differences and closed forms).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants ------------------------------------------------ */
/* K = c * 1e-13 * Mpc_in_m, with c = 299792458 m/s and
 * 1 Mpc = 1e6 * (648000/pi) * 149597870700 m (IAU 2012/2015 definitions).
 * kappa * B = 1/r_gyro for B in nG, E in eV, r in Mpc. */
static const double K_LORENTZ = 9.250628667507923e17;
/* Seconds per Mpc of path at the speed of light: Mpc_in_m / c. */
static const double MPC_OVER_C = 102927125054339.0;

/* ---- Cash-Karp 5(4) tableau ------------------------------------------- */
static const double CK_A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0},
};
static const double CK_C[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
/* fifth-order weights */
static const double CK_B5[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
/* fourth-order weights */
static const double CK_B4[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                                277.0 / 14336.0, 1.0 / 4.0};
/* error weights b5 - b4, each the rounded exact rational difference */
static const double CK_E[6] = {-277.0 / 64512.0, 0.0, 6925.0 / 370944.0, -6925.0 / 202752.0,
                               -277.0 / 14336.0, 277.0 / 7084.0};

/* 2^(-j/5), j = 0..4, rounded to nearest FP64 (checked against mpmath). */
static const double TWO_POW_NEG_FIFTHS[5] = {
    0x1.0000000000000p+0, 0x1.bdb8cdadbe120p-1, 0x1.8406003b2ae5cp-1,
    0x1.51cb453b9536cp-1, 0x1.2611186bae675p-1};

/* status codes of a particle */
enum { ST_ACTIVE = 0, ST_ARRIVED = 1, ST_MAX_LENGTH = 2, ST_MAX_STEPS = 3,
       ST_NONFINITE = 4, ST_CANCELLED = 5, ST_BAD_INPUT = 6 };

/* ---- the periodic vector grid ----------------------------------------- */
/* Optional modulation (section 3.2, modulated grids): a low-resolution scalar
 * grid m, itself periodic over its own extent, that multiplies the vector
 * grid's value: B(x) = b(x) * m(x). */
typedef struct {
    int present;
    int64_t n[3];
    double origin[3];
    double inv_spacing;
    const double *v64;       /* [n0][n1][n2], dimensionless; exactly one of v64/v32 set */
    const float *v32;
} modgrid_t;

typedef struct {
    int64_t n[3];
    double origin[3];
    double inv_spacing;      /* 1.0 / spacing, one FP64 division */
    const double *v64;       /* [n0][n1][n2][3], nG; exactly one of v64/v32 set */
    const float *v32;
    modgrid_t mod;
} grid_t;

static double grid_value(const grid_t *g, int64_t i, int64_t j, int64_t k, int c)
{
    int64_t idx = ((i * g->n[1] + j) * g->n[2] + k) * 3 + c;
    return g->v64 ? g->v64[idx] : (double)g->v32[idx];
}

static int64_t pmod(int64_t a, int64_t n)
{
    int64_t r = a % n;
    return r < 0 ? r + n : r;
}

/* linear interpolation a + t (b - a), one fused multiply-add */
static double lerp(double a, double b, double t) { return fma(t, b - a, a); }

/* Trilinear interpolation of the periodic grid at X (Mpc) -> B (nG).
 * Cell index i0 = floor(f), f = (X - origin) / spacing (as a product with the
 * reciprocal), fraction t = f - floor(f); corners i0 and i0 + 1, wrapped.
 * Interpolate along x first, then y, then z. */
static void field_at(const grid_t *g, const double X[3], double B[3])
{
    int64_t i0[3], i1[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double f = (X[a] - g->origin[a]) * g->inv_spacing;
        if (!(fabs(f) < 4.0e15)) {          /* NaN or absurd position */
            B[0] = B[1] = B[2] = NAN;
            return;
        }
        double fl = floor(f);
        t[a] = f - fl;
        i0[a] = pmod((int64_t)fl, g->n[a]);
        i1[a] = pmod(i0[a] + 1, g->n[a]);
    }
    for (int c = 0; c < 3; ++c) {
        double v000 = grid_value(g, i0[0], i0[1], i0[2], c);
        double v100 = grid_value(g, i1[0], i0[1], i0[2], c);
        double v010 = grid_value(g, i0[0], i1[1], i0[2], c);
        double v110 = grid_value(g, i1[0], i1[1], i0[2], c);
        double v001 = grid_value(g, i0[0], i0[1], i1[2], c);
        double v101 = grid_value(g, i1[0], i0[1], i1[2], c);
        double v011 = grid_value(g, i0[0], i1[1], i1[2], c);
        double v111 = grid_value(g, i1[0], i1[1], i1[2], c);
        double c00 = lerp(v000, v100, t[0]);
        double c10 = lerp(v010, v110, t[0]);
        double c01 = lerp(v001, v101, t[0]);
        double c11 = lerp(v011, v111, t[0]);
        double c0 = lerp(c00, c10, t[1]);
        double c1 = lerp(c01, c11, t[1]);
        B[c] = lerp(c0, c1, t[2]);
    }
}

/* Trilinear interpolation of the periodic modulation grid at X, in the same
 * order as the vector grid (x, then y, then z).  NaN for an absurd position. */
static double mod_at(const modgrid_t *m, const double X[3])
{
    int64_t i0[3], i1[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double f = (X[a] - m->origin[a]) * m->inv_spacing;
        if (!(fabs(f) < 4.0e15))
            return NAN;
        double fl = floor(f);
        t[a] = f - fl;
        i0[a] = pmod((int64_t)fl, m->n[a]);
        i1[a] = pmod(i0[a] + 1, m->n[a]);
    }
#define MODV(i, j, k) (m->v64 ? m->v64[((i) * m->n[1] + (j)) * m->n[2] + (k)] \
                              : (double)m->v32[((i) * m->n[1] + (j)) * m->n[2] + (k)])
    double c00 = lerp(MODV(i0[0], i0[1], i0[2]), MODV(i1[0], i0[1], i0[2]), t[0]);
    double c10 = lerp(MODV(i0[0], i1[1], i0[2]), MODV(i1[0], i1[1], i0[2]), t[0]);
    double c01 = lerp(MODV(i0[0], i0[1], i1[2]), MODV(i1[0], i0[1], i1[2]), t[0]);
    double c11 = lerp(MODV(i0[0], i1[1], i1[2]), MODV(i1[0], i1[1], i1[2]), t[0]);
#undef MODV
    return lerp(lerp(c00, c10, t[1]), lerp(c01, c11, t[1]), t[2]);
}

/* The field at X: the vector grid's value times the modulation, if any. */
static void field_total(const grid_t *g, const double X[3], double B[3])
{
    field_at(g, X, B);
    if (g->mod.present) {
        double m = mod_at(&g->mod, X);
        B[0] = B[0] * m;
        B[1] = B[1] * m;
        B[2] = B[2] * m;
    }
}

/* Right-hand side of the Lorentz-force system in path length:
 * y = (x, u) -> (u, kappa * u x B(x)). */
static void rhs(const grid_t *g, double kappa, const double Y[6], double k[6])
{
    double B[3];
    field_total(g, Y, B);
    k[0] = Y[3];
    k[1] = Y[4];
    k[2] = Y[5];
    double cx = Y[4] * B[2] - Y[5] * B[1];
    double cy = Y[5] * B[0] - Y[3] * B[2];
    double cz = Y[3] * B[1] - Y[4] * B[0];
    k[3] = kappa * cx;
    k[4] = kappa * cy;
    k[5] = kappa * cz;
}

/* One Cash-Karp evaluation of step h from y: the fifth-order solution y5
 * and the embedded error vector delta = h * sum_i (b5_i - b4_i) k_i.
 * Stage sums run over j in increasing order with fma, starting from zero. */
static void ck_eval(const grid_t *g, double kappa, const double y[6], double h,
                    double y5[6], double delta[6])
{
    double k[6][6];
    for (int i = 0; i < 6; ++i) {
        double Y[6];
        for (int c = 0; c < 6; ++c) {
            if (i == 0) {
                Y[c] = y[c];
                continue;
            }
            double acc = 0.0;
            for (int j = 0; j < i; ++j)
                acc = fma(CK_A[i][j], k[j][c], acc);
            Y[c] = fma(h, acc, y[c]);
        }
        rhs(g, kappa, Y, k[i]);
    }
    for (int c = 0; c < 6; ++c) {
        double a5 = 0.0, ae = 0.0;
        for (int i = 0; i < 6; ++i) {
            a5 = fma(CK_B5[i], k[i][c], a5);
            ae = fma(CK_E[i], k[i][c], ae);
        }
        y5[c] = fma(h, a5, y[c]);
        delta[c] = h * ae;
    }
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* err^(-1/5) for finite err > 0 without pow(): err = m 2^e with m in [0.5, 1),
 * e = 5q + j (floor division, j in 0..4); r -> m^(-1/5) by exactly six Newton
 * steps r <- r (6 - m r^5) / 5 on r^-5 - m = 0 from r = 1 (monotone from
 * below); result r * 2^(-j/5) * 2^(-q). */
static double inv_fifth_root(double err)
{
    int e;
    double m = frexp(err, &e);
    int q = e >= 0 ? e / 5 : -((-e + 4) / 5);
    int j = e - 5 * q;
    double r = 1.0;
    for (int it = 0; it < 6; ++it) {
        double r2 = r * r;
        double r5 = (r2 * r2) * r;
        r = r * (6.0 - m * r5) * 0.2;
    }
    return ldexp(r * TWO_POW_NEG_FIFTHS[j], -q);
}

/* ---- propagation parameters ------------------------------------------- */
typedef struct {
    double tol, h_min, h_max;
    double center[3];
    double radius;        /* <= 0: no observer sphere */
    double l_max;         /* +inf: no length limit */
    int64_t max_steps;    /* accepted steps allowed in this call; 0 = no limit */
    int reflect;          /* reflective box on */
    double box_lo[3], box_hi[3];
    int backtrack;        /* propagate the antiparticle backwards */
} params_t;

/* Parameter block: [tol, h_min, h_max, cx, cy, cz, R, l_max, box lo x, y, z,
 * box hi x, y, z, reflect, backtrack].  Returns 0, or -1 for a box that is on
 * with lo >= hi on some axis. */
static int read_params(const double *prm, params_t *p)
{
    p->tol = prm[0];
    p->h_min = prm[1];
    p->h_max = prm[2];
    p->center[0] = prm[3];
    p->center[1] = prm[4];
    p->center[2] = prm[5];
    p->radius = prm[6];
    p->l_max = prm[7];
    for (int a = 0; a < 3; ++a) {
        p->box_lo[a] = prm[8 + a];
        p->box_hi[a] = prm[11 + a];
    }
    p->reflect = prm[14] != 0.0;
    p->backtrack = prm[15] != 0.0;
    if (p->reflect && !(p->box_lo[0] < p->box_hi[0] && p->box_lo[1] < p->box_hi[1] && p->box_lo[2] < p->box_hi[2]))
        return -1;
    return 0;
}

/* Reflective box (the example of section 4 uses reflective boundaries): a
 * particle whose accepted step ends outside the box on an axis is mirrored on
 * that face, position x -> 2 face - x and that direction component negated. */
static void reflect_state(const params_t *p, double y[6])
{
    for (int a = 0; a < 3; ++a) {
        if (y[a] > p->box_hi[a]) {
            y[a] = 2.0 * p->box_hi[a] - y[a];
            y[3 + a] = -y[3 + a];
        } else if (y[a] < p->box_lo[a]) {
            y[a] = 2.0 * p->box_lo[a] - y[a];
            y[3 + a] = -y[3 + a];
        }
    }
}

static double sphere_g(const params_t *p, const double x[3])
{
    double d0 = x[0] - p->center[0], d1 = x[1] - p->center[1], d2 = x[2] - p->center[2];
    return (d0 * d0 + d1 * d1 + d2 * d2) - p->radius * p->radius;
}

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i]))
            return 0;
    return 1;
}

/* Per-particle outcome counters summed by the caller. */
typedef struct {
    int64_t evals;        /* Cash-Karp evaluations (6 field lookups each) */
    int64_t accepted, rejected, event_evals, floor_hits;
} counts_t;

/* Optional tape of accepted step sizes (for the adjoint); NULL = none. */
typedef struct {
    double *h;            /* accepted step sizes, in order */
    int64_t cap, len;
    double s_event;       /* event step s* (0 if no event) */
    int event;            /* 1 if the run ended by sphere crossing */
    int length_bound;     /* 1 if the last accepted step was the length bid */
} tape_t;

/* Propagate one particle in place.  State y = (x, u); L = path length;
 * *h_next = controller bid carried between calls (0 = fresh start). */
static int propagate_one(const grid_t *g, const params_t *p, double y[6], double energy,
                         int32_t charge, double *L, double *h_next, int64_t *n_acc,
                         int64_t *n_rej, counts_t *cnt, tape_t *tape)
{
    const int sphere = p->radius > 0.0;
    const int lmax_on = isfinite(p->l_max);
    const double R2 = p->radius * p->radius;

    if (!(energy > 0.0) || !isfinite(energy) || !all_finite(y, 6) || !isfinite(*L) ||
        !(*h_next >= 0.0) || !isfinite(*h_next))
        return ST_BAD_INPUT;

    double hctrl;
    if (*h_next == 0.0) {                  /* fresh start: unit direction, first bid h_max */
        double n2 = y[3] * y[3] + y[4] * y[4] + y[5] * y[5];
        if (!(n2 > 0.0))
            return ST_BAD_INPUT;
        double nrm = sqrt(n2);
        y[3] = y[3] / nrm;
        y[4] = y[4] / nrm;
        y[5] = y[5] / nrm;
        hctrl = p->h_max;
    } else {
        hctrl = *h_next;
    }
    if (sphere && sphere_g(p, y) >= 0.0)
        return ST_ARRIVED;
    if (lmax_on && *L >= p->l_max)
        return ST_MAX_LENGTH;

    const double kappa = ((double)charge * K_LORENTZ) / energy;
    int64_t steps_this_call = 0;

    for (;;) {
        /* bids: controller, h_max, sphere distance (all floored by h_min),
         * then the remaining length (not floored) */
        double h = hctrl;
        if (h > p->h_max) h = p->h_max;
        if (sphere) {
            double d0 = y[0] - p->center[0], d1 = y[1] - p->center[1], d2 = y[2] - p->center[2];
            double dist = p->radius - sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            if (dist < h) h = dist;
        }
        if (p->reflect) {         /* the distance to the nearest face of the box bids too */
            for (int a = 0; a < 3; ++a) {
                double dlo = y[a] - p->box_lo[a], dhi = p->box_hi[a] - y[a];
                if (dlo < h) h = dlo;
                if (dhi < h) h = dhi;
            }
        }
        if (h < p->h_min) h = p->h_min;
        int binding = 0;
        if (lmax_on) {
            double rem = p->l_max - *L;
            if (rem <= h) {
                h = rem;
                binding = 1;
            }
        }

        /* attempts until accepted */
        double y5[6], delta[6], err;
        for (;;) {
            ck_eval(g, kappa, y, h, y5, delta);
            cnt->evals++;
            double eu = norm3(delta + 3);
            double exh = norm3(delta) / h;
            if (!isfinite(eu) || !isfinite(exh)) {
                *h_next = hctrl;
                return ST_NONFINITE;
            }
            double em = eu > exh ? eu : exh;
            err = em / p->tol;
            if (err > 1.0 && h > p->h_min) {
                double fac = 0.9 * (1.0 / sqrt(sqrt(err)));
                if (fac < 0.1) fac = 0.1;
                h = h * fac;
                if (h < p->h_min) h = p->h_min;
                binding = 0;
                (*n_rej)++;
                cnt->rejected++;
                continue;
            }
            break;
        }

        /* accepted: next controller bid */
        int floor_hit = err > 1.0;
        double gfac;
        if (floor_hit) {
            gfac = 1.0;
            cnt->floor_hits++;
        } else if (err == 0.0) {
            gfac = 5.0;
        } else {
            gfac = 0.9 * inv_fifth_root(err);
            if (gfac > 5.0) gfac = 5.0;
        }
        hctrl = h * gfac;
        if (hctrl < p->h_min) hctrl = p->h_min;
        if (hctrl > p->h_max) hctrl = p->h_max;

        double un2 = y5[3] * y5[3] + y5[4] * y5[4] + y5[5] * y5[5];
        double un = sqrt(un2);
        double ynew[6] = {y5[0], y5[1], y5[2], y5[3] / un, y5[4] / un, y5[5] / un};
        double Lnew = binding ? p->l_max : *L + h;
        (*n_acc)++;
        cnt->accepted++;
        steps_this_call++;
        if (tape && tape->h) {
            if (tape->len < tape->cap) tape->h[tape->len] = h;
            tape->len++;
            tape->length_bound = binding;
        }

        /* stops, in order: sphere crossing, length, step budget */
        if (sphere && sphere_g(p, ynew) >= 0.0) {
            double lo = 0.0, glo = sphere_g(p, y), hi = h, ghi = sphere_g(p, ynew);
            int side = 0;
            for (int it = 0; it < 30; ++it) {
                /* converged when the outside end is on the sphere to 1e-14 R^2,
                 * or the bracket is below 1e-15 h; s* is always the outside end */
                if (ghi <= 1e-14 * R2 || (hi - lo) <= 1e-15 * h)
                    break;
                double s = (lo * ghi - hi * glo) / (ghi - glo);
                double ys[6], ds[6];
                ck_eval(g, kappa, y, s, ys, ds);
                cnt->evals++;
                cnt->event_evals++;
                double gs = sphere_g(p, ys);
                if (!isfinite(gs)) {
                    *h_next = hctrl;
                    return ST_NONFINITE;
                }
                if (gs >= 0.0) {
                    hi = s;
                    ghi = gs;
                    if (side == 1) glo = glo * 0.5;
                    side = 1;
                } else {
                    lo = s;
                    glo = gs;
                    if (side == -1) ghi = ghi * 0.5;
                    side = -1;
                }
            }
            if (hi != h) {
                double ys[6], ds[6];
                ck_eval(g, kappa, y, hi, ys, ds);
                cnt->evals++;
                cnt->event_evals++;
                double sn = sqrt(ys[3] * ys[3] + ys[4] * ys[4] + ys[5] * ys[5]);
                ynew[0] = ys[0];
                ynew[1] = ys[1];
                ynew[2] = ys[2];
                ynew[3] = ys[3] / sn;
                ynew[4] = ys[4] / sn;
                ynew[5] = ys[5] / sn;
                Lnew = *L + hi;
            }
            memcpy(y, ynew, sizeof ynew);
            *L = Lnew;
            *h_next = hctrl;
            if (tape) {
                tape->event = 1;
                tape->s_event = hi;
            }
            return ST_ARRIVED;
        }
        if (p->reflect)
            reflect_state(p, ynew);
        memcpy(y, ynew, sizeof ynew);
        *L = Lnew;
        if (lmax_on && *L >= p->l_max) {
            *h_next = hctrl;
            return ST_MAX_LENGTH;
        }
        if (p->max_steps > 0 && steps_this_call >= p->max_steps) {
            *h_next = hctrl;
            return ST_MAX_STEPS;
        }
    }
}

/* ======================= exported C interface ============================ */

/* mod: NULL for no modulation, else the modulation values ([n0][n1][n2],
 * dtype mod_desc[3]); mod_desc = {n0, n1, n2, dtype, origin x, y, z, spacing}. */
static int make_grid(grid_t *g, const void *data, int dtype, int64_t n0, int64_t n1, int64_t n2,
                     const double origin[3], double spacing, const void *mod, const double *mod_desc)
{
    if (!data || n0 < 2 || n1 < 2 || n2 < 2 || !(spacing > 0.0) || (dtype != 0 && dtype != 1))
        return -1;
    g->mod.present = 0;
    if (mod) {
        if (!mod_desc)
            return -1;
        int64_t m0 = (int64_t)mod_desc[0], m1 = (int64_t)mod_desc[1], m2 = (int64_t)mod_desc[2];
        int mdt = (int)mod_desc[3];
        if (m0 < 2 || m1 < 2 || m2 < 2 || !(mod_desc[7] > 0.0) || (mdt != 0 && mdt != 1))
            return -1;
        g->mod.present = 1;
        g->mod.n[0] = m0;
        g->mod.n[1] = m1;
        g->mod.n[2] = m2;
        for (int a = 0; a < 3; ++a)
            g->mod.origin[a] = mod_desc[4 + a];
        g->mod.inv_spacing = 1.0 / mod_desc[7];
        g->mod.v64 = mdt == 0 ? (const double *)mod : NULL;
        g->mod.v32 = mdt == 1 ? (const float *)mod : NULL;
    }
    g->n[0] = n0;
    g->n[1] = n1;
    g->n[2] = n2;
    for (int a = 0; a < 3; ++a)
        g->origin[a] = origin ? origin[a] : 0.0;
    g->inv_spacing = 1.0 / spacing;
    g->v64 = dtype == 0 ? (const double *)data : NULL;
    g->v32 = dtype == 1 ? (const float *)data : NULL;
    return 0;
}

/* Constants and tableau, for the pins. out: [K, Mpc/c, A(36), c(6), b5(6), b4(6), e(6), T(5)] */
void oracle_constants(double *out)
{
    out[0] = K_LORENTZ;
    out[1] = MPC_OVER_C;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j)
            out[2 + 6 * i + j] = j < 5 ? CK_A[i][j] : 0.0;
    for (int i = 0; i < 6; ++i) {
        out[38 + i] = CK_C[i];
        out[44 + i] = CK_B5[i];
        out[50 + i] = CK_B4[i];
        out[56 + i] = CK_E[i];
    }
    for (int j = 0; j < 5; ++j)
        out[62 + j] = TWO_POW_NEG_FIFTHS[j];
}

double oracle_inv_fifth_root(double err) { return inv_fifth_root(err); }

/* Field at n points X[n][3] -> B[n][3]. Returns 0 or -1 on bad arguments. */
int oracle_field_at(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2,
                    const double *origin, double spacing, const void *mod, const double *mod_desc, const double *X, double *B, int64_t n)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc))
        return -1;
    for (int64_t i = 0; i < n; ++i)
        field_total(&g, X + 3 * i, B + 3 * i);
    return 0;
}

/* One Cash-Karp evaluation (no control): y[6], h -> y5[6], delta[6]. */
int oracle_ck_eval(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2,
                   const double *origin, double spacing, const void *mod, const double *mod_desc, double kappa, const double *y, double h,
                   double *y5, double *delta)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc))
        return -1;
    ck_eval(&g, kappa, y, h, y5, delta);
    return 0;
}

/* Fixed-step integration (no controller, no normalisation): nsteps of size h. */
int oracle_fixed_steps(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2,
                       const double *origin, double spacing, const void *mod, const double *mod_desc, double kappa, double *y, double h,
                       int64_t nsteps)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc))
        return -1;
    for (int64_t s = 0; s < nsteps; ++s) {
        double y5[6], d[6];
        ck_eval(&g, kappa, y, h, y5, d);
        memcpy(y, y5, sizeof y5);
    }
    return 0;
}

/* Propagate n particles in place.  prm: the parameter block of read_params.
 * Arrays of length n (pos/dir are n x 3).  counters (may be NULL): 5 int64 summed
 * [evals, accepted, rejected, event_evals, floor_hits].  Returns 0 or -1. */
int oracle_propagate(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2,
                     const double *origin, double spacing, const void *mod, const double *mod_desc, const double *prm, int64_t max_steps,
                     int64_t n, double *pos, double *dir, const double *energy,
                     const int32_t *charge, double *length, double *h_next, int32_t *status,
                     int64_t *n_acc, int64_t *n_rej, int64_t *counters, int nthreads)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc) || n < 0 || !prm)
        return -1;
    params_t p;
    if (read_params(prm, &p))
        return -1;
    p.max_steps = max_steps;
    if (!(p.tol > 0.0) || !(p.h_min > 0.0) || !(p.h_max >= p.h_min) || isnan(p.l_max) ||
        !(p.l_max > 0.0) || (!isfinite(p.l_max) && max_steps <= 0))
        return -1;
    int64_t c_evals = 0, c_acc = 0, c_rej = 0, c_ev = 0, c_fl = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads) \
    reduction(+ : c_evals, c_acc, c_rej, c_ev, c_fl)
#endif
    for (int64_t i = 0; i < n; ++i) {
        if (status[i] != ST_ACTIVE)
            continue;
        double y[6] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2],
                       dir[3 * i], dir[3 * i + 1], dir[3 * i + 2]};
        int32_t z = charge[i];
        if (p.backtrack) { /* the antiparticle, moving the other way */
            for (int c = 3; c < 6; ++c)
                y[c] = -y[c];
            z = -z;
        }
        counts_t cnt = {0, 0, 0, 0, 0};
        double L = length[i], hn = h_next[i];
        int st = propagate_one(&g, &p, y, energy[i], z, &L, &hn, &n_acc[i], &n_rej[i], &cnt, NULL);
        status[i] = st;
        if (st != ST_BAD_INPUT) {
            for (int c = 0; c < 3; ++c) {
                pos[3 * i + c] = y[c];
                dir[3 * i + c] = p.backtrack ? -y[3 + c] : y[3 + c];
            }
            length[i] = L;
            h_next[i] = hn;
        }
        c_evals += cnt.evals;
        c_acc += cnt.accepted;
        c_rej += cnt.rejected;
        c_ev += cnt.event_evals;
        c_fl += cnt.floor_hits;
    }
    if (counters) {
        counters[0] += c_evals;
        counters[1] += c_acc;
        counters[2] += c_rej;
        counters[3] += c_ev;
        counters[4] += c_fl;
    }
    return 0;
}

/* Propagate one particle recording the accepted step sizes (for the adjoint
 * and for tests).  h_tape has capacity cap; returns the number of accepted
 * steps (may exceed cap, then the tape is truncated) or -1.  info[0] = status,
 * info[1] = event flag, info[2] = s* of the event, info[3] = length-bound flag. */
int64_t oracle_propagate_taped(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2,
                               const double *origin, double spacing, const void *mod, const double *mod_desc, const double *prm,
                               double *y, double energy, int32_t charge, double *length,
                               double *h_next, double *h_tape, int64_t cap, double *info)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc))
        return -1;
    params_t p;
    if (read_params(prm, &p))
        return -1;
    if (p.backtrack) /* the replayed map has no reversal (the caller reverses the particle) */
        return -1;
    p.max_steps = 0;
    if (!isfinite(p.l_max))
        return -1;
    tape_t tape = {h_tape, cap, 0, 0.0, 0, 0};
    counts_t cnt = {0, 0, 0, 0, 0};
    int64_t na = 0, nr = 0;
    int st = propagate_one(&g, &p, y, energy, charge, length, h_next, &na, &nr, &cnt, &tape);
    info[0] = st;
    info[1] = tape.event;
    info[2] = tape.s_event;
    info[3] = tape.length_bound;
    return tape.len;
}

/* ======================= derivatives of the replayed map ==================
 *
 * The map differentiated is the replay of a forward run with its accepted
 * step sizes h_0 .. h_{N-1} frozen: y_{n+1} = N(Phi(y_n, h_n)), N normalising
 * the direction, y_0 = (x_0, u_0/|u_0|).  The last step is either the fixed
 * recorded step (length stop) or the sphere crossing s*, defined implicitly
 * by |X(y_{N-1}, s*) - c|^2 = R^2 inside [0, h_{N-1}] (implicit function
 * theorem for its derivative).  Outputs: final direction u_N and path length
 * L = sum of the steps (time = L * Mpc / c).  The energy is unchanged, so its
 * derivative is zero.
 *
 * In a reflective box every step but an event step is followed by the mirror
 * of the forward run, decided on the replayed state's value as the propagator
 * decides it and then held fixed: on each mirrored axis the position becomes
 * 2 face - x and the direction component changes sign, so the tangent and
 * the cotangent of both change sign there.
 *
 * Jacobians: f(Y) = (U, kappa U x B(X)); for a cotangent (kx, ku) of f,
 *   U-bar = kx + kappa B x ku,  B-bar = kappa ku x U,
 *   X-bar = (dB/dX)^T B-bar,    G-bar[node] += w_node B-bar,
 * with the trilinear weights w_node and gradient dB/dX of the cell in which
 * the stage was evaluated.  For a modulated field B = b m the vector grid's
 * value b takes the cotangent b-bar = m B-bar, so X-bar = (db/dX)^T b-bar +
 * (b . B-bar) dm/dX and G-bar[node] += w_node b-bar (the modulation grid's
 * own values get no gradient).
 */

typedef struct {
    double v, d;
} dual;

static dual dl(double v, double d) { dual r = {v, d}; return r; }
static dual d_add(dual a, dual b) { return dl(a.v + b.v, a.d + b.d); }
static dual d_sub(dual a, dual b) { return dl(a.v - b.v, a.d - b.d); }
static dual d_mul(dual a, dual b) { return dl(a.v * b.v, a.d * b.v + a.v * b.d); }
static dual d_fma(dual a, dual b, dual c) { return dl(fma(a.v, b.v, c.v), a.d * b.v + a.v * b.d + c.d); }
static dual d_sqrt(dual a)
{
    double s = sqrt(a.v);
    return dl(s, a.d / (2.0 * s));
}
static dual d_div(dual a, dual b)
{
    double q = a.v / b.v;
    return dl(q, (a.d - q * b.d) / b.v);
}

/* Trilinear weights of the 8 corners, their flat indices, and dB/dX of the cell
 * containing X.  Corner order: (dx, dy, dz) with dx fastest. */
static int cell_stencil(const grid_t *g, const double X[3], double w[8], int64_t idx[8], double dw[3][8])
{
    int64_t i0[3], i1[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double f = (X[a] - g->origin[a]) * g->inv_spacing;
        if (!(fabs(f) < 4.0e15))
            return -1;
        double fl = floor(f);
        t[a] = f - fl;
        i0[a] = pmod((int64_t)fl, g->n[a]);
        i1[a] = pmod(i0[a] + 1, g->n[a]);
    }
    for (int c = 0; c < 8; ++c) {
        int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        double wx = dx ? t[0] : 1.0 - t[0], wy = dy ? t[1] : 1.0 - t[1], wz = dz ? t[2] : 1.0 - t[2];
        double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
        w[c] = wx * wy * wz;
        dw[0][c] = sx * wy * wz * g->inv_spacing;
        dw[1][c] = wx * sy * wz * g->inv_spacing;
        dw[2][c] = wx * wy * sz * g->inv_spacing;
        idx[c] = ((dx ? i1[0] : i0[0]) * g->n[1] + (dy ? i1[1] : i0[1])) * g->n[2] + (dz ? i1[2] : i0[2]);
    }
    return 0;
}

/* Gradient dm/dX of the modulation (trilinear in its own cell, the cell
 * mod_at reads), summed over the corners in the order of cell_stencil. */
static int mod_gradient(const modgrid_t *m, const double X[3], double dm[3])
{
    int64_t i0[3], i1[3];
    double t[3];
    for (int a = 0; a < 3; ++a) {
        double f = (X[a] - m->origin[a]) * m->inv_spacing;
        if (!(fabs(f) < 4.0e15))
            return -1;
        double fl = floor(f);
        t[a] = f - fl;
        i0[a] = pmod((int64_t)fl, m->n[a]);
        i1[a] = pmod(i0[a] + 1, m->n[a]);
    }
    dm[0] = dm[1] = dm[2] = 0.0;
    for (int c = 0; c < 8; ++c) {
        int dx = c & 1, dy = (c >> 1) & 1, dz = (c >> 2) & 1;
        double wx = dx ? t[0] : 1.0 - t[0], wy = dy ? t[1] : 1.0 - t[1], wz = dz ? t[2] : 1.0 - t[2];
        double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
        int64_t k = ((dx ? i1[0] : i0[0]) * m->n[1] + (dy ? i1[1] : i0[1])) * m->n[2] + (dz ? i1[2] : i0[2]);
        double v = m->v64 ? m->v64[k] : (double)m->v32[k];
        dm[0] += sx * wy * wz * m->inv_spacing * v;
        dm[1] += wx * sy * wz * m->inv_spacing * v;
        dm[2] += wx * wy * sz * m->inv_spacing * v;
    }
    return 0;
}

/* Field value (bitwise the propagator's) and its tangent along X-dot, plus the
 * tangent of the vector grid's values vg (FP64, same layout) when given.  A
 * modulated field B = b m has the tangent b-dot m + b m-dot. */
static void field_dual(const grid_t *g, const double *vg, const dual X[3], dual B[3])
{
    double x[3] = {X[0].v, X[1].v, X[2].v}, b[3];
    field_at(g, x, b);
    double w[8], dw[3][8], dm[3] = {0.0, 0.0, 0.0};
    int64_t idx[8];
    if (cell_stencil(g, x, w, idx, dw) || (g->mod.present && mod_gradient(&g->mod, x, dm))) {
        for (int c = 0; c < 3; ++c)
            B[c] = dl(NAN, NAN);
        return;
    }
    double m = g->mod.present ? mod_at(&g->mod, x) : 1.0;
    double mdot = dm[0] * X[0].d + dm[1] * X[1].d + dm[2] * X[2].d;
    for (int c = 0; c < 3; ++c) {
        double d = 0.0;
        for (int k = 0; k < 8; ++k) {
            double val = g->v64 ? g->v64[3 * idx[k] + c] : (double)g->v32[3 * idx[k] + c];
            d += (dw[0][k] * X[0].d + dw[1][k] * X[1].d + dw[2][k] * X[2].d) * val;
            if (vg)
                d += w[k] * vg[3 * idx[k] + c];
        }
        B[c] = g->mod.present ? dl(b[c] * m, d * m + b[c] * mdot) : dl(b[c], d);
    }
}

static void rhs_dual(const grid_t *g, const double *vg, double kappa, const dual Y[6], dual k[6])
{
    dual B[3];
    field_dual(g, vg, Y, B);
    dual kp = dl(kappa, 0.0);
    k[0] = Y[3];
    k[1] = Y[4];
    k[2] = Y[5];
    k[3] = d_mul(kp, d_sub(d_mul(Y[4], B[2]), d_mul(Y[5], B[1])));
    k[4] = d_mul(kp, d_sub(d_mul(Y[5], B[0]), d_mul(Y[3], B[2])));
    k[5] = d_mul(kp, d_sub(d_mul(Y[3], B[1]), d_mul(Y[4], B[0])));
}

/* Cash-Karp step on dual numbers: primal values are bitwise those of ck_eval. */
static void ck_eval_dual(const grid_t *g, const double *vg, double kappa, const dual y[6], dual h, dual y5[6])
{
    dual k[6][6];
    for (int i = 0; i < 6; ++i) {
        dual Y[6];
        for (int c = 0; c < 6; ++c) {
            if (i == 0) {
                Y[c] = y[c];
                continue;
            }
            dual acc = dl(0.0, 0.0);
            for (int j = 0; j < i; ++j)
                acc = d_fma(dl(CK_A[i][j], 0.0), k[j][c], acc);
            Y[c] = d_fma(h, acc, y[c]);
        }
        rhs_dual(g, vg, kappa, Y, k[i]);
    }
    for (int c = 0; c < 6; ++c) {
        dual a5 = dl(0.0, 0.0);
        for (int i = 0; i < 6; ++i)
            a5 = d_fma(dl(CK_B5[i], 0.0), k[i][c], a5);
        y5[c] = d_fma(h, a5, y[c]);
    }
}

static void normalize_dual(dual y[6])
{
    dual n = d_sqrt(d_add(d_add(d_mul(y[3], y[3]), d_mul(y[4], y[4])), d_mul(y[5], y[5])));
    y[3] = d_div(y[3], n);
    y[4] = d_div(y[4], n);
    y[5] = d_div(y[5], n);
}

/* Axes on which a reflective box (box = lo x, y, z, hi x, y, z; NULL: none)
 * mirrors a step ending at x: bit a for axis a (the test of reflect_state). */
static int mirror_mask(const double *box, const double x[3])
{
    int m = 0;
    if (box)
        for (int a = 0; a < 3; ++a)
            if (x[a] > box[3 + a] || x[a] < box[a])
                m |= 1 << a;
    return m;
}

/* The mirror of reflect_state on the axes of mask m: position 2 face - x,
 * direction component negated. */
static void mirror_apply(const double *box, int m, double y[6])
{
    for (int a = 0; a < 3; ++a)
        if (m >> a & 1) {
            y[a] = 2.0 * (y[a] > box[3 + a] ? box[3 + a] : box[a]) - y[a];
            y[3 + a] = -y[3 + a];
        }
}

/* The same on a state with tangents: the tangents of the mirrored components
 * change sign. */
static void mirror_apply_dual(const double *box, dual y[6])
{
    double v[3] = {y[0].v, y[1].v, y[2].v};
    int m = mirror_mask(box, v);
    for (int a = 0; a < 3; ++a)
        if (m >> a & 1) {
            y[a] = dl(2.0 * (y[a].v > box[3 + a] ? box[3 + a] : box[a]) - y[a].v, -y[a].d);
            y[3 + a] = dl(-y[3 + a].v, -y[3 + a].d);
        }
}

/* Cotangent through the mirror of mask m: the mirrored components change sign. */
static void mirror_cotangent(int m, double lam[6])
{
    for (int a = 0; a < 3; ++a)
        if (m >> a & 1) {
            lam[a] = -lam[a];
            lam[3 + a] = -lam[3 + a];
        }
}

static double sphere_g_xyz(const double c[3], double R, const double x[3])
{
    double d0 = x[0] - c[0], d1 = x[1] - c[1], d2 = x[2] - c[2];
    return (d0 * d0 + d1 * d1 + d2 * d2) - R * R;
}

/* Crossing s* of the sphere inside [0, h] from y (Illinois, as in propagate_one). */
static double locate_crossing(const grid_t *g, double kappa, const double y[6], double h, const double c[3],
                              double R)
{
    double y5[6], d5[6];
    ck_eval(g, kappa, y, h, y5, d5);
    double R2 = R * R;
    double lo = 0.0, glo = sphere_g_xyz(c, R, y), hi = h, ghi = sphere_g_xyz(c, R, y5);
    int side = 0;
    for (int it = 0; it < 30; ++it) {
        if (ghi <= 1e-14 * R2 || (hi - lo) <= 1e-15 * h)
            break;
        double s = (lo * ghi - hi * glo) / (ghi - glo);
        double ys[6], ds[6];
        ck_eval(g, kappa, y, s, ys, ds);
        double gs = sphere_g_xyz(c, R, ys);
        if (gs >= 0.0) {
            hi = s;
            ghi = gs;
            if (side == 1) glo = glo * 0.5;
            side = 1;
        } else {
            lo = s;
            glo = gs;
            if (side == -1) ghi = ghi * 0.5;
            side = -1;
        }
    }
    return hi;
}

/* Root of |X(y, s) - c|^2 = R^2 near s = 0 by Newton's method on the step
 * map continued analytically to small negative s (for replays of perturbed
 * inputs whose crossing moved just outside the frozen last step). */
static int crossing_newton(const grid_t *g, double kappa, const double y[6], const double c[3], double R,
                           double *sout)
{
    double s = 0.0;
    dual yd[6];
    for (int a = 0; a < 6; ++a)
        yd[a] = dl(y[a], 0.0);
    for (int it = 0; it < 40; ++it) {
        dual z[6];
        ck_eval_dual(g, NULL, kappa, yd, dl(s, 1.0), z);
        double gv = -R * R, gs = 0.0;
        for (int a = 0; a < 3; ++a) {
            double r = z[a].v - c[a];
            gv += r * r;
            gs += 2.0 * r * z[a].d;
        }
        if (!(gs != 0.0) || !isfinite(gv))
            return -1;
        double ds = gv / gs;
        s -= ds;
        if (fabs(gv) <= 1e-14 * R * R || fabs(ds) <= 1e-16 * (fabs(s) + 1e-300)) {
            *sout = s;
            return 0;
        }
    }
    *sout = s;
    return 0;
}

/* Forward-mode replay.  Inputs: x0, raw u0 (normalised inside), tangents du0
 * and dx0 of the initial direction and position (each may be NULL) and grid
 * tangent vg (may be NULL), the frozen steps h[0..n-1]
 * (h[n-1] is the last accepted step), event != 0 for a sphere crossing in the
 * last step (centre c, radius R; s* found here: by the propagator's Illinois
 * iteration when [0, h[n-1]] brackets it, else by Newton's method on the
 * step map continued to small negative s), box: the reflective box (lo x, y,
 * z, hi x, y, z) or NULL.  out: [u_N(3), L, du_N(3), dL, x_N(3), s*].
 * Returns 0, or -1 on bad arguments or no root. */
int oracle_replay_tangent(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2, const double *origin,
                          double spacing, const void *mod, const double *mod_desc, double kappa, const double *x0, const double *u0, const double *du0,
                          const double *dx0, const double *vg, const double *h, int64_t n, int event, const double *c,
                          double R, const double *box, double *out)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc) || n < 1)
        return -1;
    dual y[6];
    for (int a = 0; a < 3; ++a) {
        y[a] = dl(x0[a], dx0 ? dx0[a] : 0.0);
        y[3 + a] = dl(u0[a], du0 ? du0[a] : 0.0);
    }
    normalize_dual(y);
    double L = 0.0;
    for (int64_t s = 0; s + 1 < n; ++s) {
        dual y5[6];
        ck_eval_dual(&g, vg, kappa, y, dl(h[s], 0.0), y5);
        normalize_dual(y5);
        mirror_apply_dual(box, y5);
        memcpy(y, y5, sizeof y);
        L += h[s];
    }
    double sstar = h[n - 1];
    double ds = 0.0;
    dual z[6];
    if (event) {
        double yv[6] = {y[0].v, y[1].v, y[2].v, y[3].v, y[4].v, y[5].v};
        double y5[6], d5[6];
        ck_eval(&g, kappa, yv, h[n - 1], y5, d5);
        if (sphere_g_xyz(c, R, yv) < 0.0 && sphere_g_xyz(c, R, y5) >= 0.0)
            sstar = locate_crossing(&g, kappa, yv, h[n - 1], c, R);
        else if (crossing_newton(&g, kappa, yv, c, R, &sstar))
            return -1;
        /* tangent of the position at fixed s*, and dPhi/ds at s* */
        ck_eval_dual(&g, vg, kappa, y, dl(sstar, 0.0), z);
        dual ys[6];
        for (int a = 0; a < 6; ++a)
            ys[a] = dl(y[a].v, 0.0);
        dual zs[6];
        ck_eval_dual(&g, NULL, kappa, ys, dl(sstar, 1.0), zs);
        double gdot = 0.0, gs = 0.0;
        for (int a = 0; a < 3; ++a) {
            double r = z[a].v - c[a];
            gdot += 2.0 * r * z[a].d;
            gs += 2.0 * r * zs[a].d;
        }
        ds = -gdot / gs;
        for (int a = 0; a < 6; ++a)
            z[a].d += zs[a].d * ds;
    } else {
        ck_eval_dual(&g, vg, kappa, y, dl(sstar, 0.0), z);
    }
    normalize_dual(z);
    if (!event) /* an event step ends on the sphere, unmirrored */
        mirror_apply_dual(box, z);
    L += sstar;
    for (int a = 0; a < 3; ++a) {
        out[a] = z[3 + a].v;
        out[4 + a] = z[3 + a].d;
        out[8 + a] = z[a].v;
    }
    out[3] = L;
    out[7] = ds;
    out[11] = sstar;
    return 0;
}

/* Reverse sweep of one step y -> N(Phi(y, s)) given the cotangent lam of the
 * normalised output (6); comb (may be NULL) is an extra cotangent added to the
 * unnormalised output (the event term).  ybar gets the cotangent of y; the grid
 * cotangent is accumulated into gbar (may be NULL). */
static void step_vjp(const grid_t *g, double kappa, const double y[6], double s, const double lam[6],
                     const double *comb, double ybar[6], double *gbar, double *kbar)
{
    double k[6][6], Y[6][6];
    for (int i = 0; i < 6; ++i) {
        for (int c = 0; c < 6; ++c) {
            if (i == 0) {
                Y[i][c] = y[c];
                continue;
            }
            double acc = 0.0;
            for (int j = 0; j < i; ++j)
                acc = fma(CK_A[i][j], k[j][c], acc);
            Y[i][c] = fma(s, acc, y[c]);
        }
        rhs(g, kappa, Y[i], k[i]);
    }
    double z[6];
    for (int c = 0; c < 6; ++c) {
        double a5 = 0.0;
        for (int i = 0; i < 6; ++i)
            a5 = fma(CK_B5[i], k[i][c], a5);
        z[c] = fma(s, a5, y[c]);
    }
    /* normalisation: u = z_u/|z_u|; zbar_u = (lam_u - (lam_u.u) u)/|z_u| */
    double zn = sqrt(z[3] * z[3] + z[4] * z[4] + z[5] * z[5]);
    double u[3] = {z[3] / zn, z[4] / zn, z[5] / zn};
    double lu = lam[3] * u[0] + lam[4] * u[1] + lam[5] * u[2];
    double zbar[6] = {lam[0], lam[1], lam[2], (lam[3] - lu * u[0]) / zn, (lam[4] - lu * u[1]) / zn,
                      (lam[5] - lu * u[2]) / zn};
    if (comb)
        for (int c = 0; c < 6; ++c)
            zbar[c] += comb[c];
    double Ybar[6][6];
    for (int c = 0; c < 6; ++c)
        ybar[c] = zbar[c];
    for (int i = 5; i >= 0; --i) {
        double kb[6];
        for (int c = 0; c < 6; ++c) {
            double v = s * CK_B5[i] * zbar[c];
            for (int j = i + 1; j < 6; ++j)
                v += s * CK_A[j][i] * Ybar[j][c];
            kb[c] = v;
        }
        /* B = b m: the value the stage used, the vector grid's value b and the
         * modulation m (1 without one) */
        double B[3], b[3], m = 1.0;
        field_at(g, Y[i], b);
        if (g->mod.present)
            m = mod_at(&g->mod, Y[i]);
        field_total(g, Y[i], B);
        const double *U = Y[i] + 3;
        double w[8], dw[3][8];
        int64_t idx[8];
        /* B-bar = kappa ku x U, U-bar = kx + kappa B x ku */
        double Bb[3] = {kappa * (kb[4] * U[2] - kb[5] * U[1]), kappa * (kb[5] * U[0] - kb[3] * U[2]),
                        kappa * (kb[3] * U[1] - kb[4] * U[0])};
        /* kappa enters the stage as kappa U x B: kappa-bar += ku . (U x B) */
        *kbar += kb[3] * (U[1] * B[2] - U[2] * B[1]) + kb[4] * (U[2] * B[0] - U[0] * B[2]) +
                 kb[5] * (U[0] * B[1] - U[1] * B[0]);
        Ybar[i][3] = kb[0] + kappa * (B[1] * kb[5] - B[2] * kb[4]);
        Ybar[i][4] = kb[1] + kappa * (B[2] * kb[3] - B[0] * kb[5]);
        Ybar[i][5] = kb[2] + kappa * (B[0] * kb[4] - B[1] * kb[3]);
        Ybar[i][0] = Ybar[i][1] = Ybar[i][2] = 0.0;
        /* cotangent of the vector grid's interpolated value: b-bar = m B-bar */
        double bb[3] = {Bb[0] * m, Bb[1] * m, Bb[2] * m};
        if (cell_stencil(g, Y[i], w, idx, dw) == 0) {
            for (int kk = 0; kk < 8; ++kk) {
                double val[3];
                for (int c = 0; c < 3; ++c)
                    val[c] = g->v64 ? g->v64[3 * idx[kk] + c] : (double)g->v32[3 * idx[kk] + c];
                /* X-bar += (db/dX)^T b-bar, written as the gradient of the scalar
                 * b-bar . b(X) = sum over corners of w(X) (G . b-bar): each
                 * corner's value dotted with b-bar, times grad w */
                double vb = val[0] * bb[0] + val[1] * bb[1] + val[2] * bb[2];
                for (int a = 0; a < 3; ++a)
                    Ybar[i][a] += dw[a][kk] * vb;
                if (gbar)
                    for (int c = 0; c < 3; ++c)
                        gbar[3 * idx[kk] + c] += w[kk] * bb[c];
            }
        }
        double dm[3];
        if (g->mod.present && mod_gradient(&g->mod, Y[i], dm) == 0) {
            /* X-bar += (b . B-bar) dm/dX */
            double bB = b[0] * Bb[0] + b[1] * Bb[1] + b[2] * Bb[2];
            for (int a = 0; a < 3; ++a)
                Ybar[i][a] += dm[a] * bB;
        }
        for (int c = 0; c < 6; ++c)
            ybar[c] += Ybar[i][c];
    }
}

/* Reverse-mode replay (full tape; box: the reflective box or NULL, as in
 * oracle_replay_tangent).  ubar: cotangent of u_N (3); Lbar:
 * cotangent of the path length (t-bar * Mpc / c).  Outputs: u0bar (cotangent
 * of the raw initial direction), x0bar; gbar (3 n0 n1 n2, FP64) accumulated if
 * not NULL; kappabar (may be NULL): the cotangent of kappa = Z K / E, summed
 * over the stages from the last step to the first (the crossing s* depends on
 * kappa too and is carried by the combined cotangent of the last step); the
 * energy gradient is kappabar * (-kappa / E).  Returns 0 or -1. */
int oracle_replay_adjoint(const void *grid, int dtype, int64_t n0, int64_t n1, int64_t n2, const double *origin,
                          double spacing, const void *mod, const double *mod_desc, double kappa, const double *x0, const double *u0, const double *h,
                          int64_t n, int event, const double *c, double R, const double *box, const double *ubar,
                          double Lbar, double *u0bar, double *x0bar, double *gbar, double *kappabar)
{
    grid_t g;
    if (make_grid(&g, grid, dtype, n0, n1, n2, origin, spacing, mod, mod_desc) || n < 1)
        return -1;
    double *ys = (double *)malloc(sizeof(double) * 6 * (size_t)n);
    unsigned char *mir = (unsigned char *)malloc((size_t)n); /* mirror mask after each step */
    if (!ys || !mir) {
        free(ys);
        free(mir);
        return -1;
    }
    double un = sqrt(u0[0] * u0[0] + u0[1] * u0[1] + u0[2] * u0[2]);
    double y[6] = {x0[0], x0[1], x0[2], u0[0] / un, u0[1] / un, u0[2] / un};
    for (int64_t s = 0; s < n; ++s) {
        memcpy(ys + 6 * s, y, sizeof y);
        if (s + 1 < n) {
            double y5[6], d5[6];
            ck_eval(&g, kappa, y, h[s], y5, d5);
            double m = sqrt(y5[3] * y5[3] + y5[4] * y5[4] + y5[5] * y5[5]);
            y[0] = y5[0];
            y[1] = y5[1];
            y[2] = y5[2];
            y[3] = y5[3] / m;
            y[4] = y5[4] / m;
            y[5] = y5[5] / m;
            mir[s] = (unsigned char)mirror_mask(box, y);
            mirror_apply(box, mir[s], y);
        }
    }
    const double *yl = ys + 6 * (n - 1);
    double lam[6] = {0.0, 0.0, 0.0, ubar[0], ubar[1], ubar[2]};
    mir[n - 1] = 0;
    if (!event && box) { /* the last step of a length stop is mirrored too */
        double y5[6], d5[6];
        ck_eval(&g, kappa, yl, h[n - 1], y5, d5);
        mir[n - 1] = (unsigned char)mirror_mask(box, y5);
        mirror_cotangent(mir[n - 1], lam);
    }
    double ybar[6];
    double kb = 0.0;
    double sstar = h[n - 1];
    if (event) {
        double y5[6], d5[6];
        ck_eval(&g, kappa, yl, h[n - 1], y5, d5);
        if (!(sphere_g_xyz(c, R, yl) < 0.0 && sphere_g_xyz(c, R, y5) >= 0.0)) {
            free(ys);
            free(mir);
            return -1;
        }
        sstar = locate_crossing(&g, kappa, yl, h[n - 1], c, R);
        /* psi = zbar . Phi_s + Lbar; combined cotangent zbar - (psi/g_s) dg/dz */
        dual yd[6], zs[6];
        for (int a = 0; a < 6; ++a)
            yd[a] = dl(yl[a], 0.0);
        ck_eval_dual(&g, NULL, kappa, yd, dl(sstar, 1.0), zs);
        double zn = sqrt(zs[3].v * zs[3].v + zs[4].v * zs[4].v + zs[5].v * zs[5].v);
        double u[3] = {zs[3].v / zn, zs[4].v / zn, zs[5].v / zn};
        double lu = lam[3] * u[0] + lam[4] * u[1] + lam[5] * u[2];
        double zbar[6] = {lam[0], lam[1], lam[2], (lam[3] - lu * u[0]) / zn, (lam[4] - lu * u[1]) / zn,
                          (lam[5] - lu * u[2]) / zn};
        double psi = Lbar, gs = 0.0, dg[6] = {0, 0, 0, 0, 0, 0};
        for (int a = 0; a < 6; ++a)
            psi += zbar[a] * zs[a].d;
        for (int a = 0; a < 3; ++a) {
            dg[a] = 2.0 * (zs[a].v - c[a]);
            gs += dg[a] * zs[a].d;
        }
        double comb[6];
        for (int a = 0; a < 6; ++a)
            comb[a] = -(psi / gs) * dg[a];
        step_vjp(&g, kappa, yl, sstar, lam, comb, ybar, gbar, &kb);
    } else {
        step_vjp(&g, kappa, yl, sstar, lam, NULL, ybar, gbar, &kb);
    }
    for (int64_t s = n - 2; s >= 0; --s) {
        double nb[6];
        mirror_cotangent(mir[s], ybar);
        step_vjp(&g, kappa, ys + 6 * s, h[s], ybar, NULL, nb, gbar, &kb);
        memcpy(ybar, nb, sizeof nb);
    }
    /* initial normalisation */
    double u[3] = {u0[0] / un, u0[1] / un, u0[2] / un};
    double lu = ybar[3] * u[0] + ybar[4] * u[1] + ybar[5] * u[2];
    for (int a = 0; a < 3; ++a) {
        u0bar[a] = (ybar[3 + a] - lu * u[a]) / un;
        x0bar[a] = ybar[a];
    }
    if (kappabar)
        *kappabar = kb;
    free(ys);
    free(mir);
    return 0;
}
