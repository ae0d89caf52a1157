/*
 * Independent FP64 CPU oracle for longitudinal macro-particle tracking.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code, header, table or constant with the
 * HIP path.
 *
 * What it computes (paper, section 1.1.2 "The Longitudinal Plane"): every
 * macro-particle carries a position z and a relative momentum deviation
 * delta; both are integrated turn by turn, independently per particle, by an
 * Euler-Cromer (first order), leap-frog (second order Verlet) or fourth-order
 * Runge-Kutta / Ruth scheme. The paper names the schemes but prints no map;
 * the map used here is the standard single-harmonic stationary RF bucket:
 *
 *   drift of weight w:  z     <- z - w * (eta * C) * delta
 *   kick  of weight w:  delta <- delta + w * A * sin(k * z)
 *   with A = q V / (beta p0 c)  (V in volts, p0 c in eV, so c cancels),
 *        k = 2 pi h / C,  eta = 1/gamma_t^2 - 1/gamma^2.
 *
 * The loop order follows the paper's sequential C code (section 2.3): the
 * turns outside, the particles inside. The particle loop may be split over
 * OpenMP threads because particles are independent during tracking
 * (section 2.3); results do not depend on the thread count.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no fast-math, no
 * FMA contraction), so every operation below rounds exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_EULER_CROMER = 0, OR_LEAPFROG = 1, OR_RUTH4 = 2, OR_RK4 = 3 };

/* Machine constants of one ring, derived once (the paper's profile, section
 * 2.2, shows the Python code re-deriving eta, beta, p0 on every call; they
 * are fixed for a stationary bucket). */
typedef struct {
    double gamma, beta, eta, A, k, D;
} or_consts;

static int or_make_consts(double C, double h, double V, double p0c, double m,
                          double gamma_t, double q, or_consts *c)
{
    if (!(C > 0.0) || !(h > 0.0) || !(p0c > 0.0) || !(m >= 0.0) ||
        !(gamma_t > 0.0) || !isfinite(C) || !isfinite(h) || !isfinite(V) ||
        !isfinite(p0c) || !isfinite(m) || !isfinite(gamma_t) || !isfinite(q))
        return -1;
    /* total energy E = sqrt(p^2 + m^2) (units of eV), gamma = E/m, beta = p/E */
    double E = sqrt(p0c * p0c + m * m);
    c->gamma = E / m; /* +inf for m = 0 */
    c->beta = p0c / E;
    c->eta = 1.0 / (gamma_t * gamma_t) - 1.0 / (c->gamma * c->gamma);
    c->A = q * V / (c->beta * p0c);
    c->k = 2.0 * M_PI * h / C;
    c->D = c->eta * C;
    return 0;
}

/* Derived quantities for reports and tests, in this order:
 * gamma, beta, eta, A, k, D, omega_s (small-amplitude angular frequency per
 * turn of the smooth motion), Q_s = omega_s / 2pi, Q of the linearised
 * leap-frog map (cos mu = 1 - omega^2/2), bucket half-length C/(2h),
 * bucket half-height, separatrix Hamiltonian H_sep.
 * The smooth Hamiltonian with one turn as the time unit is
 *   H(z, delta) = -(D/2) delta^2 + (A/k) (cos(k z) - 1),
 * whose unstable fixed point z = C/(2h) gives H_sep = -2A/k. */
int oracle_derive(double C, double h, double V, double p0c, double m,
                  double gamma_t, double q, double out[12])
{
    or_consts c;
    if (or_make_consts(C, h, V, p0c, m, gamma_t, q, &c) != 0)
        return -1;
    double w2 = c.A * c.k * c.D;
    double omega = sqrt(fabs(w2));
    out[0] = c.gamma;
    out[1] = c.beta;
    out[2] = c.eta;
    out[3] = c.A;
    out[4] = c.k;
    out[5] = c.D;
    out[6] = omega;
    out[7] = omega / (2.0 * M_PI);
    /* mu = 2 asin(omega/2) is the same angle as acos(1 - omega^2/2) */
    out[8] = 2.0 * asin(omega / 2.0) / (2.0 * M_PI);
    out[9] = C / (2.0 * h);
    out[10] = 2.0 * sqrt(fabs(c.A / (c.k * c.D)));
    out[11] = -2.0 * c.A / c.k;
    return 0;
}

static void drift(const or_consts *c, double w, double *z, double dp)
{
    *z = *z - (w * c->D) * dp;
}

static void kick(const or_consts *c, double w, double z, double *dp)
{
    *dp = *dp + (w * c->A) * sin(c->k * z);
}

/* Fourth-order symplectic composition of Forest & Ruth (1990), identical to
 * Yoshida's (1990) triple-jump of the leap-frog step. */
static double ruth_theta(void)
{
    return 1.0 / (2.0 - cbrt(2.0));
}

/* One integration step of length w (in turns) of the chosen scheme. */
static void step(const or_consts *c, int integrator, double w, double *z, double *dp)
{
    switch (integrator) {
    case OR_EULER_CROMER: /* symplectic Euler: drift, then kick */
        drift(c, w, z, *dp);
        kick(c, w, *z, dp);
        break;
    case OR_LEAPFROG: /* Verlet: half drift, kick, half drift */
        drift(c, 0.5 * w, z, *dp);
        kick(c, w, *z, dp);
        drift(c, 0.5 * w, z, *dp);
        break;
    case OR_RUTH4: {
        double th = ruth_theta();
        drift(c, 0.5 * th * w, z, *dp);
        kick(c, th * w, *z, dp);
        drift(c, 0.5 * (1.0 - th) * w, z, *dp);
        kick(c, (1.0 - 2.0 * th) * w, *z, dp);
        drift(c, 0.5 * (1.0 - th) * w, z, *dp);
        kick(c, th * w, *z, dp);
        drift(c, 0.5 * th * w, z, *dp);
        break;
    }
    case OR_RK4: {
        /* classical Runge-Kutta on dz/dn = -D delta, d(delta)/dn = A sin(k z) */
        double z0 = *z, d0 = *dp;
        double k1z = -c->D * d0, k1d = c->A * sin(c->k * z0);
        double z2 = z0 + 0.5 * w * k1z, d2 = d0 + 0.5 * w * k1d;
        double k2z = -c->D * d2, k2d = c->A * sin(c->k * z2);
        double z3 = z0 + 0.5 * w * k2z, d3 = d0 + 0.5 * w * k2d;
        double k3z = -c->D * d3, k3d = c->A * sin(c->k * z3);
        double z4 = z0 + w * k3z, d4 = d0 + w * k3d;
        double k4z = -c->D * d4, k4d = c->A * sin(c->k * z4);
        *z = z0 + (w / 6.0) * (k1z + 2.0 * k2z + 2.0 * k3z + k4z);
        *dp = d0 + (w / 6.0) * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
        break;
    }
    }
}

/* Neumaier's compensated summation (an improved Kahan-Babuska sum). */
typedef struct {
    double s, c;
} or_sum;

static void sum_add(or_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x))
        a->c += (a->s - t) + x;
    else
        a->c += (x - t) + a->s;
    a->s = t;
}

static double sum_value(const or_sum *a)
{
    return a->s + a->c;
}

/* Fixed chunking of the particle axis: chunk partial sums are combined in
 * chunk order, so the result does not depend on the thread count. */
#define OR_CHUNK 4096

/* Population moments of one bunch, two-pass and compensated:
 * out = {mean_z, rms_z, mean_dp, rms_dp, emit_rms} with
 *   rms_z^2 = sum (z - mean_z)^2 / n,  cov = sum (z - mean_z)(dp - mean_dp) / n,
 *   emit_rms = sqrt(max(0, rms_z^2 rms_dp^2 - cov^2))  [metres].
 * n = 0 gives NaN everywhere. */
void oracle_moments(const double *z, const double *dp, int64_t n, double out[5])
{
    if (n <= 0) {
        for (int i = 0; i < 5; ++i)
            out[i] = NAN;
        return;
    }
    int64_t nchunks = (n + OR_CHUNK - 1) / OR_CHUNK;
    or_sum sz = {0, 0}, sd = {0, 0};
#pragma omp parallel
    {
        /* each thread owns whole chunks; partials are merged in chunk order */
#pragma omp for ordered schedule(static, 1)
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            or_sum cz = {0, 0}, cd = {0, 0};
            int64_t hi = (ch + 1) * OR_CHUNK < n ? (ch + 1) * OR_CHUNK : n;
            for (int64_t i = ch * OR_CHUNK; i < hi; ++i) {
                sum_add(&cz, z[i]);
                sum_add(&cd, dp[i]);
            }
#pragma omp ordered
            {
                sum_add(&sz, cz.s);
                sum_add(&sz, cz.c);
                sum_add(&sd, cd.s);
                sum_add(&sd, cd.c);
            }
        }
    }
    double mz = sum_value(&sz) / (double)n;
    double md = sum_value(&sd) / (double)n;
    or_sum szz = {0, 0}, sdd = {0, 0}, szd = {0, 0};
#pragma omp parallel
    {
#pragma omp for ordered schedule(static, 1)
        for (int64_t ch = 0; ch < nchunks; ++ch) {
            or_sum czz = {0, 0}, cdd = {0, 0}, czd = {0, 0};
            int64_t hi = (ch + 1) * OR_CHUNK < n ? (ch + 1) * OR_CHUNK : n;
            for (int64_t i = ch * OR_CHUNK; i < hi; ++i) {
                double a = z[i] - mz, b = dp[i] - md;
                sum_add(&czz, a * a);
                sum_add(&cdd, b * b);
                sum_add(&czd, a * b);
            }
#pragma omp ordered
            {
                sum_add(&szz, czz.s);
                sum_add(&szz, czz.c);
                sum_add(&sdd, cdd.s);
                sum_add(&sdd, cdd.c);
                sum_add(&szd, czd.s);
                sum_add(&szd, czd.c);
            }
        }
    }
    double vz = sum_value(&szz) / (double)n;
    double vd = sum_value(&sdd) / (double)n;
    double cov = sum_value(&szd) / (double)n;
    double e2 = vz * vd - cov * cov;
    out[0] = mz;
    out[1] = sqrt(vz);
    out[2] = md;
    out[3] = sqrt(vd);
    out[4] = sqrt(e2 > 0.0 ? e2 : 0.0);
}

/* Track n particles for `turns` turns in place. Each turn is `substeps`
 * steps of length 1/substeps (substeps = 1 is the production map: one step
 * per turn). If `moments` is not NULL it receives turns rows of 5 values,
 * row t holding the moments after turn t+1. `threads` <= 0 means the OpenMP
 * default. Returns 0, or -1 for invalid arguments. */
int oracle_track(double *z, double *dp, int64_t n, int64_t turns, double C, double h,
                 double V, double p0c, double m, double gamma_t, double q, int integrator,
                 int substeps, double *moments, int threads)
{
    or_consts c;
    if (n < 0 || turns < 0 || substeps < 1 || integrator < 0 || integrator > 3)
        return -1;
    if (or_make_consts(C, h, V, p0c, m, gamma_t, q, &c) != 0)
        return -1;
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    double w = 1.0 / (double)substeps;
    for (int64_t t = 0; t < turns; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int s = 0; s < substeps; ++s)
                step(&c, integrator, w, &z[i], &dp[i]);
        }
        if (moments)
            oracle_moments(z, dp, n, moments + 5 * t);
    }
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return 0;
}

/* ------------------------------------------------------------------------
 * Extended map: double-harmonic RF with phase offsets and a slip factor
 * expanded in delta. The paper's hollow-bunch run applies two RF kicks and
 * two drifts per turn and re-evaluates eta and the RF phase at every step
 * (section 2.2, cProfile listing); the stationary form of that is
 *   drift of weight w:  z     <- z - w C (eta0 + eta1 delta + eta2 delta^2) delta
 *   kick  of weight w:  delta <- delta + w [A1 sin(k1 z + phi1) + A2 sin(k2 z + phi2)]
 * with A_i = q V_i / (beta p0 c), k_i = 2 pi h_i / C and eta0 as above. It is
 * the flow of H = -C (eta0 d^2/2 + eta1 d^3/3 + eta2 d^4/4)
 *               + sum_i (A_i / k_i) cos(k_i z + phi_i).
 * ---------------------------------------------------------------------- */
typedef struct {
    double C, eta0, eta1, eta2;
    double A1, k1, phi1;
    double A2, k2, phi2;
} or_rf2;

static void drift2(const or_rf2 *c, double w, double *z, double dp)
{
    double eta = c->eta0 + c->eta1 * dp + c->eta2 * dp * dp;
    *z = *z - (w * c->C) * eta * dp;
}

static double force2(const or_rf2 *c, double z)
{
    return c->A1 * sin(c->k1 * z + c->phi1) + c->A2 * sin(c->k2 * z + c->phi2);
}

static void kick2(const or_rf2 *c, double w, double z, double *dp)
{
    *dp = *dp + w * force2(c, z);
}

static double slip2(const or_rf2 *c, double dp)
{
    return -c->C * (c->eta0 + c->eta1 * dp + c->eta2 * dp * dp) * dp;
}

static void step2(const or_rf2 *c, int integrator, double w, double *z, double *dp)
{
    switch (integrator) {
    case OR_EULER_CROMER:
        drift2(c, w, z, *dp);
        kick2(c, w, *z, dp);
        break;
    case OR_LEAPFROG:
        drift2(c, 0.5 * w, z, *dp);
        kick2(c, w, *z, dp);
        drift2(c, 0.5 * w, z, *dp);
        break;
    case OR_RUTH4: {
        double th = ruth_theta();
        drift2(c, 0.5 * th * w, z, *dp);
        kick2(c, th * w, *z, dp);
        drift2(c, 0.5 * (1.0 - th) * w, z, *dp);
        kick2(c, (1.0 - 2.0 * th) * w, *z, dp);
        drift2(c, 0.5 * (1.0 - th) * w, z, *dp);
        kick2(c, th * w, *z, dp);
        drift2(c, 0.5 * th * w, z, *dp);
        break;
    }
    case OR_RK4: {
        double z0 = *z, d0 = *dp;
        double k1z = slip2(c, d0), k1d = force2(c, z0);
        double k2z = slip2(c, d0 + 0.5 * w * k1d), k2d = force2(c, z0 + 0.5 * w * k1z);
        double k3z = slip2(c, d0 + 0.5 * w * k2d), k3d = force2(c, z0 + 0.5 * w * k2z);
        double k4z = slip2(c, d0 + w * k3d), k4d = force2(c, z0 + w * k3z);
        *z = z0 + (w / 6.0) * (k1z + 2.0 * k2z + 2.0 * k3z + k4z);
        *dp = d0 + (w / 6.0) * (k1d + 2.0 * k2d + 2.0 * k3d + k4d);
        break;
    }
    }
}

/* As oracle_track for the extended map. h2 and V2 describe the second
 * harmonic (V2 = 0: none); phi1, phi2 in radians. */
int oracle_track_rf2(double *z, double *dp, int64_t n, int64_t turns, double C, double h,
                     double V, double p0c, double m, double gamma_t, double q, double phi1,
                     double h2, double V2, double phi2, double eta1, double eta2,
                     int integrator, int substeps, double *moments, int threads)
{
    or_consts b;
    if (n < 0 || turns < 0 || substeps < 1 || integrator < 0 || integrator > 3)
        return -1;
    if (or_make_consts(C, h, V, p0c, m, gamma_t, q, &b) != 0)
        return -1;
    if (!isfinite(phi1) || !isfinite(h2) || !isfinite(V2) || !isfinite(phi2) ||
        !isfinite(eta1) || !isfinite(eta2) || (V2 != 0.0 && !(h2 > 0.0)))
        return -1;
    or_rf2 c;
    c.C = C;
    c.eta0 = b.eta;
    c.eta1 = eta1;
    c.eta2 = eta2;
    c.A1 = b.A;
    c.k1 = b.k;
    c.phi1 = phi1;
    c.A2 = q * V2 / (b.beta * p0c);
    c.k2 = 2.0 * M_PI * h2 / C;
    c.phi2 = phi2;
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    double w = 1.0 / (double)substeps;
    for (int64_t t = 0; t < turns; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int s = 0; s < substeps; ++s)
                step2(&c, integrator, w, &z[i], &dp[i]);
        }
        if (moments)
            oracle_moments(z, dp, n, moments + 5 * t);
    }
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return 0;
}

/* ------------------------------------------------------------------------
 * RF programme: the extended map with per-turn RF voltages and phases and a
 * per-turn reference momentum (the "parameter changes of the accelerator
 * setting" of the paper's hollow-bunch run, section 2.2).
 *
 * Turn n runs from reference momentum p_a = p(n) to p_b = p(n+1) (p(0) is the
 * ring's p0c, p(n+1) the programme's entry n) with the RF settings of entry
 * n. The RF gives a particle the energy q sum_i V_i sin(k_i z + phi_i), i.e.
 * the momentum (energy gain) / beta_a with beta_a the reference beta at p_a;
 * the reference itself gains p_b - p_a over the turn. Each kick of weight w
 * (the scheme's kick weights sum to one) carries the fraction w of both, so
 * the reference moves p_cur -> p_new = p_cur + w (p_b - p_a) and
 *   absolute momentum:  P' = P + w q sum_i V_i sin(k_i z + phi_i) / beta_a,
 *   with P = p_cur (1 + delta) and delta' = P' / p_new - 1, i.e.
 *   delta' = (p_cur / p_new) delta + (p_cur - p_new) / p_new
 *            + w q sum_i V_i sin(k_i z + phi_i) / (beta_a p_new)
 * (the same expression rearranged so that delta never passes through 1 +
 * delta, which would cost ~1e-13 of its relative precision per kick). A
 * drift uses eta0 at the reference momentum current at that point of the
 * turn. With p constant this is the extended map above with the entry's
 * voltages and phases; a particle at z = 0, delta = 0 stays there when
 * q V1 sin(phi1) / beta_a = p_b - p_a (the synchronous phase).
 * RK4 integrates a vector field at fixed parameters and supports only
 * programmes with a constant reference momentum.
 * ---------------------------------------------------------------------- */
typedef struct {
    double C, m, gamma_t, q, eta1, eta2, k1, k2;
    /* this turn */
    double V1, phi1, V2, phi2, beta_a, p_a, p_b;
} or_prog;

static double eta0_at(const or_prog *c, double p)
{
    double E = sqrt(p * p + c->m * c->m);
    double gamma = E / c->m;
    return 1.0 / (c->gamma_t * c->gamma_t) - 1.0 / (gamma * gamma);
}

static void drift_p(const or_prog *c, double w, double p_ref, double *z, double dp)
{
    double eta = eta0_at(c, p_ref) + c->eta1 * dp + c->eta2 * dp * dp;
    *z = *z - (w * c->C) * eta * dp;
}

/* q sum_i V_i sin(k_i z + phi_i): energy gain in eV */
static double energy_gain(const or_prog *c, double z)
{
    return c->q * (c->V1 * sin(c->k1 * z + c->phi1) + c->V2 * sin(c->k2 * z + c->phi2));
}

static void kick_p(const or_prog *c, double w, double p_cur, double p_new, double z, double *dp)
{
    *dp = (p_cur / p_new) * *dp + (p_cur - p_new) / p_new +
          w * energy_gain(c, z) / (c->beta_a * p_new);
}

/* One step of length w turns, during which the reference goes from p0 to p1. */
static void step_p(const or_prog *c, int integrator, double w, double p0, double p1, double *z,
                   double *dp)
{
    double dpr = p1 - p0;
    switch (integrator) {
    case OR_EULER_CROMER:
        drift_p(c, w, p0, z, *dp);
        kick_p(c, w, p0, p1, *z, dp);
        break;
    case OR_LEAPFROG:
        drift_p(c, 0.5 * w, p0, z, *dp);
        kick_p(c, w, p0, p1, *z, dp);
        drift_p(c, 0.5 * w, p1, z, *dp);
        break;
    case OR_RUTH4: {
        double th = ruth_theta();
        double q1 = p0 + th * dpr, q2 = p0 + (1.0 - th) * dpr;
        drift_p(c, 0.5 * th * w, p0, z, *dp);
        kick_p(c, th * w, p0, q1, *z, dp);
        drift_p(c, 0.5 * (1.0 - th) * w, q1, z, *dp);
        kick_p(c, (1.0 - 2.0 * th) * w, q1, q2, *z, dp);
        drift_p(c, 0.5 * (1.0 - th) * w, q2, z, *dp);
        kick_p(c, th * w, q2, p1, *z, dp);
        drift_p(c, 0.5 * th * w, p1, z, *dp);
        break;
    }
    case OR_RK4: { /* constant reference momentum only (checked by the caller) */
        or_rf2 f;
        f.C = c->C;
        f.eta0 = eta0_at(c, p0);
        f.eta1 = c->eta1;
        f.eta2 = c->eta2;
        f.A1 = c->q * c->V1 / (c->beta_a * p0);
        f.k1 = c->k1;
        f.phi1 = c->phi1;
        f.A2 = c->q * c->V2 / (c->beta_a * p0);
        f.k2 = c->k2;
        f.phi2 = c->phi2;
        step2(&f, OR_RK4, w, z, dp);
        break;
    }
    }
}

/* As oracle_track_rf2 with per-turn settings: entry t of V1, phi1, V2, phi2
 * applies to turn t, and p0c_after[t] is the reference momentum (eV) after
 * turn t; p0c is the momentum before the first turn. Substeps split a turn
 * into equal steps and its momentum step into equal parts. Returns -1 for
 * invalid arguments, RK4 with a changing momentum included. */
int oracle_track_program(double *z, double *dp, int64_t n, int64_t turns, double C, double h,
                         double p0c, double m, double gamma_t, double q, double h2,
                         double eta1, double eta2, const double *V1, const double *phi1,
                         const double *V2, const double *phi2, const double *p0c_after,
                         int integrator, int substeps, double *moments, int threads)
{
    or_consts b;
    if (n < 0 || turns < 0 || substeps < 1 || integrator < 0 || integrator > 3)
        return -1;
    if (or_make_consts(C, h, 0.0, p0c, m, gamma_t, q, &b) != 0)
        return -1;
    if (!isfinite(h2) || !isfinite(eta1) || !isfinite(eta2))
        return -1;
    for (int64_t t = 0; t < turns; ++t) {
        if (!isfinite(V1[t]) || !isfinite(phi1[t]) || !isfinite(V2[t]) || !isfinite(phi2[t]) ||
            !(p0c_after[t] > 0.0) || !isfinite(p0c_after[t]) || (V2[t] != 0.0 && !(h2 > 0.0)))
            return -1;
        double before = t == 0 ? p0c : p0c_after[t - 1];
        if (integrator == OR_RK4 && p0c_after[t] != before)
            return -1;
    }
    or_prog c;
    c.C = C;
    c.m = m;
    c.gamma_t = gamma_t;
    c.q = q;
    c.eta1 = eta1;
    c.eta2 = eta2;
    c.k1 = b.k;
    c.k2 = 2.0 * M_PI * h2 / C;
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    double w = 1.0 / (double)substeps;
    for (int64_t t = 0; t < turns; ++t) {
        c.V1 = V1[t];
        c.phi1 = phi1[t];
        c.V2 = V2[t];
        c.phi2 = phi2[t];
        c.p_a = t == 0 ? p0c : p0c_after[t - 1];
        c.p_b = p0c_after[t];
        c.beta_a = c.p_a / sqrt(c.p_a * c.p_a + m * m);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            for (int s = 0; s < substeps; ++s) {
                double pa = c.p_a + (c.p_b - c.p_a) * ((double)s / substeps);
                double pb = s + 1 == substeps ? c.p_b
                                              : c.p_a + (c.p_b - c.p_a) * ((double)(s + 1) / substeps);
                step_p(&c, integrator, w, pa, pb, &z[i], &dp[i]);
            }
        }
        if (moments)
            oracle_moments(z, dp, n, moments + 5 * t);
    }
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return 0;
}

/* ------------------------------------------------------------------------
 * Transverse linear one-turn map (paper, section 1.1.1: the same linear
 * transfer matrix acts on every particle's transverse state each turn),
 * with the chromatic phase advance that couples it to the longitudinal
 * momentum. Per plane u in {x, y}, with the Twiss parameters alpha, beta
 * (gamma = (1 + alpha^2) / beta) at the observation point, tune Q and
 * chromaticity Q' (tune shift per unit delta):
 *   phi = 2 pi (Q + Q' delta)
 *   u   <- (cos phi + alpha sin phi) u + beta sin phi u'
 *   u'  <- -gamma sin phi u + (cos phi - alpha sin phi) u'
 * One turn applies the transverse map with the turn's starting delta, then
 * the longitudinal step of the extended map.
 * ---------------------------------------------------------------------- */
typedef struct {
    double Q, Qp, alpha, beta, gamma;
} or_plane;

/* The rotation depends on the tune modulo one: the integer part is dropped
 * exactly (Q - floor(Q) has no rounding error) before the phase is formed,
 * so its rounding is that of a phase below 2 pi rather than of 2 pi Q. */
static void transverse(const or_plane *p, double dp, double *u, double *up)
{
    double phi = 2.0 * M_PI * ((p->Q - floor(p->Q)) + p->Qp * dp);
    double c = cos(phi), s = sin(phi);
    double u0 = *u, v0 = *up;
    *u = (c + p->alpha * s) * u0 + p->beta * s * v0;
    *up = -p->gamma * s * u0 + (c - p->alpha * s) * v0;
}

/* As oracle_track_rf2 with a transverse state (x, xp, y, yp) besides (z, dp).
 * `tw` = {Qx, Qpx, alpha_x, beta_x, Qy, Qpy, alpha_y, beta_y}. If `moments`
 * is not NULL it receives turns rows of 15 values: the 5 moments of (z, dp),
 * then of (x, xp), then of (y, yp), each as oracle_moments. */
int oracle_track_6d(double *z, double *dp, double *x, double *xp, double *y, double *yp,
                    int64_t n, int64_t turns, double C, double h, double V, double p0c,
                    double m, double gamma_t, double q, double phi1, double h2, double V2,
                    double phi2, double eta1, double eta2, const double tw[8], int integrator,
                    double *moments, int threads)
{
    or_consts b;
    if (n < 0 || turns < 0 || integrator < 0 || integrator > 3)
        return -1;
    if (or_make_consts(C, h, V, p0c, m, gamma_t, q, &b) != 0)
        return -1;
    if (!isfinite(phi1) || !isfinite(h2) || !isfinite(V2) || !isfinite(phi2) ||
        !isfinite(eta1) || !isfinite(eta2) || (V2 != 0.0 && !(h2 > 0.0)))
        return -1;
    for (int i = 0; i < 8; ++i)
        if (!isfinite(tw[i]))
            return -1;
    if (!(tw[3] > 0.0) || !(tw[7] > 0.0))
        return -1;
    or_rf2 c;
    c.C = C;
    c.eta0 = b.eta;
    c.eta1 = eta1;
    c.eta2 = eta2;
    c.A1 = b.A;
    c.k1 = b.k;
    c.phi1 = phi1;
    c.A2 = q * V2 / (b.beta * p0c);
    c.k2 = 2.0 * M_PI * h2 / C;
    c.phi2 = phi2;
    or_plane px = {tw[0], tw[1], tw[2], tw[3], (1.0 + tw[2] * tw[2]) / tw[3]};
    or_plane py = {tw[4], tw[5], tw[6], tw[7], (1.0 + tw[6] * tw[6]) / tw[7]};
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    for (int64_t t = 0; t < turns; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            transverse(&px, dp[i], &x[i], &xp[i]);
            transverse(&py, dp[i], &y[i], &yp[i]);
            step2(&c, integrator, 1.0, &z[i], &dp[i]);
        }
        if (moments) {
            oracle_moments(z, dp, n, moments + 15 * t);
            oracle_moments(x, xp, n, moments + 15 * t + 5);
            oracle_moments(y, yp, n, moments + 15 * t + 10);
        }
    }
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    return 0;
}

/* ------------------------------------------------------------------------
 * Longitudinal wake kick (the impedance effects the paper's conclusion names
 * as the memory-bound next step, section 3). Once per turn, after the map
 * step: the bunch is cut into n_slices equal slices over [z_lo, z_hi)
 * (particles outside are neither counted nor kicked); the wake potential at
 * slice centre c_k is
 *   V_k = Q_mp sum_{j >= k} count_j W((c_j - c_k) / (beta c)),
 * the charge of every slice at or ahead of it (z grows toward the head)
 * times the wake function, Q_mp = q e N_b / N_mp the charge of one
 * macro-particle; a particle at z gets V(z) by linear interpolation between
 * the centres (constant beyond the first and last centre) and
 *   delta <- delta - q V(z) / (beta p0 c)      (V in volts, p0 c in eV).
 * Wake function of a resonator (shunt impedance R_s, resonance frequency
 * f_r = omega_r / 2 pi, quality factor Q > 1/2), alpha = omega_r / (2 Q),
 * omega' = sqrt(omega_r^2 - alpha^2):
 *   W(tau) = 2 alpha R_s exp(-alpha tau) (cos omega' tau - alpha/omega' sin omega' tau), tau > 0,
 *   W(0)   = alpha R_s (half the limit: a charge sees half its own wake).
 * model 1 is a constant wake W(tau > 0) = R_s, W(0) = R_s / 2 (the potential
 * is then the charge ahead; used to pin the slicing).
 * ---------------------------------------------------------------------- */
typedef struct {
    int model;
    double Rs, alpha, omega_bar;
    double kappa;           /* q Q_mp / (beta p0 c): delta kick per volt of potential per count */
    double z_lo, dz;        /* slice edges z_lo + k dz */
    double per_dz;          /* n_slices / (z_hi - z_lo): slice coordinate per metre */
    int64_t n_slices;
    double tau_per_slice;   /* dz / (beta c) */
} or_wake;

static double wake_fn(const or_wake *w, double tau)
{
    if (w->model == 1)
        return tau > 0.0 ? w->Rs : 0.5 * w->Rs;
    if (tau == 0.0)
        return w->alpha * w->Rs;
    return 2.0 * w->alpha * w->Rs * exp(-w->alpha * tau) *
           (cos(w->omega_bar * tau) - w->alpha / w->omega_bar * sin(w->omega_bar * tau));
}

/* Slice of z, or -1 outside the slices. The slice coordinate of z is
 * u = (z - z_lo) * per_dz, a difference and a product each rounded once;
 * slice k holds the u in [k, k + 1). */
static int64_t slice_of(const or_wake *w, double z)
{
    double u = (z - w->z_lo) * w->per_dz;
    if (!(u >= 0.0))
        return -1;
    double f = floor(u);
    if (f >= (double)w->n_slices)
        return -1;
    return (int64_t)f;
}

/* Wm[m] = W(m dz / (beta c)): the wake at the lags between slice centres. */
static void wake_kick(const or_wake *w, const double *Wm, const double *z, double *dp, int64_t n,
                      int64_t *count, double *V)
{
    int64_t ns = w->n_slices;
    for (int64_t k = 0; k < ns; ++k)
        count[k] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t k = slice_of(w, z[i]);
        if (k >= 0)
            count[k] += 1;
    }
    for (int64_t k = 0; k < ns; ++k) {
        double v = 0.0;
        for (int64_t j = k; j < ns; ++j)
            v += (double)count[j] * Wm[j - k];
        V[k] = v;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (slice_of(w, z[i]) < 0)
            continue;
        double s = (z[i] - w->z_lo) * w->per_dz - 0.5; /* in slice-centre units */
        double pot;
        if (s <= 0.0) {
            pot = V[0];
        } else if (s >= (double)(ns - 1)) {
            pot = V[ns - 1];
        } else {
            double k0 = floor(s);
            double f = s - k0;
            int64_t k = (int64_t)k0;
            pot = (1.0 - f) * V[k] + f * V[k + 1];
        }
        dp[i] = dp[i] - w->kappa * pot;
    }
}

/* As oracle_track_rf2 with a wake kick after every map step. wk = {model,
 * R_s (ohm; model 1: V/C), f_r (Hz), Q, N_b (particles in the bunch),
 * n_slices, z_lo, z_hi}. */
int oracle_track_wake(double *z, double *dp, int64_t n, int64_t turns, double C, double h,
                      double V, double p0c, double m, double gamma_t, double q, double phi1,
                      double h2, double V2, double phi2, double eta1, double eta2,
                      const double wk[8], int integrator, double *moments, int threads)
{
    or_consts b;
    if (n < 0 || turns < 0 || integrator < 0 || integrator > 3)
        return -1;
    if (or_make_consts(C, h, V, p0c, m, gamma_t, q, &b) != 0)
        return -1;
    if (!isfinite(phi1) || !isfinite(h2) || !isfinite(V2) || !isfinite(phi2) ||
        !isfinite(eta1) || !isfinite(eta2) || (V2 != 0.0 && !(h2 > 0.0)))
        return -1;
    for (int i = 0; i < 8; ++i)
        if (!isfinite(wk[i]))
            return -1;
    int model = (int)wk[0];
    int64_t ns = (int64_t)wk[5];
    if ((model != 0 && model != 1) || (double)model != wk[0] || (double)ns != wk[5] || ns < 1 ||
        ns > (1 << 20) || !(wk[7] > wk[6]) || !(wk[4] >= 0.0) ||
        (model == 0 && (!(wk[2] > 0.0) || !(wk[3] > 0.5))))
        return -1;
    or_rf2 c;
    c.C = C;
    c.eta0 = b.eta;
    c.eta1 = eta1;
    c.eta2 = eta2;
    c.A1 = b.A;
    c.k1 = b.k;
    c.phi1 = phi1;
    c.A2 = q * V2 / (b.beta * p0c);
    c.k2 = 2.0 * M_PI * h2 / C;
    c.phi2 = phi2;
    const double e_charge = 1.602176634e-19, c_light = 299792458.0;
    or_wake w;
    w.model = model;
    w.Rs = wk[1];
    double omega_r = 2.0 * M_PI * wk[2];
    w.alpha = model == 0 ? omega_r / (2.0 * wk[3]) : 0.0;
    w.omega_bar = model == 0 ? sqrt(omega_r * omega_r - w.alpha * w.alpha) : 0.0;
    w.n_slices = ns;
    w.z_lo = wk[6];
    w.dz = (wk[7] - wk[6]) / (double)ns;
    w.per_dz = (double)ns / (wk[7] - wk[6]);
    w.tau_per_slice = w.dz / (b.beta * c_light);
    double q_mp = n > 0 ? q * e_charge * wk[4] / (double)n : 0.0;
    w.kappa = q * q_mp / (b.beta * p0c);
    int64_t *count = (int64_t *)malloc(sizeof(int64_t) * (size_t)ns);
    double *Vk = (double *)malloc(sizeof(double) * (size_t)ns);
    double *Wm = (double *)malloc(sizeof(double) * (size_t)ns);
    if (!count || !Vk || !Wm) {
        free(count);
        free(Vk);
        free(Wm);
        return -1;
    }
    for (int64_t k = 0; k < ns; ++k)
        Wm[k] = wake_fn(&w, (double)k * w.tau_per_slice);
#ifdef _OPENMP
    int saved = omp_get_max_threads();
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
    for (int64_t t = 0; t < turns; ++t) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            step2(&c, integrator, 1.0, &z[i], &dp[i]);
        wake_kick(&w, Wm, z, dp, n, count, Vk);
        if (moments)
            oracle_moments(z, dp, n, moments + 5 * t);
    }
#ifdef _OPENMP
    omp_set_num_threads(saved);
#endif
    free(count);
    free(Vk);
    free(Wm);
    return 0;
}

/* Number of OpenMP threads a parallel region would use right now. */
int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
