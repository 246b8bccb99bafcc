/*
 * u1ml_oracle.c -- plain FP64 CPU oracle for multilevel compact U(1) lattice
 * gauge theory in 3+1 dimensions (Amado, Cardoso, Cardoso, Bicudo,
 * "Study of compact U(1) flux tubes in 3+1 dimensions in lattice gauge theory
 * using GPU's", arXiv:1208.0166).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker that the GPU library is
 * compared against.  It is loaded by the tests, by the smoke check and by the
 * CPU-baseline leg of the benchmark, and by nothing else; the product library
 * neither links nor calls it, and it shares no code with the GPU sources.
 *
 * Everything here is written for clarity, not speed: links are stored as FP64
 * angles in the natural order theta[t][z][y][x][mu], every observable is its
 * textbook definition, and the multilevel estimators keep one accumulator per
 * source position exactly as in Eq. (9).  Build with
 *     gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC
 * (no fused multiply-add, no fast-math) so that every floating-point step is
 * one IEEE-754 operation in program order.
 *
 * Readings of the paper taken here (the paper leaves these open):
 *  - mu = 0 is time (the temporal links are written U_0 in Eq. (8)),
 *    mu = 1,2,3 are x,y,z; site (t,x,y,z) has canonical index
 *    n = ((t*L + z)*L + y)*L + x and parity (t+x+y+z) mod 2.
 *  - One "iterate" (Sec. 2.1) is one compound sweep: one Metropolis pass
 *    (n_metro hits per link, proposal theta + eps*U(-1,1)) followed by n_or
 *    overrelaxation passes.  A pass visits the eight checkerboard classes in
 *    the order mu = 0..3 (outer), parity 0,1 (inner).
 *  - Random numbers: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *    key = (seed, 0); counter = (n, purpose<<32 | hit<<8 | mu, pass_id, 0)
 *    with purpose 1 = hot start, 2 = Metropolis; pass_id counts Metropolis
 *    passes in program order.  Uniforms are (w >> 11) * 2^-53.
 *  - The multilevel method (Sec. 2.2) freezes, at a level of slab thickness
 *    th, the spatial links U_i(x,t) with t = 0 (mod th); every other link is
 *    updated.  Each level iteration is "update, then measure/recurse"; the
 *    chain is never restored.
 *  - sin, cos and atan2 inside the link updates are evaluated by the small
 *    routines below (Cody-Waite argument reduction plus Taylor / Gregory
 *    series in Horner form, only IEEE +,-,*,/), so that the update sequence is
 *    a fixed function of the inputs on any IEEE-754 machine.  Measurements
 *    use the C library.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_PI 3.14159265358979311600e+00 /* the double nearest pi */
#define OR_TWO_PI (2.0 * OR_PI)

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon et al., SC'11): multipliers and Weyl increments as   */
/* published there.                                                           */
/* ------------------------------------------------------------------------ */
static const uint64_t PHILOX_M0 = 0xD2E7470EE14C6C93ULL;
static const uint64_t PHILOX_M1 = 0xCA5A826395121157ULL;
static const uint64_t PHILOX_W0 = 0x9E3779B97F4A7C15ULL;
static const uint64_t PHILOX_W1 = 0xBB67AE8584CAA73BULL;

void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4])
{
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        unsigned __int128 p0 = (unsigned __int128)PHILOX_M0 * x0;
        unsigned __int128 p1 = (unsigned __int128)PHILOX_M1 * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ x1 ^ k0;
        uint64_t n2 = hi0 ^ x3 ^ k1;
        x0 = n0;
        x1 = lo1;
        x2 = n2;
        x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static double u01(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------------ */
/* Elementary functions used by the link updates.                             */
/* ------------------------------------------------------------------------ */
/* pi/2 = P1 + P2 + P3: P1 and P2 carry 32 significant bits each, so k*P1 and
 * k*P2 are exact for |k| < 2^20 (Cody & Waite reduction). */
static const double CW_P1 = 0x1.921fb544p+0;
static const double CW_P2 = 0x1.0b4611a6p-34;
static const double CW_P3 = 0x1.3198a2e037073p-69;
static const double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
static const double TAN_PI_8 = 0x1.a827999fcef32p-2; /* sqrt(2) - 1 */

/* sin(x), cos(x) for |x| < 1e6: x = k*pi/2 + r, |r| <= pi/4, then the Taylor
 * series of sin r (through r^19) and cos r (through r^18) by Horner's rule. */
void or_sincos(double x, double *s, double *c)
{
    double q = x * TWO_OVER_PI;
    int k = (int)(q >= 0.0 ? q + 0.5 : q - 0.5);
    double kd = (double)k;
    double r = ((x - kd * CW_P1) - kd * CW_P2) - kd * CW_P3;
    double z = r * r;
    double ps = -1.0 / 121645100408832000.0;     /* -1/19! */
    ps = ps * z + 1.0 / 355687428096000.0;       /* +1/17! */
    ps = ps * z - 1.0 / 1307674368000.0;         /* -1/15! */
    ps = ps * z + 1.0 / 6227020800.0;            /* +1/13! */
    ps = ps * z - 1.0 / 39916800.0;              /* -1/11! */
    ps = ps * z + 1.0 / 362880.0;                /* +1/9!  */
    ps = ps * z - 1.0 / 5040.0;                  /* -1/7!  */
    ps = ps * z + 1.0 / 120.0;                   /* +1/5!  */
    ps = ps * z - 1.0 / 6.0;                     /* -1/3!  */
    double sn = r + (r * z) * ps;
    double pc = 1.0 / 6402373705728000.0;        /* +1/18! */
    pc = pc * z - 1.0 / 20922789888000.0;        /* -1/16! */
    pc = pc * z + 1.0 / 87178291200.0;           /* +1/14! */
    pc = pc * z - 1.0 / 479001600.0;             /* -1/12! */
    pc = pc * z + 1.0 / 3628800.0;               /* +1/10! */
    pc = pc * z - 1.0 / 40320.0;                 /* -1/8!  */
    pc = pc * z + 1.0 / 720.0;                   /* +1/6!  */
    pc = pc * z - 1.0 / 24.0;                    /* -1/4!  */
    pc = pc * z + 1.0 / 2.0;                     /* +1/2!  */
    double cs = 1.0 - z * pc;
    switch (k & 3) {
    case 0: *s = sn;  *c = cs;  break;
    case 1: *s = cs;  *c = -sn; break;
    case 2: *s = -sn; *c = -cs; break;
    default: *s = -cs; *c = sn; break;
    }
}

/* atan2(y, x): fold into t = min/max in [0,1]; for t > tan(pi/8) use
 * atan t = pi/4 + atan((t-1)/(t+1)); then the Gregory series through u^39. */
double or_atan2(double y, double x)
{
    double ax = fabs(x), ay = fabs(y);
    if (ax == 0.0 && ay == 0.0) return 0.0;
    int swap = ay > ax;
    double t = swap ? ax / ay : ay / ax;
    double base = 0.0, u = t;
    if (t > TAN_PI_8) {
        u = (t - 1.0) / (t + 1.0);
        base = OR_PI / 4.0;
    }
    double z = u * u;
    double p = -1.0 / 39.0;
    for (int k = 37; k >= 3; k -= 2) {
        double a = 1.0 / (double)k;
        p = p * z + ((k & 2) ? -a : a); /* (-1)^((k-1)/2) / k */
    }
    double a = base + (u + (u * z) * p);
    if (swap) a = OR_PI / 2.0 - a;
    if (x < 0.0) a = OR_PI - a;
    if (y < 0.0) a = -a;
    return a;
}

static double wrap_angle(double a)
{
    while (a >= OR_PI) a -= OR_TWO_PI;
    while (a < -OR_PI) a += OR_TWO_PI;
    return a;
}

/* ------------------------------------------------------------------------ */
/* Lattice.                                                                    */
/* ------------------------------------------------------------------------ */
typedef struct or_lat {
    int L, T;
    long V;         /* L^3 * T sites */
    double beta;    /* 1/g^2, Eq. (3) */
    double eps;     /* Metropolis proposal half-width */
    uint64_t seed;
    uint64_t pass_id;
    double *th;     /* th[4*n + mu] */
} or_lat;

static long site_index(const or_lat *g, int t, int x, int y, int z)
{
    int L = g->L, T = g->T;
    t = ((t % T) + T) % T;
    x = ((x % L) + L) % L;
    y = ((y % L) + L) % L;
    z = ((z % L) + L) % L;
    return (((long)t * L + z) * L + y) * L + x;
}

static void site_coords(const or_lat *g, long n, int c[4])
{
    int L = g->L;
    c[1] = (int)(n % L); n /= L;
    c[2] = (int)(n % L); n /= L;
    c[3] = (int)(n % L); n /= L;
    c[0] = (int)n;
}

static long shifted(const or_lat *g, const int c[4], int d0, int d1, int d2, int d3)
{
    return site_index(g, c[0] + d0, c[1] + d1, c[2] + d2, c[3] + d3);
}

/* neighbour of site with coordinates c displaced by +a*e_mu + b*e_nu */
static long nbr(const or_lat *g, const int c[4], int mu, int a, int nu, int b)
{
    int d[4] = {0, 0, 0, 0};
    d[mu] += a;
    d[nu] += b;
    return shifted(g, c, d[0], d[1], d[2], d[3]);
}

static double TH(const or_lat *g, long n, int mu) { return g->th[4 * n + mu]; }

or_lat *or_create(int L, int T, double beta, double eps, uint64_t seed, int hot)
{
    if (L < 2 || T < 2 || (L & 1) || (T & 1)) return NULL;
    or_lat *g = (or_lat *)calloc(1, sizeof(or_lat));
    if (!g) return NULL;
    g->L = L; g->T = T;
    g->V = (long)L * L * L * T;
    g->beta = beta; g->eps = eps; g->seed = seed; g->pass_id = 0;
    g->th = (double *)calloc((size_t)4 * g->V, sizeof(double));
    if (!g->th) { free(g); return NULL; }
    if (hot) {
        /* hot start: theta = pi*(2u - 1), u from counter (n, 1<<32 | mu, 0, 0) */
        uint64_t key[2] = {seed, 0};
        for (long n = 0; n < g->V; ++n)
            for (int mu = 0; mu < 4; ++mu) {
                uint64_t ctr[4] = {(uint64_t)n, (1ULL << 32) | (uint64_t)mu, 0, 0};
                uint64_t w[4];
                or_philox4x64_10(ctr, key, w);
                g->th[4 * n + mu] = OR_PI * (2.0 * u01(w[0]) - 1.0);
            }
    }
    return g;
}

void or_destroy(or_lat *g)
{
    if (!g) return;
    free(g->th);
    free(g);
}

long or_volume(const or_lat *g) { return g->V; }

/* threads the OpenMP loops of the oracle use */
/* threads of the OpenMP loops that follow (results do not depend on it) */
void or_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int or_max_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
uint64_t or_get_pass_id(const or_lat *g) { return g->pass_id; }
void or_set_pass_id(or_lat *g, uint64_t p) { g->pass_id = p; }
void or_set_beta(or_lat *g, double beta) { g->beta = beta; }
void or_get_links(const or_lat *g, double *out) { memcpy(out, g->th, sizeof(double) * 4 * g->V); }
void or_set_links(or_lat *g, const double *in) { memcpy(g->th, in, sizeof(double) * 4 * g->V); }

/* ------------------------------------------------------------------------ */
/* Staple of link (n, mu): Wilson action Eq. (3), plaquette angle            */
/* theta_munu(x) = theta_mu(x) + theta_nu(x+mu) - theta_mu(x+nu) - theta_nu(x). */
/* The six plaquettes containing the link contribute cos(theta + a_k);       */
/* S = sum_k exp(i a_k) so that their sum is Re(exp(i theta) S).              */
/* Order: nu ascending over {0..3}\{mu}; the forward plaquette before the     */
/* backward one.                                                              */
/* ------------------------------------------------------------------------ */
void or_staple(const or_lat *g, long n, int mu, double *re, double *im)
{
    int c[4];
    site_coords(g, n, c);
    double sr = 0.0, si = 0.0;
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        long xpmu = nbr(g, c, mu, 1, nu, 0);
        long xpnu = nbr(g, c, nu, 1, mu, 0);
        long xmnu = nbr(g, c, nu, -1, mu, 0);
        long xpmu_mnu = nbr(g, c, mu, 1, nu, -1);
        double ap = (TH(g, xpmu, nu) - TH(g, xpnu, mu)) - TH(g, n, nu);
        double am = -((TH(g, xmnu, mu) + TH(g, xpmu_mnu, nu)) - TH(g, xmnu, nu));
        double s, co;
        or_sincos(ap, &s, &co);
        sr += co; si += s;
        or_sincos(am, &s, &co);
        sr += co; si += s;
    }
    *re = sr;
    *im = si;
}

/* Re(exp(i phi) S) */
static double re_phase_staple(double phi, double sr, double si)
{
    double s, c;
    or_sincos(phi, &s, &c);
    return c * sr - s * si;
}

/* change of beta*S (Eq. (3)) when link (n,mu) goes from its value to v */
double or_local_delta(const or_lat *g, long n, int mu, double v)
{
    double sr, si;
    or_staple(g, n, mu, &sr, &si);
    return g->beta * (re_phase_staple(TH(g, n, mu), sr, si) - re_phase_staple(v, sr, si));
}

/* beta*S of Eq. (3): beta * sum_x sum_{mu<nu} (1 - cos theta_munu(x)) */
double or_total_action(const or_lat *g)
{
    double acc = 0.0;
    for (long n = 0; n < g->V; ++n) {
        int c[4];
        site_coords(g, n, c);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) {
                double p = TH(g, n, mu) + TH(g, nbr(g, c, mu, 1, nu, 0), nu)
                         - TH(g, nbr(g, c, nu, 1, mu, 0), mu) - TH(g, n, nu);
                acc += 1.0 - cos(p);
            }
    }
    return g->beta * acc;
}

/* ------------------------------------------------------------------------ */
/* Link updates (Sec. 2.1).                                                   */
/* ------------------------------------------------------------------------ */
static int is_frozen(int t, int mu, int th_frozen)
{
    return th_frozen > 0 && mu > 0 && (t % th_frozen) == 0;
}

/* Metropolis: n_hits hits on link (n,mu) with its staple fixed.
 * Returns the new angle and writes one byte per hit (1 accepted, 0 rejected). */
static double metropolis_link(const or_lat *g, long n, int mu, int n_hits, uint64_t pass_id,
                              unsigned char *log)
{
    double sr, si;
    or_staple(g, n, mu, &sr, &si);
    double th = TH(g, n, mu);
    uint64_t key[2] = {g->seed, 0};
    for (int h = 0; h < n_hits; ++h) {
        uint64_t ctr[4] = {(uint64_t)n, (2ULL << 32) | ((uint64_t)h << 8) | (uint64_t)mu, pass_id, 0};
        uint64_t w[4];
        or_philox4x64_10(ctr, key, w);
        double u1 = u01(w[0]), u2 = u01(w[1]);
        double thn = wrap_angle(th + g->eps * (2.0 * u1 - 1.0));
        double dS = g->beta * (re_phase_staple(th, sr, si) - re_phase_staple(thn, sr, si));
        int acc = (dS <= 0.0) || (u2 < exp(-dS));
        if (acc) th = thn;
        if (log) log[h] = (unsigned char)acc;
    }
    return th;
}

/* Overrelaxation: reflect theta + alpha -> -(theta + alpha), alpha = arg S.
 * Leaves Re(exp(i theta) S) unchanged; the identity when S = 0. */
static double overrelax_link(const or_lat *g, long n, int mu)
{
    double sr, si;
    or_staple(g, n, mu, &sr, &si);
    double th = TH(g, n, mu);
    if (sr == 0.0 && si == 0.0) return th;
    double alpha = or_atan2(si, sr);
    return wrap_angle(-th - 2.0 * alpha);
}

/* One checkerboard class (mu, parity).  kind 0 = Metropolis, 1 = OR.
 * The log (Metropolis only) holds n_hits bytes per site of the class, in
 * increasing canonical index; frozen links are marked 2. */
void or_class_pass(or_lat *g, int mu, int parity, int kind, int n_hits, int th_frozen,
                   uint64_t pass_id, unsigned char *log)
{
    long V = g->V;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; ++n) {
        int c[4];
        site_coords(g, n, c);
        if (((c[0] + c[1] + c[2] + c[3]) & 1) != parity) continue;
        long slot = n >> 1; /* rank of n among the sites of its parity */
        if (is_frozen(c[0], mu, th_frozen)) {
            if (log && kind == 0)
                for (int h = 0; h < n_hits; ++h) log[slot * n_hits + h] = 2;
            continue;
        }
        double v;
        if (kind == 0)
            v = metropolis_link(g, n, mu, n_hits, pass_id, log ? log + slot * n_hits : NULL);
        else
            v = overrelax_link(g, n, mu);
        g->th[4 * n + mu] = v;
    }
}

/* Compound sweep: one Metropolis pass of n_metro hits then n_or OR passes.
 * Returns the number of bytes written to log (8 * V/2 * n_metro, or 0). */
long or_sweep(or_lat *g, int n_metro, int n_or, int th_frozen, unsigned char *log)
{
    long half = g->V / 2, written = 0;
    if (n_metro > 0) {
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p) {
                or_class_pass(g, mu, p, 0, n_metro, th_frozen, g->pass_id,
                              log ? log + written : NULL);
                if (log) written += half * n_metro;
            }
        g->pass_id += 1;
    }
    for (int k = 0; k < n_or; ++k)
        for (int mu = 0; mu < 4; ++mu)
            for (int p = 0; p < 2; ++p)
                or_class_pass(g, mu, p, 1, 0, th_frozen, 0, NULL);
    return written;
}

/* ------------------------------------------------------------------------ */
/* Plain observables.                                                          */
/* ------------------------------------------------------------------------ */
static double plaq_angle(const or_lat *g, long n, const int c[4], int mu, int nu)
{
    return TH(g, n, mu) + TH(g, nbr(g, c, mu, 1, nu, 0), nu) - TH(g, nbr(g, c, nu, 1, mu, 0), mu)
         - TH(g, n, nu);
}

/* average plaquette (1/6V) sum_x sum_{mu<nu} Re U_munu(x) */
double or_plaquette(const or_lat *g)
{
    double acc = 0.0;
    for (long n = 0; n < g->V; ++n) {
        int c[4];
        site_coords(g, n, c);
        for (int mu = 0; mu < 4; ++mu)
            for (int nu = mu + 1; nu < 4; ++nu) acc += cos(plaq_angle(g, n, c, mu, nu));
    }
    return acc / (6.0 * (double)g->V);
}

/* Polyakov loop P(xvec) = prod_t U_0(xvec, t), as a product of U(1) elements */
static void polyakov_line(const or_lat *g, int x, int y, int z, double *re, double *im)
{
    double pr = 1.0, pi = 0.0;
    for (int t = 0; t < g->T; ++t) {
        double a = TH(g, site_index(g, t, x, y, z), 0);
        double ur = cos(a), ui = sin(a);
        double nr = pr * ur - pi * ui;
        double ni = pr * ui + pi * ur;
        pr = nr; pi = ni;
    }
    *re = pr; *im = pi;
}

/* spatial average of P: out = {Re, Im, |.|} */
void or_polyakov(const or_lat *g, double *out)
{
    int L = g->L;
    double sr = 0.0, si = 0.0;
    for (int z = 0; z < L; ++z)
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x) {
                double r, i;
                polyakov_line(g, x, y, z, &r, &i);
                sr += r; si += i;
            }
    double l3 = (double)L * L * L;
    out[0] = sr / l3;
    out[1] = si / l3;
    out[2] = hypot(out[0], out[1]);
}

/* plain C(r) = L^-3 sum_x P*(x) P(x + r e_x): out[2*k] = Re, out[2*k+1] = Im */
void or_plain_correlator(const or_lat *g, int n_r, const int *r_list, double *out)
{
    int L = g->L;
    for (int k = 0; k < n_r; ++k) {
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < L; ++z)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    double ar, ai, br, bi;
                    polyakov_line(g, x, y, z, &ar, &ai);
                    polyakov_line(g, x + r_list[k], y, z, &br, &bi);
                    sr += ar * br + ai * bi;
                    si += ar * bi - ai * br;
                }
        double l3 = (double)L * L * L;
        out[2 * k] = sr / l3;
        out[2 * k + 1] = si / l3;
    }
}

/* Field operators, Eq. (5): a^2 F_munu = sqrt(beta) Im P_munu.
 * comp 0..2 = E_x,E_y,E_z from P_01,P_02,P_03;
 * comp 3..5 = B_x,B_y,B_z from P_23,P_31,P_12. */
static const int FIELD_MU[6] = {0, 0, 0, 2, 3, 1};
static const int FIELD_NU[6] = {1, 2, 3, 3, 1, 2};

double or_field_op(const or_lat *g, int comp, int t, int x, int y, int z)
{
    long n = site_index(g, t, x, y, z);
    int c[4];
    site_coords(g, n, c);
    return sqrt(g->beta) * sin(plaq_angle(g, n, c, FIELD_MU[comp], FIELD_NU[comp]));
}

/* squared components (Eq. (6)): a^4 F_munu^2 = beta (1 - Re P_munu) */
double or_field_op2(const or_lat *g, int comp, int t, int x, int y, int z)
{
    long n = site_index(g, t, x, y, z);
    int c[4];
    site_coords(g, n, c);
    return g->beta * (1.0 - cos(plaq_angle(g, n, c, FIELD_MU[comp], FIELD_NU[comp])));
}

/* lattice averages of the six squared components */
void or_field2_means(const or_lat *g, double *out)
{
    int L = g->L;
    for (int comp = 0; comp < 6; ++comp) {
        double acc = 0.0;
        for (int t = 0; t < g->T; ++t)
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) acc += or_field_op2(g, comp, t, x, y, z);
        out[comp] = acc / (double)g->V;
    }
}

/* lattice averages <O_c> of the six field operators */
void or_field_means(const or_lat *g, double *out)
{
    int L = g->L;
    for (int comp = 0; comp < 6; ++comp) {
        double acc = 0.0;
        for (int t = 0; t < g->T; ++t)
            for (int z = 0; z < L; ++z)
                for (int y = 0; y < L; ++y)
                    for (int x = 0; x < L; ++x) acc += or_field_op(g, comp, t, x, y, z);
        out[comp] = acc / (double)g->V;
    }
}

/* ------------------------------------------------------------------------ */
/* Multilevel algorithm (Sec. 2.2, Eqs. (8), (9)).                            */
/* ------------------------------------------------------------------------ */
typedef struct { double re, im; } cplx;

static cplx cmul(cplx a, cplx b)
{
    cplx r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}

/* ------------------------------------------------------------------------ */
/* Analytical multihit (Sec. 2.2, the variance reduction the paper applies   */
/* to the temporal links of the potential).  Given all other links, a link   */
/* with staple S = |S| e^{i alpha} has the conditional density               */
/* exp(beta |S| cos(theta + alpha)) / (2 pi I_0(beta |S|)), whose mean of    */
/* e^{i theta} is e^{-i alpha} I_1(beta |S|) / I_0(beta |S|).                */
/* ------------------------------------------------------------------------ */

/* I_1(x) / I_0(x) for x >= 0 from the power series
 *   I_n(x) = sum_k (x/2)^(2k+n) / (k! (k+n)!):
 * with a_k = (x^2/4)^k / (k!)^2, I_0 = sum_k a_k and I_1 = (x/2) sum_k a_k/(k+1).
 * Every term is positive, so both sums are accurate to a few ulp.  Above
 * x = 600 the terms would overflow and the large-x expansion
 * 1 - 1/(2x) - 1/(8x^2) - 1/(8x^3) - 25/(128x^4) is used (error < 1e-12). */
double or_bessel_ratio(double x)
{
    if (x <= 0.0) return 0.0;
    if (x > 600.0) {
        double u = 1.0 / x;
        return 1.0 - u / 2.0 - u * u / 8.0 - u * u * u / 8.0 - 25.0 * u * u * u * u / 128.0;
    }
    double q = x * x / 4.0, a = 1.0, s0 = 1.0, s1 = 1.0;
    for (int k = 1; k < 2000; ++k) {
        a *= q / ((double)k * (double)k);
        s0 += a;
        s1 += a / (double)(k + 1);
        if (a < 1e-18 * s0) break;
    }
    return 0.5 * x * s1 / s0;
}

/* multihit mean of the temporal link at canonical site n: out = (re, im) */
void or_multihit_mean(const or_lat *g, long n, double *out)
{
    double sr, si;
    or_staple(g, n, 0, &sr, &si);
    double a = hypot(sr, si);
    if (a == 0.0) {
        out[0] = out[1] = 0.0;
        return;
    }
    double q = or_bessel_ratio(g->beta * a) / a;
    out[0] = q * sr;
    out[1] = -q * si;
}

typedef struct ml_ctx {
    or_lat *g;
    int multihit;       /* correlator lines at r >= 2 from multihit means */
    int field_squared;  /* insert beta (1 - Re P) instead of sqrt(beta) Im P */
    int n_levels;
    const int *th;      /* slab thickness per level, outer to inner */
    const int *n_sub;   /* updates per level */
    int n_metro, n_or;
    int n_r;
    const int *r_list;
    int n_dir;          /* 1: separations along +x; 6: along +-x, +-y, +-z */
    int n_rf;           /* field insertion separations (0 = no field) */
    const int *rf_list;
    long L3;
    int n_d;            /* 2 planes * L * L offsets per rf */
    unsigned char *log;
    long log_cap, log_used;
} ml_ctx;

/* the six directions of a separation: +x, -x, +y, -y, +z, -z */
static const int DIR_VEC[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};

/* site x0 + r e_dir at time t */
static long source_shift(const or_lat *g, long x0, int t, int r, int dir)
{
    int L = g->L;
    int x = (int)(x0 % L), y = (int)((x0 / L) % L), z = (int)(x0 / ((long)L * L));
    return site_index(g, t, x + r * DIR_VEC[dir][0], y + r * DIR_VEC[dir][1], z + r * DIR_VEC[dir][2]);
}

/* T(x0, t, r) = U_0*(x0, t) U_0(x0 + r e, t), Eq. (8) without the operator,
 * for the direction e = e_dir */
static cplx two_link(const or_lat *g, long x0, int t, int r, int dir)
{
    double a = TH(g, source_shift(g, x0, t, 0, 0), 0);
    double b = TH(g, source_shift(g, x0, t, r, dir), 0);
    cplx ua = {cos(a), -sin(a)};
    cplx ub = {cos(b), sin(b)};
    return cmul(ua, ub);
}

/* the same product from the multihit means of both temporal links; used for
 * the correlator at r >= 2, where the two links share no plaquette */
static cplx two_link_mh(const or_lat *g, long x0, int t, int r, int dir)
{
    double a[2], b[2];
    or_multihit_mean(g, source_shift(g, x0, t, 0, 0), a);
    or_multihit_mean(g, source_shift(g, x0, t, r, dir), b);
    cplx ua = {a[0], -a[1]};
    cplx ub = {b[0], b[1]};
    return cmul(ua, ub);
}

/* displacement d of the field operator relative to the source x0:
 * index d = (plane*L + dy)*L + dz, plane 0 at x offset (r-1)/2, plane 1 at r/2 */
static double field_at(const or_lat *g, int comp, long x0, int t, int rf, int d, int squared)
{
    int L = g->L;
    int x = (int)(x0 % L), y = (int)((x0 / L) % L), z = (int)(x0 / ((long)L * L));
    int plane = d / (L * L), dy = (d / L) % L, dz = d % L;
    int m = plane == 0 ? (rf - 1) / 2 : rf / 2;
    return squared ? or_field_op2(g, comp, t, x + m, y + dy, z + dz) : or_field_op(g, comp, t, x + m, y + dy, z + dz);
}

/* Accumulator sizes: corr[slab][x0][dir][r], field[slab][x0][rf][d][comp] (complex) */
static size_t corr_len(const ml_ctx *c, int nslab) { return (size_t)nslab * c->L3 * c->n_dir * c->n_r; }
static size_t field_len(const ml_ctx *c, int nslab)
{
    return (size_t)nslab * c->L3 * c->n_rf * c->n_d * 6;
}

static void do_sweep(ml_ctx *c, int th_frozen)
{
    long want = c->log ? (long)8 * (c->g->V / 2) * c->n_metro : 0;
    unsigned char *dst = NULL;
    if (c->log && c->log_used + want <= c->log_cap) dst = c->log + c->log_used;
    long w = or_sweep(c->g, c->n_metro, c->n_or, th_frozen, dst);
    if (dst) c->log_used += w;
}

/* Level lev: n_sub[lev] iterations of (update with this level's slabs frozen,
 * then measure or recurse).  Returns the averages over the iterations of the
 * slab products ([T] in the multilevel notation) and of the slab products
 * with one field insertion ([TO]). */
static void ml_level(ml_ctx *c, int lev, cplx *avg, cplx *favg)
{
    or_lat *g = c->g;
    int th = c->th[lev];
    int nslab = g->T / th;
    size_t cl = corr_len(c, nslab), fl = field_len(c, nslab);
    memset(avg, 0, cl * sizeof(cplx));
    if (fl) memset(favg, 0, fl * sizeof(cplx));

    int inner = lev == c->n_levels - 1;
    int nchild = inner ? 0 : th / c->th[lev + 1];
    int cslab = inner ? 0 : g->T / c->th[lev + 1];
    cplx *cavg = NULL, *cfavg = NULL;
    if (!inner) {
        cavg = (cplx *)malloc(corr_len(c, cslab) * sizeof(cplx));
        cfavg = field_len(c, cslab) ? (cplx *)malloc(field_len(c, cslab) * sizeof(cplx)) : NULL;
    }

    for (int it = 0; it < c->n_sub[lev]; ++it) {
        do_sweep(c, th);
        if (!inner) ml_level(c, lev + 1, cavg, cfavg);
#pragma omp parallel for schedule(static)
        for (long x0 = 0; x0 < c->L3; ++x0) {
            for (int s = 0; s < nslab; ++s) {
                int nk = c->n_dir * c->n_r;  /* (direction, r) pairs */
                for (int k = 0; k < nk; ++k) {
                    cplx p = {1.0, 0.0};
                    if (inner) {
                        int r = c->r_list[k % c->n_r], dir = k / c->n_r;
                        for (int t = s * th; t < (s + 1) * th; ++t)
                            p = cmul(p, c->multihit && r >= 2 ? two_link_mh(g, x0, t, r, dir)
                                                              : two_link(g, x0, t, r, dir));
                    } else {
                        for (int ch = 0; ch < nchild; ++ch)
                            p = cmul(p, cavg[((size_t)(s * nchild + ch) * c->L3 + x0) * nk + k]);
                    }
                    cplx *a = &avg[((size_t)s * c->L3 + x0) * nk + k];
                    a->re += p.re;
                    a->im += p.im;
                }
                for (int f = 0; f < c->n_rf; ++f) {
                    int r = c->rf_list[f];
                    for (int d = 0; d < c->n_d; ++d)
                        for (int comp = 0; comp < 6; ++comp) {
                            cplx sum = {0.0, 0.0};
                            if (inner) {
                                /* TO = sum over the insertion time t of
                                 * prod_{t' != t} T(t') * O(t) with O(t) = T(t) O(x,t) */
                                for (int ti = s * th; ti < (s + 1) * th; ++ti) {
                                    cplx p = {1.0, 0.0};
                                    for (int t = s * th; t < (s + 1) * th; ++t) {
                                        cplx tl = two_link(g, x0, t, r, 0);
                                        if (t == ti) {
                                            double o = field_at(g, comp, x0, t, r, d, c->field_squared);
                                            tl.re *= o;
                                            tl.im *= o;
                                        }
                                        p = cmul(p, tl);
                                    }
                                    sum.re += p.re;
                                    sum.im += p.im;
                                }
                            } else {
                                /* the insertion sits in one child slab; the
                                 * others contribute their plain averages */
                                for (int ci = 0; ci < nchild; ++ci) {
                                    cplx p = {1.0, 0.0};
                                    for (int ch = 0; ch < nchild; ++ch) {
                                        int sc = s * nchild + ch;
                                        cplx v;
                                        if (ch == ci)
                                            v = cfavg[((((size_t)sc * c->L3 + x0) * c->n_rf + f) * c->n_d + d) * 6 + comp];
                                        else {
                                            /* plain average at the field separation r along +x */
                                            size_t base = ((size_t)sc * c->L3 + x0) * c->n_dir * c->n_r;
                                            v = cavg[base];
                                            for (int kk = 0; kk < c->n_r; ++kk)
                                                if (c->r_list[kk] == r) v = cavg[base + kk];
                                        }
                                        p = cmul(p, v);
                                    }
                                    sum.re += p.re;
                                    sum.im += p.im;
                                }
                            }
                            cplx *a = &favg[((((size_t)s * c->L3 + x0) * c->n_rf + f) * c->n_d + d) * 6 + comp];
                            a->re += sum.re;
                            a->im += sum.im;
                        }
                }
            }
        }
    }
    double inv = 1.0 / (double)c->n_sub[lev];
    for (size_t i = 0; i < cl; ++i) { avg[i].re *= inv; avg[i].im *= inv; }
    for (size_t i = 0; i < fl; ++i) { favg[i].re *= inv; favg[i].im *= inv; }
    free(cavg);
    free(cfavg);
}

/* Multilevel estimators.
 *   corr_out[2*k + {0,1}] = C_ML(r_k) = L^-3 sum_x0 prod_{top slabs} A_s(x0, r_k)
 *   field_out[((((f*2 + plane)*6 + comp)*L + dy)*L + dz)*2 + {0,1}]
 *       = <P*(0) P(r) O_comp(m, dy, dz)> of Eq. (9): (1/V) sum_x0 sum over the
 *         slab s holding the insertion of B_s(x0) prod_{s' != s} A_s'(x0).
 * Every r_f in rf_list must also appear in r_list.  flags & 1 (multihit)
 * replaces, for every r >= 2, the temporal links of both lines by their
 * multihit means in the correlator products (and so in the slab averages that
 * multiply a field insertion elsewhere); r = 1 and the slab holding a field
 * insertion use the links themselves.  flags & 2 inserts the squared
 * components beta (1 - Re P) of Eq. (6) instead of sqrt(beta) Im P.  flags & 4
 * makes C_ML(r) the average over the six separations r e with e = +-x, +-y,
 * +-z, each estimated by the same nested averages (the field insertion stays
 * along +x; its slab averages use the +x lines).  Returns
 * 0, or -1 on a bad argument (slab sizes must divide T and each other). */
int or_multilevel(or_lat *g, int n_levels, const int *th, const int *n_sub, int n_metro, int n_or,
                  int n_r, const int *r_list, double *corr_out, int n_rf, const int *rf_list,
                  double *field_out, unsigned char *log, long log_cap, long *log_used, int flags)
{
    if (n_levels < 1 || n_r < 1) return -1;
    for (int l = 0; l < n_levels; ++l) {
        if (th[l] < 1 || g->T % th[l] || n_sub[l] < 1) return -1;
        if (l > 0 && th[l - 1] % th[l]) return -1;
    }
    for (int f = 0; f < n_rf; ++f) {
        int ok = 0;
        for (int k = 0; k < n_r; ++k) ok |= r_list[k] == rf_list[f];
        if (!ok) return -1;
    }
    ml_ctx c;
    memset(&c, 0, sizeof c);
    c.g = g; c.n_levels = n_levels; c.th = th; c.n_sub = n_sub;
    c.multihit = flags & 1; c.field_squared = (flags >> 1) & 1;
    c.n_dir = (flags & 4) ? 6 : 1;
    c.n_metro = n_metro; c.n_or = n_or;
    c.n_r = n_r; c.r_list = r_list; c.n_rf = n_rf; c.rf_list = rf_list;
    c.L3 = (long)g->L * g->L * g->L;
    c.n_d = 2 * g->L * g->L;
    c.log = log; c.log_cap = log_cap; c.log_used = 0;

    int nslab = g->T / th[0];
    cplx *A = (cplx *)malloc(corr_len(&c, nslab) * sizeof(cplx));
    size_t fl = field_len(&c, nslab);
    cplx *B = fl ? (cplx *)malloc(fl * sizeof(cplx)) : NULL;
    ml_level(&c, 0, A, B);

    int nk = c.n_dir * n_r;
    for (int k = 0; k < n_r; ++k) {
        double cr = 0.0, ci = 0.0;
        for (int dir = 0; dir < c.n_dir; ++dir) {
            double sr = 0.0, si = 0.0;
            for (long x0 = 0; x0 < c.L3; ++x0) {
                cplx p = {1.0, 0.0};
                for (int s = 0; s < nslab; ++s) p = cmul(p, A[((size_t)s * c.L3 + x0) * nk + dir * n_r + k]);
                sr += p.re;
                si += p.im;
            }
            cr += sr / (double)c.L3;
            ci += si / (double)c.L3;
        }
        corr_out[2 * k] = cr / c.n_dir;
        corr_out[2 * k + 1] = ci / c.n_dir;
    }
    for (int f = 0; f < n_rf; ++f) {
        int kr = 0;
        for (int k = 0; k < n_r; ++k)
            if (r_list[k] == rf_list[f]) kr = k;
        for (int d = 0; d < c.n_d; ++d)
            for (int comp = 0; comp < 6; ++comp) {
                double sr = 0.0, si = 0.0;
                for (long x0 = 0; x0 < c.L3; ++x0)
                    for (int s = 0; s < nslab; ++s) {
                        cplx p = B[((((size_t)s * c.L3 + x0) * n_rf + f) * c.n_d + d) * 6 + comp];
                        for (int s2 = 0; s2 < nslab; ++s2)
                            if (s2 != s) p = cmul(p, A[((size_t)s2 * c.L3 + x0) * nk + kr]);
                        sr += p.re;
                        si += p.im;
                    }
                int plane = d / (g->L * g->L), rest = d % (g->L * g->L);
                size_t o = ((((size_t)f * 2 + plane) * 6 + comp) * (size_t)(g->L * g->L) + rest) * 2;
                field_out[o] = sr / (double)g->V;
                field_out[o + 1] = si / (double)g->V;
            }
    }
    free(A);
    free(B);
    if (log_used) *log_used = c.log_used;
    return 0;
}
