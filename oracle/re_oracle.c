/*
 * re_oracle.c -- plain, slow FP64 CPU oracle for replica-exchange
 * Lennard-Jones molecular dynamics (Bussi, "A simple asynchronous
 * replica-exchange implementation").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * generator with the GPU library; the two are written independently from the
 * paper and from the published definitions named below.
 *
 * Every function is written for obviousness, not speed: double precision,
 * plain loops, no blocking, no fusion.  Each cites the passage it follows.
 *
 * Readings of the paper where it is silent:
 *   - periodic cubic box, minimum image; side L rounded to a multiple of
 *     2^-12 so that the box and grid-aligned positions are exact in both
 *     single and double precision;
 *   - truncated-and-shifted LJ energy, plain truncated force (strict r < r_c);
 *   - BAOAB Langevin splitting (velocity-Verlet core, gamma = 0 is NVE);
 *   - stochastic velocity rescaling (the thermostat the Example section
 *     names): velocity Verlet, then once per step the rescale of Bussi,
 *     Donadio and Parrinello with N_f = 3N - 3, relaxation time tau (0.5 by
 *     default; the paper gives none) and the positive root;
 *   - Verlet list to r_c + skin rebuilt when one displacement exceeds skin/2
 *     (strict >), measured from the positions at the last rebuild;
 *   - exchange pattern alternates even/odd ladder pairs; "lowest rank" is the
 *     lower replica id; u is a 53-bit uniform; accept iff D >= 0 or u < e^D;
 *   - velocities scaled by sqrt(T_new/T_old) at the step boundary.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PURPOSE_INITVEL 0u
#define ORACLE_PURPOSE_OSTEP 1u
#define ORACLE_PURPOSE_EXCHANGE 2u
#define ORACLE_PURPOSE_VACANCY 3u
#define ORACLE_PURPOSE_SVR 4u
#define ORACLE_PURPOSE_PATTERN 5u

#define ORACLE_LANGEVIN 0
#define ORACLE_SVR 1

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator, from its published definition:
 * J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11.  Four 32-bit counter words, two key
 * words, ten rounds; each round multiplies counter words 0 and 2 by the two
 * Philox multipliers, and mixes the high halves with the odd words and the
 * round key; the key is advanced by the two Weyl constants between rounds.  */
static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
}

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

static void draw4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t w[4])
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, w);
}

/* Open-interval uniform from one 32-bit word: (w + 1/2) 2^-32 in (0, 1). */
static double open_uniform(uint32_t w)
{
    return ((double)w + 0.5) * (1.0 / 4294967296.0);
}

/* Three standard normals from one Philox draw by the Box-Muller transform
 * (G. E. P. Box, M. E. Muller, Ann. Math. Stat. 29, 1958): words (0,1) give
 * a cosine/sine pair, words (2,3) give one more cosine.  The counter is
 * (c0, c1, c2, purpose).                                                     */
void oracle_normals3(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t purpose, double z[3])
{
    uint32_t w[4];
    draw4(seed, c0, c1, c2, purpose, w);
    const double two_pi = 6.283185307179586476925286766559;
    double r01 = sqrt(-2.0 * log(open_uniform(w[0])));
    double a01 = two_pi * open_uniform(w[1]);
    double r23 = sqrt(-2.0 * log(open_uniform(w[2])));
    double a23 = two_pi * open_uniform(w[3]);
    z[0] = r01 * cos(a01);
    z[1] = r01 * sin(a01);
    z[2] = r23 * cos(a23);
}

/* Uniform random number of an exchange attempt (Implementation: the number
 * drawn by the lower-ranked member of the pair decides).  Counter =
 * (attempt low word, attempt high word, lower replica id, purpose 2); the
 * 53-bit value ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 lies in [0, 1).           */
double oracle_uniform53(uint64_t seed, int64_t attempt, int32_t lower_id)
{
    uint32_t w[4];
    uint64_t a = (uint64_t)attempt;
    draw4(seed, (uint32_t)a, (uint32_t)(a >> 32), (uint32_t)lower_id, ORACLE_PURPOSE_EXCHANGE, w);
    uint64_t hi = (uint64_t)(w[0] >> 5);
    uint64_t lo = (uint64_t)(w[1] >> 6);
    return (double)(hi * 67108864u + lo) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Box (Example section: LJ units, N particles at density rho).  Periodic
 * cube of side (N/rho)^(1/3), rounded to a multiple of 2^-12.               */
double oracle_box_length(int32_t N, double rho)
{
    double L = cbrt((double)N / rho);
    return nearbyint(L * 4096.0) / 4096.0;
}

static double min_image(double d, double L)
{
    return d - L * nearbyint(d / L);
}

static double wrap_into_box(double x, double L)
{
    /* result in [-L/2, L/2) */
    return x - L * floor((x + 0.5 * L) / L);
}

/* ------------------------------------------------------------------------ */
/* Initial state.  The paper gives only N and rho (Example section); the
 * start is a face-centred-cubic lattice of n^3 cells, n the smallest integer
 * with 4 n^3 >= N, cell a = L/n, basis {0, (a/2,a/2,0), (a/2,0,a/2),
 * (0,a/2,a/2)} shifted by a/4 in every direction.  When 4 n^3 > N the N kept
 * sites are those with the smallest Philox key (purpose 3, ties by site
 * index); atom ids follow ascending site index.  Velocities are sqrt(T)
 * times Philox normals (purpose 0), minus their mean, then scaled so that
 * sum |v|^2 = (3N - 3) T (m = 1).                                           */
typedef struct { uint32_t key; int32_t site; } site_key;

static int cmp_site_key(const void* pa, const void* pb)
{
    const site_key* a = (const site_key*)pa;
    const site_key* b = (const site_key*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->site < b->site ? -1 : (a->site > b->site ? 1 : 0);
}

static int cmp_int(const void* pa, const void* pb)
{
    int a = *(const int*)pa, b = *(const int*)pb;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int oracle_fcc_cells(int32_t N)
{
    int n = 1;
    while (4 * n * n * n < N) ++n;
    return n;
}

int oracle_init(int32_t N, double L, double T, uint64_t seed, int32_t replica, double* x, double* v)
{
    if (N < 2 || L <= 0.0 || T <= 0.0) return -1;
    int n = oracle_fcc_cells(N);
    int M = 4 * n * n * n;
    int* kept = (int*)malloc(sizeof(int) * (size_t)M);
    if (!kept) return -2;
    if (M == N) {
        for (int m = 0; m < M; ++m) kept[m] = m;
    } else {
        site_key* keys = (site_key*)malloc(sizeof(site_key) * (size_t)M);
        if (!keys) { free(kept); return -2; }
        for (int m = 0; m < M; ++m) {
            uint32_t w[4];
            draw4(seed, (uint32_t)m, 0u, (uint32_t)replica, ORACLE_PURPOSE_VACANCY, w);
            keys[m].key = w[0];
            keys[m].site = m;
        }
        qsort(keys, (size_t)M, sizeof(site_key), cmp_site_key);
        for (int i = 0; i < N; ++i) kept[i] = keys[i].site;
        qsort(kept, (size_t)N, sizeof(int), cmp_int);
        free(keys);
    }
    const double a = L / (double)n;
    const double basis[4][3] = {{0.0, 0.0, 0.0}, {0.5, 0.5, 0.0}, {0.5, 0.0, 0.5}, {0.0, 0.5, 0.5}};
    for (int i = 0; i < N; ++i) {
        int m = kept[i];
        int b = m % 4;
        int cell = m / 4;
        int iz = cell % n;
        int iy = (cell / n) % n;
        int ix = cell / (n * n);
        x[3 * i + 0] = ((double)ix + basis[b][0] + 0.25) * a - 0.5 * L;
        x[3 * i + 1] = ((double)iy + basis[b][1] + 0.25) * a - 0.5 * L;
        x[3 * i + 2] = ((double)iz + basis[b][2] + 0.25) * a - 0.5 * L;
    }
    free(kept);

    double sqrtT = sqrt(T);
    double mean[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < N; ++i) {
        double z[3];
        oracle_normals3(seed, (uint32_t)i, 0u, (uint32_t)replica, ORACLE_PURPOSE_INITVEL, z);
        for (int d = 0; d < 3; ++d) {
            v[3 * i + d] = sqrtT * z[d];
            mean[d] += v[3 * i + d];
        }
    }
    for (int d = 0; d < 3; ++d) mean[d] /= (double)N;
    double sumv2 = 0.0;
    for (int i = 0; i < N; ++i)
        for (int d = 0; d < 3; ++d) {
            v[3 * i + d] -= mean[d];
            sumv2 += v[3 * i + d] * v[3 * i + d];
        }
    double scale = sqrt((double)(3 * N - 3) * T / sumv2);
    for (int i = 0; i < 3 * N; ++i) v[i] *= scale;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pair interaction (Example section: LJ liquid, cutoff 2.5 in LJ units).
 * u(r) = 4 (r^-12 - r^-6) - u_lj(r_c) for r < r_c, 0 otherwise; the force is
 * the plain truncated -du/dr, so for r < r_c:
 *   F_i = 24 (2 r^-14 - r^-8) (x_i - x_j).                                   */
double oracle_lj_shift(double rc)
{
    double ir6 = 1.0 / (rc * rc * rc * rc * rc * rc);
    return 4.0 * (ir6 * ir6 - ir6);
}

/* Returns the pair energy and stores f/r (so that F_i = fr * d) for r2 < rc2. */
static double lj_pair(double r2, double ushift, double* fr)
{
    double ir2 = 1.0 / r2;
    double ir6 = ir2 * ir2 * ir2;
    *fr = 24.0 * ir2 * ir6 * (2.0 * ir6 - 1.0);
    return 4.0 * ir6 * (ir6 - 1.0) - ushift;
}

/* Forces as the plain sum over all pairs i < j with r_ij < r_c (minimum
 * image).  Also the potential energy U and the pair virial W = sum f.r.      */
int oracle_forces(int32_t N, double L, double rc, const double* x, double* F, double* U, double* W)
{
    const double rc2 = rc * rc;
    const double ushift = oracle_lj_shift(rc);
    double u = 0.0, w = 0.0;
    for (int i = 0; i < 3 * N; ++i) F[i] = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int j = i + 1; j < N; ++j) {
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = min_image(x[3 * i + k] - x[3 * j + k], L);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) {
                double fr;
                u += lj_pair(r2, ushift, &fr);
                w += fr * r2;
                for (int k = 0; k < 3; ++k) {
                    F[3 * i + k] += fr * d[k];
                    F[3 * j + k] -= fr * d[k];
                }
            }
        }
    }
    if (U) *U = u;
    if (W) *W = w;
    return 0;
}

/* Force on one atom i and its pair-energy sum e_i = sum_j u(r_ij) (so that
 * U = e/2 summed over atoms): the definition restricted to one row, for
 * checking sampled atoms of large systems.                                  */
int oracle_force_on(int32_t N, double L, double rc, const double* x, int32_t i, double* Fi, double* ei)
{
    const double rc2 = rc * rc;
    const double ushift = oracle_lj_shift(rc);
    double f[3] = {0.0, 0.0, 0.0}, e = 0.0;
    for (int j = 0; j < N; ++j) {
        if (j == i) continue;
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = min_image(x[3 * i + k] - x[3 * j + k], L);
        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        if (r2 < rc2) {
            double fr;
            e += lj_pair(r2, ushift, &fr);
            for (int k = 0; k < 3; ++k) f[k] += fr * d[k];
        }
    }
    for (int k = 0; k < 3; ++k) Fi[k] = f[k];
    *ei = e;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Verlet neighbour list (Example section: pairs up to r_c + skin, updated
 * when one particle moved more than half the skin since the last update).
 * The list holds, for each i, the j > i (ascending) whose distance at the
 * last update was below r_c + skin.  Forces over the list run the same
 * floating-point operations in the same order as oracle_forces, because
 * every pair omitted from the list is beyond r_c until the next update.     */
typedef struct {
    int32_t* start; /* N + 1 */
    int32_t* nbr;
    int64_t cap;
} vlist;

static int vlist_build(vlist* vl, int32_t N, double L, double rlist, const double* xref)
{
    const double rl2 = rlist * rlist;
    int64_t count = 0;
    if (!vl->start) {
        vl->start = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 1));
        if (!vl->start) return -2;
    }
    for (int pass = 0; pass < 2; ++pass) {
        count = 0;
        for (int i = 0; i < N; ++i) {
            if (pass == 1) vl->start[i] = (int32_t)count;
            for (int j = i + 1; j < N; ++j) {
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = min_image(xref[3 * i + k] - xref[3 * j + k], L);
                double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                if (r2 < rl2) {
                    if (pass == 1) vl->nbr[count] = j;
                    ++count;
                }
            }
        }
        if (pass == 0 && count > vl->cap) {
            free(vl->nbr);
            vl->cap = count + count / 4 + 16;
            vl->nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)vl->cap);
            if (!vl->nbr) return -2;
        }
    }
    vl->start[N] = (int32_t)count;
    return 0;
}

static void vlist_free(vlist* vl)
{
    free(vl->start);
    free(vl->nbr);
    vl->start = NULL;
    vl->nbr = NULL;
    vl->cap = 0;
}

static void forces_from_list(const vlist* vl, int32_t N, double L, double rc, const double* x, double* F, double* U)
{
    const double rc2 = rc * rc;
    const double ushift = oracle_lj_shift(rc);
    double u = 0.0;
    for (int i = 0; i < 3 * N; ++i) F[i] = 0.0;
    for (int i = 0; i < N; ++i) {
        for (int32_t p = vl->start[i]; p < vl->start[i + 1]; ++p) {
            int j = vl->nbr[p];
            double d[3];
            for (int k = 0; k < 3; ++k) d[k] = min_image(x[3 * i + k] - x[3 * j + k], L);
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (r2 < rc2) {
                double fr;
                u += lj_pair(r2, ushift, &fr);
                for (int k = 0; k < 3; ++k) {
                    F[3 * i + k] += fr * d[k];
                    F[3 * j + k] -= fr * d[k];
                }
            }
        }
    }
    *U = u;
}

/* Largest displacement since the last list update exceeds skin/2 (strict). */
static int needs_rebuild(int32_t N, double L, double skin, const double* x, const double* xref)
{
    const double lim2 = 0.25 * skin * skin;
    for (int i = 0; i < N; ++i) {
        double d[3];
        for (int k = 0; k < 3; ++k) d[k] = min_image(x[3 * i + k] - xref[3 * i + k], L);
        if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > lim2) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Stochastic velocity rescaling (Example section: the thermostat; G. Bussi,
 * D. Donadio, M. Parrinello, J. Chem. Phys. 126, 014101 (2007)).  Over a
 * time dt the kinetic energy K relaxes towards Kbar = N_f T / 2 with time
 * constant tau plus a noise term chosen so that K samples the canonical
 * distribution (Gamma with shape N_f/2 and scale T):
 *   K' = K + (1 - c) (Kbar (R1^2 + S) / N_f - K) + 2 R1 sqrt(c (1 - c) K Kbar / N_f),
 * c = exp(-dt / tau), R1 a standard normal and S a chi-square variate with
 * N_f - 1 degrees of freedom; the velocities are multiplied by
 * sqrt(K' / K) (the positive root).  K = 0 leaves them unchanged.           */
double oracle_svr_factor(double K, double Kbar, double Nf, double c, double R1, double S)
{
    if (!(K > 0.0)) return 1.0;
    double Knew = K + (1.0 - c) * (Kbar * (R1 * R1 + S) / Nf - K) + 2.0 * R1 * sqrt(c * (1.0 - c) * K * Kbar / Nf);
    return sqrt(Knew / K);
}

/* The normals of the rescale of replica r at step boundary s: Philox
 * counter (atom id, s, r, purpose 4) gives three normals per atom.  R1 is
 * the first normal of atom 0; S is the sum of the squares of all others
 * except the last two of atom 0 and the first of atom 1, i.e. 3N - 4 =
 * N_f - 1 squared standard normals (a chi-square variate by definition).   */
void oracle_svr_noise(uint64_t seed, int32_t N, int32_t replica, int64_t s, double* R1, double* S)
{
    double acc = 0.0;
    for (int i = 0; i < N; ++i) {
        double z[3];
        oracle_normals3(seed, (uint32_t)i, (uint32_t)s, (uint32_t)replica, ORACLE_PURPOSE_SVR, z);
        if (i == 0) {
            *R1 = z[0];
        } else if (i == 1) {
            acc += z[1] * z[1] + z[2] * z[2];
        } else {
            acc += z[0] * z[0] + z[1] * z[1] + z[2] * z[2];
        }
    }
    *S = acc;
}

/* One rescale of replica r at step boundary s (temperature T). */
static void svr_rescale(int32_t N, double* v, double T, double c, uint64_t seed, int32_t replica, int64_t s)
{
    double K = 0.0;
    for (int i = 0; i < 3 * N; ++i) K += 0.5 * v[i] * v[i];
    const double Nf = 3.0 * N - 3.0;
    double R1, S;
    oracle_svr_noise(seed, N, replica, s, &R1, &S);
    const double a = oracle_svr_factor(K, 0.5 * Nf * T, Nf, c, R1, S);
    for (int i = 0; i < 3 * N; ++i) v[i] *= a;
}

/* ------------------------------------------------------------------------ */
/* Molecular dynamics of one replica (Example section: time step dt, the
 * temperature held by a thermostat).  thermostat ORACLE_LANGEVIN: Langevin
 * dynamics with friction gamma in the BAOAB splitting (B. Leimkuhler,
 * C. Matthews, Appl. Math. Res. Express 2013), m = 1, h = dt/2,
 * c1 = exp(-gamma dt),
 * c2 = sqrt((1 - c1^2) T):
 *     v += h F;  x += h v;  v = c1 v + c2 xi;  x += h v;  wrap;
 *     [list update if triggered];  F = F(x);  v += h F.
 * xi for atom id i at the step leaving step count s is the Box-Muller
 * triple of Philox counter (i, s, replica, purpose 1).
 * thermostat ORACLE_SVR (the paper's thermostat): the same steps without O
 * (c1 = 1, c2 = 0), then at each new step boundary s + 1 the stochastic
 * velocity rescale above with c = exp(-dt / tau).
 *
 * State on entry: x, v at a step boundary, F = forces at x, xref = positions
 * at the last list update.  step0 = steps already done.  Runs nsteps steps,
 * counts list updates into *rebuilds and stores U at the final positions
 * (left unchanged when nsteps = 0: on entry *U is the energy at x).
 * use_list = 0 evaluates every step by the all-pairs definition; 1 uses the
 * Verlet list (bit-identical results, see vlist above).                      */
int oracle_md(int32_t N, double L, double rc, double skin, double dt, double gamma, double T,
              uint64_t seed, int32_t replica, int64_t step0, int64_t nsteps,
              double* x, double* v, double* F, double* xref,
              int64_t* rebuilds, double* U, int use_list, int thermostat, double tau)
{
    const double h = 0.5 * dt;
    const int svr = thermostat == ORACLE_SVR;
    const double c1 = svr ? 1.0 : exp(-gamma * dt);
    const double c2 = svr ? 0.0 : sqrt((1.0 - c1 * c1) * T);
    const double csvr = svr ? exp(-dt / tau) : 1.0;
    vlist vl = {NULL, NULL, 0};
    double u = 0.0;
    int rc_ok = 0;
    if (use_list) {
        if (vlist_build(&vl, N, L, rc + skin, xref) != 0) { vlist_free(&vl); return -2; }
    }
    for (int64_t s = step0; s < step0 + nsteps; ++s) {
        for (int i = 0; i < N; ++i) {
            double z[3] = {0.0, 0.0, 0.0};
            if (!svr) oracle_normals3(seed, (uint32_t)i, (uint32_t)s, (uint32_t)replica, ORACLE_PURPOSE_OSTEP, z);
            for (int k = 0; k < 3; ++k) {
                double vi = v[3 * i + k] + h * F[3 * i + k];
                double xi = x[3 * i + k] + h * vi;
                vi = c1 * vi + c2 * z[k];
                xi = xi + h * vi;
                x[3 * i + k] = wrap_into_box(xi, L);
                v[3 * i + k] = vi;
            }
        }
        if (needs_rebuild(N, L, skin, x, xref)) {
            memcpy(xref, x, sizeof(double) * 3 * (size_t)N);
            *rebuilds += 1;
            if (use_list && vlist_build(&vl, N, L, rc + skin, xref) != 0) { rc_ok = -2; break; }
        }
        if (use_list)
            forces_from_list(&vl, N, L, rc, x, F, &u);
        else
            oracle_forces(N, L, rc, x, F, &u, NULL);
        for (int i = 0; i < 3 * N; ++i) v[i] += h * F[i];
        if (svr) svr_rescale(N, v, T, csvr, seed, replica, s + 1);
    }
    if (nsteps > 0) *U = u;
    vlist_free(&vl);
    return rc_ok;
}

/* ------------------------------------------------------------------------ */
/* Exchange rule (Implementation section).  Temperatures, not coordinates,
 * move: slot[r] is the ladder index held by replica r.  Attempt k pairs the
 * ladder slots (j, j+1) with j = k mod 2, j+1 < R.  For the replicas a, b
 * holding them, D = (1/T_j - 1/T_{j+1}) (U_a - U_b); the uniform of the
 * lower replica id decides; accept iff D >= 0 or u < exp(D) (standard
 * Metropolis rule of Sugita and Okamoto).  On acceptance the slots swap and
 * each velocity scale factor is sqrt(T_new / T_old).
 *
 * Non-nearest-neighbour exchanges (Implementation section: the scheme
 * extends to them) take the pairing distance d of attempt k at random in
 * 1 .. max_distance: d = 1 + (w0 mod max_distance) with w0 the first word of
 * Philox counter (k low, k high, 0, purpose 5) (d = 1 when max_distance is
 * 1).  With o = (k mod 2) d, ladder slot j >= o is paired with j + d when
 * floor((j - o) / d) is even and j + d < R; the rule above applies to the
 * pair (j, j + d) with T_j, T_{j+d}.  For d = 1 this is the alternating
 * pattern.  The pattern never depends on the replicas' state, so detailed
 * balance holds for every d.                                                 */
int oracle_metropolis(double Ua, double Ub, double Tj, double Tj1, double u)
{
    double delta = (1.0 / Tj - 1.0 / Tj1) * (Ua - Ub);
    return (delta >= 0.0 || u < exp(delta)) ? 1 : 0;
}

typedef struct {
    int64_t attempt;
    int32_t slot_lo, rep_a, rep_b, accepted;
    int64_t step_a, step_b;
    double U_a, U_b, T_a, T_b, u;
    int32_t slot_hi, pad;
} oracle_xrec;

int oracle_pattern_distance(uint64_t seed, int64_t k, int32_t max_distance)
{
    if (max_distance <= 1) return 1;
    uint32_t w[4];
    uint64_t a = (uint64_t)k;
    draw4(seed, (uint32_t)a, (uint32_t)(a >> 32), 0u, ORACLE_PURPOSE_PATTERN, w);
    return 1 + (int)(w[0] % (uint32_t)max_distance);
}

int oracle_exchange(int32_t R, const double* Tl, int32_t* slot, const double* U, const int64_t* steps,
                    uint64_t seed, int64_t k, int32_t max_distance, double* alpha,
                    int64_t* attempts, int64_t* accepts, oracle_xrec* log, int64_t* nlog)
{
    int32_t* rep = (int32_t*)malloc(sizeof(int32_t) * (size_t)R);
    if (!rep) return -2;
    for (int r = 0; r < R; ++r) rep[slot[r]] = r;
    for (int r = 0; r < R; ++r) alpha[r] = 1.0;
    const int d = oracle_pattern_distance(seed, k, max_distance);
    const int o = (int)(k % 2) * d;
    for (int j = o; j + d < R; ++j) {
        if (((j - o) / d) % 2 != 0) continue;
        const int h = j + d;
        int a = rep[j], b = rep[h];
        int lower = a < b ? a : b;
        double u = oracle_uniform53(seed, k, lower);
        int acc = oracle_metropolis(U[a], U[b], Tl[j], Tl[h], u);
        if (log) {
            oracle_xrec* rec = &log[*nlog];
            rec->attempt = k;
            rec->slot_lo = j;
            rec->slot_hi = h;
            rec->pad = 0;
            rec->rep_a = a;
            rec->rep_b = b;
            rec->accepted = acc;
            rec->step_a = steps ? steps[a] : 0;
            rec->step_b = steps ? steps[b] : 0;
            rec->U_a = U[a];
            rec->U_b = U[b];
            rec->T_a = Tl[j];
            rec->T_b = Tl[h];
            rec->u = u;
            *nlog += 1;
        }
        if (attempts) attempts[j] += 1;
        if (acc) {
            if (accepts) accepts[j] += 1;
            slot[a] = h;
            slot[b] = j;
            alpha[a] = sqrt(Tl[h] / Tl[j]);
            alpha[b] = sqrt(Tl[j] / Tl[h]);
        }
    }
    free(rep);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* A replica-exchange run.  Replicas are independent between attempts (one
 * computing node per replica in the paper), so the segments between two
 * attempts run in parallel over replicas.
 *
 * sched == NULL: synchronous variant (Implementation section, last
 *   paragraph): every replica attempts after each N_x of its own steps; runs
 *   until every replica has done nsteps more steps.
 * sched != NULL: replay of an asynchronous run: for attempt a (global index
 *   k0 + a) replica r joins at its step sched[a*R + r] (nondecreasing in a).
 *   nsteps is ignored.  k0 is the global index of the first replayed
 *   attempt (unused in the synchronous variant).
 *
 * Per-replica state arrays (offsets off[r] into the concatenated per-atom
 * arrays of 3 N_r doubles): x, v, F (forces at x), xref; steps[r], U[r],
 * rebuilds[r], slot[r].  At an attempt the velocities of every replica are
 * multiplied by its factor.  attempts/accepts are per ladder pair (R - 1).  */
int oracle_run(int32_t R, const int32_t* N, const int64_t* off, const double* L, const double* Tl,
               double rc, double skin, double dt, double gamma, int thermostat, double tau,
               int32_t max_distance, uint64_t seed, int use_list,
               double* x, double* v, double* F, double* xref,
               int64_t* steps, double* U, int64_t* rebuilds, int32_t* slot,
               int64_t nsteps, int32_t Nx, const int64_t* sched, int64_t A, int64_t k0,
               int64_t* attempts, int64_t* accepts, oracle_xrec* log, int64_t* nlog)
{
    double* alpha = (double*)malloc(sizeof(double) * (size_t)R);
    int64_t* target = (int64_t*)malloc(sizeof(int64_t) * (size_t)R);
    if (!alpha || !target) { free(alpha); free(target); return -2; }
    int64_t base = steps[0];
    if (!sched) {
        for (int r = 1; r < R; ++r)
            if (steps[r] != base) { free(alpha); free(target); return -1; }
    }
    int err = 0;
    int64_t a = 0;
    for (;;) {
        int do_exchange;
        if (sched) {
            if (a >= A) break;
            for (int r = 0; r < R; ++r) target[r] = sched[a * R + r];
            do_exchange = 1;
        } else {
            /* next multiple of N_x, capped at the end of the run */
            int64_t t = (steps[0] / Nx + 1) * Nx;
            if (steps[0] >= base + nsteps) break;
            if (t > base + nsteps) t = base + nsteps;
            for (int r = 0; r < R; ++r) target[r] = t;
            do_exchange = (t % Nx) == 0;
        }
        ++a;
        for (int r = 0; r < R; ++r)
            if (target[r] < steps[r]) err = -1;
        if (err) break;
#pragma omp parallel for schedule(dynamic, 1)
        for (int r = 0; r < R; ++r) {
            double Tr = Tl[slot[r]];
            int64_t n = target[r] - steps[r];
            int e = oracle_md(N[r], L[r], rc, skin, dt, gamma, Tr, seed, r, steps[r], n,
                              x + off[r], v + off[r], F + off[r], xref + off[r],
                              &rebuilds[r], &U[r], use_list, thermostat, tau);
            if (e) err = e;
            steps[r] = target[r];
        }
        if (err) break;
        if (do_exchange) {
            /* synchronous attempt k happens at step (k + 1) N_x */
            int64_t k = sched ? k0 + a - 1 : (steps[0] / Nx) - 1;
            oracle_exchange(R, Tl, slot, U, steps, seed, k, max_distance, alpha, attempts, accepts, log, nlog);
            for (int r = 0; r < R; ++r)
                if (alpha[r] != 1.0)
                    for (int64_t i = 0; i < 3 * (int64_t)N[r]; ++i) v[off[r] + i] *= alpha[r];
        }
    }
    free(alpha);
    free(target);
    return err;
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
