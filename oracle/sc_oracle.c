/*
 * FP64 CPU oracle for the single-relaxation-time Shan-Chen D3Q19 lattice
 * Boltzmann update (Chiappini, Xue, Falcucci & Sbragaglia, "Ligament break-up
 * simulation through pseudo-potential Lattice Boltzmann Method", Section 2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * statement of what the GPU library computes.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code,
 * header or table with the GPU library; it includes only libc/libm headers.
 *
 * Structure (deliberately different from the GPU path):
 *   - two lattices, PUSH streaming: the post-collision value at x is written to
 *     x + c_a in the second lattice;
 *   - rho and psi over the whole grid in a loop of their own, before any
 *     collision (psi at time t from the density at time t everywhere);
 *   - OpenMP over (z, y) rows only; no tiling, no fusion beyond the order
 *     of Eq. (3).
 *
 * Layout: f[a][z][y][x], a in 0..18, x fastest; node index ((z*ny)+y)*nx+x.
 * Direction order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = the 12 edge
 * directions in opposite pairs (+x+y,-x-y), (+x-y,-x+y), (+x+z,-x-z),
 * (+x-z,-x+z), (+y+z,-y-z), (+y-z,-y+z).
 *
 * Readings of the paper taken here (each is listed with its justification in
 * the design notes of the repository):
 *   - Eq. (2) printed without the leading "1 +"; the standard second-order
 *     equilibrium with the 1 is used (otherwise sum_a f^eq = 0, not rho).
 *   - c_s^2 = 1/3 and dt = dx = 1 (lattice units, D3Q19).
 *   - The interaction enters ONLY through the velocity shift of Eq. (6)
 *     (F_a of Eq. (3) taken as zero), as the text following Eq. (5) states.
 *   - G is signed; attraction (phase separation) needs G < 0; the paper's
 *     "G0 = 5.3" of Section 4 is G = -5.3.
 *   - Force weights in Eq. (5) are the D3Q19 weights w_a.
 *   - Periodic boundaries in x, y and z.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* D3Q19 velocity set (Section 2) */
static const int CXO[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CYO[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZO[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

/* D3Q19 weights: 1/3 rest, 1/18 faces, 1/36 edges */
static double weight(int a)
{
    if (a == 0) return 1.0 / 3.0;
    if (a <= 6) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

static const double CS2 = 1.0 / 3.0;

static int wrap(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

static size_t node(int x, int y, int z, int nx, int ny)
{
    return ((size_t)z * (size_t)ny + (size_t)y) * (size_t)nx + (size_t)x;
}

/* Number of OpenMP threads the oracle's loops use. */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_lattice(int *cx, int *cy, int *cz, double *w)
{
    for (int a = 0; a < Q; ++a) {
        cx[a] = CXO[a];
        cy[a] = CYO[a];
        cz[a] = CZO[a];
        w[a] = weight(a);
    }
}

/* pseudo-potential below Eq. (5): psi = rho0 * (1 - exp(-rho/rho0)) */
double orc_psi(double rho, double rho0)
{
    return rho0 * (1.0 - exp(-rho / rho0));
}

/* equation of state, Eq. (7): P = rho c_s^2 + c_s^2 G psi^2 / 2 */
double orc_pressure(double rho, double G, double rho0)
{
    double p = orc_psi(rho, rho0);
    return rho * CS2 + CS2 * G * p * p / 2.0;
}

/* second-order equilibrium, Eq. (2) with the leading 1 (see header) */
void orc_feq(double rho, double ux, double uy, double uz, double *feq)
{
    double uu = ux * ux + uy * uy + uz * uz;
    for (int a = 0; a < Q; ++a) {
        double cu = CXO[a] * ux + CYO[a] * uy + CZO[a] * uz;
        feq[a] = weight(a) * rho *
                 (1.0 + cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
    }
}

/* Density of every node, Eq. (4) (zeroth moment). */
static void density_field(int nx, int ny, int nz, const double *f, double *rho)
{
    long n = (long)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i) {
        double s = 0.0;
        for (int a = 0; a < Q; ++a) s += f[(size_t)a * n + i];
        rho[i] = s;
    }
}

/* Shan-Chen force at one node, Eq. (5): F = -G psi(x) sum_a w_a psi(x+c_a) c_a */
static void force_at(int x, int y, int z, int nx, int ny, int nz, double G,
                     const double *psi, double *F)
{
    double sx = 0.0, sy = 0.0, sz = 0.0;
    for (int a = 1; a < Q; ++a) {
        size_t j = node(wrap(x + CXO[a], nx), wrap(y + CYO[a], ny), wrap(z + CZO[a], nz), nx, ny);
        sx += weight(a) * psi[j] * CXO[a];
        sy += weight(a) * psi[j] * CYO[a];
        sz += weight(a) * psi[j] * CZO[a];
    }
    double pc = psi[node(x, y, z, nx, ny)];
    F[0] = -G * pc * sx;
    F[1] = -G * pc * sy;
    F[2] = -G * pc * sz;
}

/*
 * One time step, Eq. (3) with the velocity shift of Eq. (6):
 *   rho, psi everywhere; then per node F (Eq. 5), u = j/rho (Eq. 4),
 *   u' = u + tau F / rho (Eq. 6), f* = f - (f - f^eq(rho,u'))/tau,
 *   fnext_a(x + c_a) = f*_a(x).
 * f and fnext must not alias.  rho_work and psi_work hold n doubles each.
 */
void orc_step_ws(int nx, int ny, int nz, double tau, double G, double rho0,
                 const double *f, double *fnext, double *rho_work, double *psi_work)
{
    size_t n = (size_t)nx * ny * nz;
    density_field(nx, ny, nz, f, rho_work);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)n; ++i) psi_work[i] = orc_psi(rho_work[i], rho0);

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                size_t i = node(x, y, z, nx, ny);
                double fl[Q], feq[Q], F[3];
                double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
                for (int a = 0; a < Q; ++a) {
                    fl[a] = f[(size_t)a * n + i];
                    rho += fl[a];
                    jx += CXO[a] * fl[a];
                    jy += CYO[a] * fl[a];
                    jz += CZO[a] * fl[a];
                }
                force_at(x, y, z, nx, ny, nz, G, psi_work, F);
                double ux = jx / rho + tau * F[0] / rho;
                double uy = jy / rho + tau * F[1] / rho;
                double uz = jz / rho + tau * F[2] / rho;
                orc_feq(rho, ux, uy, uz, feq);
                for (int a = 0; a < Q; ++a) {
                    double fs = fl[a] - (fl[a] - feq[a]) / tau;
                    size_t d = node(wrap(x + CXO[a], nx), wrap(y + CYO[a], ny),
                                    wrap(z + CZO[a], nz), nx, ny);
                    fnext[(size_t)a * n + d] = fs;
                }
            }
        }
    }
}

int orc_step(int nx, int ny, int nz, double tau, double G, double rho0,
             const double *f, double *fnext)
{
    size_t n = (size_t)nx * ny * nz;
    double *rho = (double *)malloc(n * sizeof(double));
    double *psi = (double *)malloc(n * sizeof(double));
    if (!rho || !psi) {
        free(rho);
        free(psi);
        return -1;
    }
    orc_step_ws(nx, ny, nz, tau, G, rho0, f, fnext, rho, psi);
    free(rho);
    free(psi);
    return 0;
}

/* nsteps updates in place on f (fnext is scratch of the same size). */
int orc_run(int nx, int ny, int nz, double tau, double G, double rho0, long nsteps,
            double *f, double *scratch)
{
    size_t n = (size_t)nx * ny * nz;
    double *rho = (double *)malloc(n * sizeof(double));
    double *psi = (double *)malloc(n * sizeof(double));
    if (!rho || !psi) {
        free(rho);
        free(psi);
        return -1;
    }
    double *a = f, *b = scratch;
    for (long s = 0; s < nsteps; ++s) {
        orc_step_ws(nx, ny, nz, tau, G, rho0, a, b, rho, psi);
        double *t = a;
        a = b;
        b = t;
    }
    if (a != f) memcpy(f, a, (size_t)Q * n * sizeof(double));
    free(rho);
    free(psi);
    return 0;
}

/*
 * Multiple-relaxation-time collision: the variant the paper's conclusion
 * names as future work (collision operators other than BGK, which would let
 * the viscosity change at a fixed density ratio).  The paper gives no
 * details; this follows the D3Q19 moment basis of d'Humieres, Ginzburg,
 * Krafczyk, Lallemand and Luo (Phil. Trans. R. Soc. A 360, 2002), with the
 * equilibrium moments that are the projections of the second-order
 * equilibrium of Eq. (2), so that equal rates reproduce BGK.
 *
 * Moments, in order: rho, e, eps, jx, qx, jy, qy, jz, qz, 3pxx, 3pixx, pww,
 * piww, pxy, pyz, pxz, mx, my, mz; row k of M is the polynomial of c that
 * defines moment k (mrt_row below), m = M f.
 *
 * Force: the velocity shift of Eq. (6) carried over to moment space: the
 * equilibrium moments are evaluated at the momentum j' = j + F / s_j, s_j the
 * rate of the momentum moments, so one collision adds exactly F to j (as
 * BGK with s_j = 1/tau does).
 *
 * s[19] holds the rate of every moment (s[0] is irrelevant: rho is its own
 * equilibrium).
 */
static double mrt_row(int k, int a)
{
    double x = CXO[a], y = CYO[a], z = CZO[a];
    double c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * c2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * c2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * c2 - 9.0) * z;
    case 9: return 3.0 * x * x - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}

/* The matrix M, row-major [19][19]. */
void orc_mrt_matrix(double *M)
{
    for (int k = 0; k < Q; ++k)
        for (int a = 0; a < Q; ++a) M[k * Q + a] = mrt_row(k, a);
}

/* Equilibrium moments at density rho and momentum (jx, jy, jz). */
void orc_mrt_equilibrium(double rho, double jx, double jy, double jz, double *meq)
{
    double jj = jx * jx + jy * jy + jz * jz;
    meq[0] = rho;
    meq[1] = -11.0 * rho + 19.0 * jj / rho;
    meq[2] = 3.0 * rho - 5.5 * jj / rho;
    meq[3] = jx;
    meq[4] = -2.0 / 3.0 * jx;
    meq[5] = jy;
    meq[6] = -2.0 / 3.0 * jy;
    meq[7] = jz;
    meq[8] = -2.0 / 3.0 * jz;
    meq[9] = (3.0 * jx * jx - jj) / rho;
    meq[10] = -0.5 * meq[9];
    meq[11] = (jy * jy - jz * jz) / rho;
    meq[12] = -0.5 * meq[11];
    meq[13] = jx * jy / rho;
    meq[14] = jy * jz / rho;
    meq[15] = jx * jz / rho;
    meq[16] = meq[17] = meq[18] = 0.0;
}

/*
 * One step with the MRT collision: rho, psi everywhere; per node F (Eq. 5),
 * m = M f, m* = m - S (m - m^eq(rho, j + F/s_j)), f* = M^-1 m* (M has
 * orthogonal rows, so M^-1 = M^T diag(1/|row|^2)), fnext_a(x + c_a) = f*_a.
 */
void orc_step_mrt_ws(int nx, int ny, int nz, const double *s, double G, double rho0,
                     const double *f, double *fnext, double *rho_work, double *psi_work)
{
    size_t n = (size_t)nx * ny * nz;
    double M[Q][Q], norm[Q];
    for (int k = 0; k < Q; ++k) {
        norm[k] = 0.0;
        for (int a = 0; a < Q; ++a) {
            M[k][a] = mrt_row(k, a);
            norm[k] += M[k][a] * M[k][a];
        }
    }
    density_field(nx, ny, nz, f, rho_work);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < (long)n; ++i) psi_work[i] = orc_psi(rho_work[i], rho0);

#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z) {
        for (int y = 0; y < ny; ++y) {
            for (int x = 0; x < nx; ++x) {
                size_t i = node(x, y, z, nx, ny);
                double fl[Q], m[Q], meq[Q], F[3];
                for (int a = 0; a < Q; ++a) fl[a] = f[(size_t)a * n + i];
                for (int k = 0; k < Q; ++k) {
                    m[k] = 0.0;
                    for (int a = 0; a < Q; ++a) m[k] += M[k][a] * fl[a];
                }
                force_at(x, y, z, nx, ny, nz, G, psi_work, F);
                orc_mrt_equilibrium(m[0], m[3] + F[0] / s[3], m[5] + F[1] / s[5], m[7] + F[2] / s[7], meq);
                for (int k = 0; k < Q; ++k) m[k] -= s[k] * (m[k] - meq[k]);
                for (int a = 0; a < Q; ++a) {
                    double fs = 0.0;
                    for (int k = 0; k < Q; ++k) fs += M[k][a] * m[k] / norm[k];
                    size_t d = node(wrap(x + CXO[a], nx), wrap(y + CYO[a], ny),
                                    wrap(z + CZO[a], nz), nx, ny);
                    fnext[(size_t)a * n + d] = fs;
                }
            }
        }
    }
}

/* nsteps MRT updates in place on f (fnext is scratch of the same size). */
int orc_run_mrt(int nx, int ny, int nz, const double *s, double G, double rho0, long nsteps,
                double *f, double *scratch)
{
    size_t n = (size_t)nx * ny * nz;
    double *rho = (double *)malloc(n * sizeof(double));
    double *psi = (double *)malloc(n * sizeof(double));
    if (!rho || !psi) {
        free(rho);
        free(psi);
        return -1;
    }
    double *a = f, *b = scratch;
    for (long t = 0; t < nsteps; ++t) {
        orc_step_mrt_ws(nx, ny, nz, s, G, rho0, a, b, rho, psi);
        double *tmp = a;
        a = b;
        b = tmp;
    }
    if (a != f) memcpy(f, a, (size_t)Q * n * sizeof(double));
    free(rho);
    free(psi);
    return 0;
}

/*
 * Macroscopic fields of a state: rho (Eq. 4), bare momentum j = sum_a c_a f_a
 * (Eq. 4), force F (Eq. 5), and the physical velocity (j + F/2)/rho.
 * Any output pointer may be NULL.  Vector fields are [3][n].
 */
int orc_fields(int nx, int ny, int nz, double G, double rho0, const double *f,
               double *rho_out, double *j_out, double *F_out, double *u_out)
{
    size_t n = (size_t)nx * ny * nz;
    double *rho = (double *)malloc(n * sizeof(double));
    double *psi = (double *)malloc(n * sizeof(double));
    if (!rho || !psi) {
        free(rho);
        free(psi);
        return -1;
    }
    density_field(nx, ny, nz, f, rho);
    for (size_t i = 0; i < n; ++i) psi[i] = orc_psi(rho[i], rho0);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t i = node(x, y, z, nx, ny);
                double j[3] = {0.0, 0.0, 0.0}, F[3];
                for (int a = 0; a < Q; ++a) {
                    double v = f[(size_t)a * n + i];
                    j[0] += CXO[a] * v;
                    j[1] += CYO[a] * v;
                    j[2] += CZO[a] * v;
                }
                force_at(x, y, z, nx, ny, nz, G, psi, F);
                if (rho_out) rho_out[i] = rho[i];
                for (int d = 0; d < 3; ++d) {
                    if (j_out) j_out[(size_t)d * n + i] = j[d];
                    if (F_out) F_out[(size_t)d * n + i] = F[d];
                    if (u_out) u_out[(size_t)d * n + i] = (j[d] + 0.5 * F[d]) / rho[i];
                }
            }
    free(rho);
    free(psi);
    return 0;
}

/*
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), used as a counter-based
 * generator: the output for counter value s is the first output of a
 * generator whose state is s.
 */
uint64_t orc_splitmix64(uint64_t s)
{
    uint64_t z = s + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* uniform in [0,1) from the top 53 bits of SplitMix64(seed + index) */
double orc_uniform(uint64_t seed, uint64_t index)
{
    return (double)(orc_splitmix64(seed + index) >> 11) * (1.0 / 9007199254740992.0);
}

/*
 * Ligament initial condition (Section 3, Fig. 1), written with a cosine and an
 * integer number of waves so that it is periodic along the axis:
 *   R(s)  = R0 (1 + amp_rel cos(2 pi s / wavelength)),   s = axis coordinate
 *   rho   = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (r - R(s)) / width)
 *   rho  += noise_amp (2U - 1),  U = uniform(seed, node index)
 *   f_a   = w_a rho   (equilibrium at rest).
 * r is the distance from (c1, c2) in the plane normal to the axis; c1 and c2
 * are coordinates along the lower- and higher-numbered in-plane axes.
 */
int orc_init_ligament(int nx, int ny, int nz, int axis, double R0, double amp_rel,
                      double wavelength, double c1, double c2, double width,
                      double rho_l, double rho_v, double noise_amp, uint64_t seed,
                      double *f)
{
    if (axis < 0 || axis > 2) return -1;
    size_t n = (size_t)nx * ny * nz;
    const double two_pi = 6.283185307179586476925286766559;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t i = node(x, y, z, nx, ny);
                double s, p1, p2;
                if (axis == 0) {
                    s = x; p1 = y; p2 = z;
                } else if (axis == 1) {
                    s = y; p1 = x; p2 = z;
                } else {
                    s = z; p1 = x; p2 = y;
                }
                double r = sqrt((p1 - c1) * (p1 - c1) + (p2 - c2) * (p2 - c2));
                double R = R0 * (1.0 + amp_rel * cos(two_pi * s / wavelength));
                double rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * tanh(2.0 * (r - R) / width);
                if (noise_amp != 0.0) rho += noise_amp * (2.0 * orc_uniform(seed, (uint64_t)i) - 1.0);
                for (int a = 0; a < Q; ++a) f[(size_t)a * n + i] = weight(a) * rho;
            }
    return 0;
}

/*
 * Global diagnostics of a state:
 *   out[0] total mass sum rho, out[1..3] total bare momentum sum j,
 *   out[4] min rho, out[5] max rho,
 *   out[6] neck = min over the axis coordinate of the max of rho over the
 *          cross-section (the thinnest point of the ligament),
 *   out[7] number of nodes whose rho or any population is non-finite, or
 *          whose rho <= 0.
 * Sums use Neumaier compensated summation in node order.
 */
static void neumaier_add(double *s, double *c, double v)
{
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

int orc_diag(int nx, int ny, int nz, int axis, const double *f, double *out)
{
    size_t n = (size_t)nx * ny * nz;
    int ns = axis == 0 ? nx : (axis == 1 ? ny : nz);
    double *smax = (double *)malloc((size_t)ns * sizeof(double));
    if (!smax) return -1;
    for (int s = 0; s < ns; ++s) smax[s] = -INFINITY;
    double m = 0, mc = 0, p[3] = {0, 0, 0}, pc[3] = {0, 0, 0};
    double rmin = INFINITY, rmax = -INFINITY;
    double bad = 0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                size_t i = node(x, y, z, nx, ny);
                double rho = 0.0, j[3] = {0, 0, 0};
                int finite = 1;
                for (int a = 0; a < Q; ++a) {
                    double v = f[(size_t)a * n + i];
                    if (!isfinite(v)) finite = 0;
                    rho += v;
                    j[0] += CXO[a] * v;
                    j[1] += CYO[a] * v;
                    j[2] += CZO[a] * v;
                }
                if (!finite || !isfinite(rho) || !(rho > 0.0)) bad += 1;
                neumaier_add(&m, &mc, rho);
                for (int d = 0; d < 3; ++d) neumaier_add(&p[d], &pc[d], j[d]);
                if (rho < rmin) rmin = rho;
                if (rho > rmax) rmax = rho;
                int s = axis == 0 ? x : (axis == 1 ? y : z);
                if (rho > smax[s]) smax[s] = rho;
            }
    double neck = INFINITY;
    for (int s = 0; s < ns; ++s)
        if (smax[s] < neck) neck = smax[s];
    out[0] = m + mc;
    out[1] = p[0] + pc[0];
    out[2] = p[1] + pc[1];
    out[3] = p[2] + pc[2];
    out[4] = rmin;
    out[5] = rmax;
    out[6] = neck;
    out[7] = bad;
    free(smax);
    return 0;
}

/*
 * Droplet labelling: 6-connected components of the set {rho > thresh} on the
 * periodic grid, by an explicit-stack flood fill in node order.  label[i] is
 * the 1-based component id, 0 outside the set.  Returns the component count,
 * or -1 on allocation failure.
 */
long orc_label(int nx, int ny, int nz, const double *rho, double thresh, int32_t *label)
{
    size_t n = (size_t)nx * ny * nz;
    size_t *stack = (size_t *)malloc((n + 1) * sizeof(size_t));
    if (!stack) return -1;
    for (size_t i = 0; i < n; ++i) label[i] = 0;
    long count = 0;
    for (size_t seed = 0; seed < n; ++seed) {
        if (label[seed] != 0 || !(rho[seed] > thresh)) continue;
        ++count;
        size_t top = 0;
        stack[top++] = seed;
        label[seed] = (int32_t)count;
        while (top > 0) {
            size_t i = stack[--top];
            int x = (int)(i % (size_t)nx);
            int y = (int)((i / (size_t)nx) % (size_t)ny);
            int z = (int)(i / ((size_t)nx * (size_t)ny));
            /* the six face neighbours are directions 1..6 of the lattice */
            for (int a = 1; a <= 6; ++a) {
                size_t j = node(wrap(x + CXO[a], nx), wrap(y + CYO[a], ny), wrap(z + CZO[a], nz), nx, ny);
                if (label[j] == 0 && rho[j] > thresh) {
                    label[j] = (int32_t)count;
                    stack[top++] = j;
                }
            }
        }
    }
    free(stack);
    return count;
}
