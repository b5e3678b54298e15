/*
 * pic_oracle.c -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * A plain, slow, obviously-correct FP64 CPU reference of one timestep of the
 * 2D electromagnetic particle-in-cell (EM-PIC) cycle studied in
 * "Particle-In-Cell Simulation using Asynchronous Tasking" (Guidotti et al.,
 * arXiv 2106.12485).  The paper describes the cycle in Sec. 2.2 (Fig. 1):
 *   (1) bilinear interpolation of the previous-iteration E, B to each particle,
 *   (2) leapfrog + Boris particle advance (second order in time),
 *   (3) exact charge-conserving current deposition (Villasenor-Buneman),
 *       optionally followed by a digital (binomial) current filter,
 *   (4) finite-difference time-domain field advance on a Yee mesh.
 * Sec. 4.1 adds the LWFA extras: laser-initialised fields, a compensated
 * binomial filter, a moving window and immobile neutralising ions.
 *
 * Everything is global arrays, particles in array order, no tiles, no
 * blocking, no fusion.  Only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg may load this file.  It shares no code with the HIP path.
 *
 * By default everything runs on one thread.  orc_set_threads(s, n > 1)
 * switches on the paper's own multicore strategy for the particle loop
 * (Sec. 3.1, "parallel for"): the particles are cut into n contiguous
 * chunks, each thread deposits into a private copy of the current, and the
 * copies are summed in thread order.  Particles come out identical to the
 * one-thread run; the current differs only by the order of the FP64 sums.
 * The grid loops (filter, Yee, window shift) are split over rows, which
 * changes no result.
 *
 * Where the paper is silent the readings are:
 *   - normalised units: c = 1, time in 1/w_p, length in c/w_p, u = gamma v,
 *     fields in m c w_p / e, dE/dt = curl B - J, dB/dt = -curl E, div E = rho;
 *   - standard 2D Yee staggering: Ex(i+1/2,j) Ey(i,j+1/2) Ez(i,j)
 *     Bx(i,j+1/2) By(i+1/2,j) Bz(i+1/2,j+1/2); J_k sits with E_k, rho on nodes;
 *     array element [i + j*nx] of each plane holds the value at that position;
 *   - E and B both live at integer time; the field advance is
 *     B half step, E full step, B half step;
 *   - relativistic Boris push, initial u taken as u^{-1/2};
 *   - Villasenor-Buneman split of the straight path at cell boundaries in the
 *     order the path crosses them; Jz carries the exact time average of the
 *     bilinear node weights along each segment;
 *   - binomial 1-2-1 filter, N passes along x then a compensator
 *     (-N, 4+2N, -N)/4, then the same along y;
 *   - y is always periodic; x is periodic, or, with the moving window, fields
 *     beyond the box are held at zero, current deposited beyond it is dropped
 *     and particles that leave it are removed after depositing;
 *   - particle loading: ppc_x*ppc_y particles per cell at sub-cell centres,
 *     u = ufl + uth*N(0,1) with normals from Philox4x32-10 (Salmon et al.,
 *     SC'11) + Box-Muller, keyed by the seed and counted by
 *     (lab cell x, cell y, sub-position, species).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_SPECIES 8

typedef struct {
    double qm;        /* charge-to-mass ratio (units e/m_e) */
    double qp;        /* charge of one macro-particle: sign(qm)*density/ppc */
    double density, x_lo, x_hi;
    int ppc_x, ppc_y;
    double uth[3], ufl[3];
    long long n, cap;
    int *ix, *iy;
    double *x, *y, *ux, *uy, *uz;
} orc_species;

typedef struct {
    int nx, ny;
    double dx, dy, dt;
    int window;       /* 1: moving window along x (x not periodic) */
    int npass;        /* binomial passes per axis */
    int compensate;   /* 1: apply the compensator after the passes */
    unsigned long long seed;
    long long iter;   /* completed steps */
    int nshift;       /* window shifts done */
    double *e[3], *b[3];
    double *jr[3];    /* current of the last deposit, before filtering */
    double *jf[3];    /* current actually used by the field solver */
    int nsp;
    orc_species sp[ORC_MAX_SPECIES];
    int nthreads;     /* 1: sequential; n > 1: parallel particle loop */
    double *priv;     /* private current copies of the parallel loop */
    int priv_nt;
} orc_sim;

/* ------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw,  */
/* "Parallel random numbers: as easy as 1, 2, 3", SC'11), from its     */
/* published definition: 10 rounds of the 4x32 S-box with multipliers  */
/* 0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9,          */
/* 0xBB67AE85.                                                         */
/* ------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Box-Muller on two pairs of 32-bit words: u1 in (0,1], u2 in [0,1). */
void orc_normals4(const uint32_t r[4], double n[4])
{
    const double two32 = 4294967296.0;
    for (int p = 0; p < 2; ++p) {
        double u1 = ((double)r[2 * p] + 1.0) / two32;
        double u2 = (double)r[2 * p + 1] / two32;
        double rad = sqrt(-2.0 * log(u1));
        double ang = 2.0 * M_PI * u2;
        n[2 * p] = rad * cos(ang);
        n[2 * p + 1] = rad * sin(ang);
    }
}

/* ------------------------------------------------------------------ */
/* grid access with the boundary rules                                 */
/* ------------------------------------------------------------------ */
static int imod(int a, int n)
{
    int r = a % n;
    return r < 0 ? r + n : r;
}

static double fget(const orc_sim *s, const double *f, int i, int j)
{
    j = imod(j, s->ny);
    if (s->window) {
        if (i < 0 || i >= s->nx) return 0.0;
    } else {
        i = imod(i, s->nx);
    }
    return f[i + (size_t)j * s->nx];
}

static void fadd(const orc_sim *s, double *f, int i, int j, double v)
{
    j = imod(j, s->ny);
    if (s->window) {
        if (i < 0 || i >= s->nx) return; /* dropped outside the window */
    } else {
        i = imod(i, s->nx);
    }
    f[i + (size_t)j * s->nx] += v;
}

/* ------------------------------------------------------------------ */
/* creation                                                            */
/* ------------------------------------------------------------------ */
orc_sim *orc_create(int nx, int ny, double lx, double ly, double dt, int window,
                    int npass, int compensate, unsigned long long seed)
{
    if (nx < 1 || ny < 1) return NULL;
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    s->nx = nx;
    s->ny = ny;
    s->dx = lx / nx;
    s->dy = ly / ny;
    s->dt = dt;
    s->window = window;
    s->npass = npass;
    s->compensate = compensate;
    s->seed = seed;
    s->nthreads = 1;
    size_t nc = (size_t)nx * ny;
    for (int c = 0; c < 3; ++c) {
        s->e[c] = (double *)calloc(nc, sizeof(double));
        s->b[c] = (double *)calloc(nc, sizeof(double));
        s->jr[c] = (double *)calloc(nc, sizeof(double));
        s->jf[c] = (double *)calloc(nc, sizeof(double));
    }
    return s;
}

static void sp_free(orc_species *p)
{
    free(p->ix); free(p->iy); free(p->x); free(p->y);
    free(p->ux); free(p->uy); free(p->uz);
    p->n = 0;
    p->cap = 0;
    p->ix = p->iy = NULL;
    p->x = p->y = p->ux = p->uy = p->uz = NULL;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    for (int c = 0; c < 3; ++c) {
        free(s->e[c]); free(s->b[c]); free(s->jr[c]); free(s->jf[c]);
    }
    free(s->priv);
    for (int k = 0; k < s->nsp; ++k) sp_free(&s->sp[k]);
    free(s);
}

static void sp_reserve(orc_species *p, long long need)
{
    if (need <= p->cap) return;
    long long cap = p->cap ? p->cap : 1024;
    while (cap < need) cap *= 2;
    p->ix = (int *)realloc(p->ix, cap * sizeof(int));
    p->iy = (int *)realloc(p->iy, cap * sizeof(int));
    p->x = (double *)realloc(p->x, cap * sizeof(double));
    p->y = (double *)realloc(p->y, cap * sizeof(double));
    p->ux = (double *)realloc(p->ux, cap * sizeof(double));
    p->uy = (double *)realloc(p->uy, cap * sizeof(double));
    p->uz = (double *)realloc(p->uz, cap * sizeof(double));
    p->cap = cap;
}

static void sp_append(orc_species *p, int ix, int iy, double x, double y,
                      double ux, double uy, double uz)
{
    sp_reserve(p, p->n + 1);
    long long k = p->n++;
    p->ix[k] = ix; p->iy[k] = iy; p->x[k] = x; p->y[k] = y;
    p->ux[k] = ux; p->uy[k] = uy; p->uz[k] = uz;
}

/* Load one cell (window column i_win, row j) of species k on the lattice of
 * sub-cell centres, where the lab-frame x of the particle lies in
 * [x_lo, x_hi). */
static void load_cell(orc_sim *s, int k, int i_win, int j)
{
    orc_species *p = &s->sp[k];
    if (p->density <= 0.0) return;
    long long ilab = (long long)i_win + s->nshift;
    uint32_t key[2] = {(uint32_t)(s->seed & 0xffffffffu), (uint32_t)(s->seed >> 32)};
    for (int l = 0; l < p->ppc_y; ++l) {
        for (int m = 0; m < p->ppc_x; ++m) {
            double xo = ((double)m + 0.5) / (double)p->ppc_x;
            double yo = ((double)l + 0.5) / (double)p->ppc_y;
            double xlab = ((double)ilab + xo) * s->dx;
            if (!(xlab >= p->x_lo && xlab < p->x_hi)) continue;
            uint32_t ctr[4] = {(uint32_t)ilab, (uint32_t)j, (uint32_t)(l * p->ppc_x + m), (uint32_t)k};
            uint32_t r[4];
            double nrm[4];
            orc_philox4x32_10(ctr, key, r);
            orc_normals4(r, nrm);
            sp_append(p, i_win, j, xo, yo,
                      p->ufl[0] + p->uth[0] * nrm[0],
                      p->ufl[1] + p->uth[1] * nrm[1],
                      p->ufl[2] + p->uth[2] * nrm[2]);
        }
    }
}

int orc_add_species(orc_sim *s, double qm, double density, double x_lo, double x_hi,
                    int ppc_x, int ppc_y, const double *uth, const double *ufl, int load)
{
    if (s->nsp >= ORC_MAX_SPECIES || ppc_x < 1 || ppc_y < 1) return -1;
    int k = s->nsp++;
    orc_species *p = &s->sp[k];
    memset(p, 0, sizeof(*p));
    p->qm = qm;
    p->density = density;
    p->x_lo = x_lo;
    p->x_hi = x_hi;
    p->ppc_x = ppc_x;
    p->ppc_y = ppc_y;
    for (int c = 0; c < 3; ++c) {
        p->uth[c] = uth[c];
        p->ufl[c] = ufl[c];
    }
    p->qp = (qm < 0 ? -1.0 : 1.0) * density / (double)(ppc_x * ppc_y);
    if (load) {
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) load_cell(s, k, i, j);
    }
    return k;
}

long long orc_count(const orc_sim *s, int k) { return s->sp[k].n; }
double orc_qp(const orc_sim *s, int k) { return s->sp[k].qp; }
long long orc_iter(const orc_sim *s) { return s->iter; }
int orc_nshift(const orc_sim *s) { return s->nshift; }

void orc_set_iter(orc_sim *s, long long iter, int nshift)
{
    s->iter = iter;
    s->nshift = nshift;
}

int orc_set_particles(orc_sim *s, int k, long long n, const int *ix, const int *iy,
                      const double *x, const double *y, const double *ux,
                      const double *uy, const double *uz)
{
    if (k < 0 || k >= s->nsp) return -1;
    orc_species *p = &s->sp[k];
    p->n = 0;
    sp_reserve(p, n);
    for (long long q = 0; q < n; ++q) sp_append(p, ix[q], iy[q], x[q], y[q], ux[q], uy[q], uz[q]);
    return 0;
}

int orc_get_particles(const orc_sim *s, int k, int *ix, int *iy, double *x, double *y,
                      double *ux, double *uy, double *uz)
{
    if (k < 0 || k >= s->nsp) return -1;
    const orc_species *p = &s->sp[k];
    for (long long q = 0; q < p->n; ++q) {
        ix[q] = p->ix[q]; iy[q] = p->iy[q]; x[q] = p->x[q]; y[q] = p->y[q];
        ux[q] = p->ux[q]; uy[q] = p->uy[q]; uz[q] = p->uz[q];
    }
    return 0;
}

/* f: 6 planes Ex Ey Ez Bx By Bz, each nx*ny with x fastest. */
void orc_set_fields(orc_sim *s, const double *f)
{
    size_t nc = (size_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) {
        memcpy(s->e[c], f + c * nc, nc * sizeof(double));
        memcpy(s->b[c], f + (3 + c) * nc, nc * sizeof(double));
    }
}

void orc_get_fields(const orc_sim *s, double *f)
{
    size_t nc = (size_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) {
        memcpy(f + c * nc, s->e[c], nc * sizeof(double));
        memcpy(f + (3 + c) * nc, s->b[c], nc * sizeof(double));
    }
}

/* j: 3 planes Jx Jy Jz; filtered != 0 returns the current the field solver used. */
void orc_get_current(const orc_sim *s, int filtered, double *j)
{
    size_t nc = (size_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) memcpy(j + c * nc, filtered ? s->jf[c] : s->jr[c], nc * sizeof(double));
}

void orc_set_current(orc_sim *s, const double *j)
{
    size_t nc = (size_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) memcpy(s->jr[c], j + c * nc, nc * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* laser initialisation (Sec. 4.1: fields start with the laser's).     */
/* A 2D paraxial Gaussian beam travelling along +x, evaluated at each  */
/* component's own staggered position at t = 0.                        */
/* ------------------------------------------------------------------ */
static double laser_eperp(double x, double y, double a0, double w0, double W0,
                          double fwhm, double xc, double focus, double axis)
{
    double d = x - xc;
    if (fabs(d) > 2.0 * fwhm) return 0.0;
    double env = exp(-2.0 * log(2.0) * d * d / (fwhm * fwhm));
    double z = x - focus;
    double r = y - axis;
    double zr = w0 * W0 * W0 / 2.0;
    double w = W0 * sqrt(1.0 + (z * z) / (zr * zr));
    double curv = (z == 0.0) ? 0.0 : w0 * r * r / (2.0 * (z * (1.0 + (zr * zr) / (z * z))));
    double gouy = 0.5 * atan(z / zr);
    return a0 * w0 * env * sqrt(W0 / w) * exp(-(r * r) / (w * w)) *
           cos(w0 * d + curv - gouy);
}

void orc_add_laser(orc_sim *s, double a0, double omega0, double W0, double fwhm,
                   double xc, double focus, double axis, double pol)
{
    double cp = cos(pol), sn = sin(pol);
    for (int j = 0; j < s->ny; ++j) {
        for (int i = 0; i < s->nx; ++i) {
            size_t q = i + (size_t)j * s->nx;
            double xi = i * s->dx, xh = (i + 0.5) * s->dx;
            double yj = j * s->dy, yh = (j + 0.5) * s->dy;
            /* Ey at (i, j+1/2), Ez at (i, j), By at (i+1/2, j), Bz at (i+1/2, j+1/2) */
            s->e[1][q] += cp * laser_eperp(xi, yh, a0, omega0, W0, fwhm, xc, focus, axis);
            s->e[2][q] += sn * laser_eperp(xi, yj, a0, omega0, W0, fwhm, xc, focus, axis);
            /* a wave travelling along +x has By = -Ez and Bz = Ey */
            s->b[1][q] += -sn * laser_eperp(xh, yj, a0, omega0, W0, fwhm, xc, focus, axis);
            s->b[2][q] += cp * laser_eperp(xh, yh, a0, omega0, W0, fwhm, xc, focus, axis);
        }
    }
}

/* ------------------------------------------------------------------ */
/* stage 1: bilinear interpolation of each component from its own grid */
/* ------------------------------------------------------------------ */
/* X, Y: particle coordinate in cells measured from the component's grid */
static double interp(const orc_sim *s, const double *f, double X, double Y)
{
    int i0 = (int)floor(X), j0 = (int)floor(Y);
    double wx = X - i0, wy = Y - j0;
    return (1 - wx) * (1 - wy) * fget(s, f, i0, j0) + wx * (1 - wy) * fget(s, f, i0 + 1, j0) +
           (1 - wx) * wy * fget(s, f, i0, j0 + 1) + wx * wy * fget(s, f, i0 + 1, j0 + 1);
}

void orc_gather(const orc_sim *s, int ix, int iy, double x, double y, double out[6])
{
    double X = ix + x, Y = iy + y;
    out[0] = interp(s, s->e[0], X - 0.5, Y);
    out[1] = interp(s, s->e[1], X, Y - 0.5);
    out[2] = interp(s, s->e[2], X, Y);
    out[3] = interp(s, s->b[0], X, Y - 0.5);
    out[4] = interp(s, s->b[1], X - 0.5, Y);
    out[5] = interp(s, s->b[2], X - 0.5, Y - 0.5);
}

/* ------------------------------------------------------------------ */
/* stage 2: relativistic Boris momentum update u^{n-1/2} -> u^{n+1/2}  */
/* ------------------------------------------------------------------ */
void orc_boris(double qm, double dt, const double E[3], const double B[3], double u[3])
{
    double tau = 0.5 * dt * qm;
    double um[3] = {u[0] + tau * E[0], u[1] + tau * E[1], u[2] + tau * E[2]};
    double g = sqrt(1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2]);
    double t[3] = {tau * B[0] / g, tau * B[1] / g, tau * B[2] / g};
    double up[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]),
                    um[1] + (um[2] * t[0] - um[0] * t[2]),
                    um[2] + (um[0] * t[1] - um[1] * t[0])};
    double f = 2.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    double sv[3] = {f * t[0], f * t[1], f * t[2]};
    double upl[3] = {um[0] + (up[1] * sv[2] - up[2] * sv[1]),
                     um[1] + (up[2] * sv[0] - up[0] * sv[2]),
                     um[2] + (up[0] * sv[1] - up[1] * sv[0])};
    u[0] = upl[0] + tau * E[0];
    u[1] = upl[1] + tau * E[1];
    u[2] = upl[2] + tau * E[2];
}

/* ------------------------------------------------------------------ */
/* stage 3: Villasenor-Buneman deposit of one straight segment lying   */
/* inside cell (i, j); (x0,y0)->(x1,y1) are cell-relative endpoints,   */
/* f the fraction of the timestep spent on it, vz the z velocity.      */
/* ------------------------------------------------------------------ */
static void deposit_segment(const orc_sim *s, double *const *jt, double qp, int i, int j,
                            double x0, double y0, double x1, double y1, double f, double vz)
{
    double xm = 0.5 * (x0 + x1), ym = 0.5 * (y0 + y1);
    double cx = qp * (x1 - x0) * s->dx / s->dt;
    double cy = qp * (y1 - y0) * s->dy / s->dt;
    fadd(s, jt[0], i, j, cx * (1 - ym));
    fadd(s, jt[0], i, j + 1, cx * ym);
    fadd(s, jt[1], i, j, cy * (1 - xm));
    fadd(s, jt[1], i + 1, j, cy * xm);
    /* Jz: time average over the segment of the bilinear weight of each
     * node; along a straight line the weight is a quadratic in time and its
     * average is (S0x S0y + S1x S1y)/3 + (S0x S1y + S1x S0y)/6. */
    double s0x[2] = {1 - x0, x0}, s1x[2] = {1 - x1, x1};
    double s0y[2] = {1 - y0, y0}, s1y[2] = {1 - y1, y1};
    for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
            double w = (s0x[a] * s0y[b] + s1x[a] * s1y[b]) / 3.0 +
                       (s0x[a] * s1y[b] + s1x[a] * s0y[b]) / 6.0;
            fadd(s, jt[2], i + a, j + b, qp * vz * f * w);
        }
}

/* Deposit the move of one particle starting at cell (ix, iy), offset (x, y),
 * displaced by (ddx, ddy) cells, cutting the path where it crosses a cell
 * boundary, in the order the path crosses them. */
static void deposit_move(const orc_sim *s, double *const *jt, double qp, int ix, int iy,
                         double x, double y, double ddx, double ddy, double vz)
{
    double x1 = x + ddx, y1 = y + ddy;
    double tx = 2.0, ty = 2.0;
    if (x1 >= 1.0) tx = (1.0 - x) / ddx;
    else if (x1 < 0.0) tx = (0.0 - x) / ddx;
    if (y1 >= 1.0) ty = (1.0 - y) / ddy;
    else if (y1 < 0.0) ty = (0.0 - y) / ddy;
    double tb[4];
    int nb = 0;
    tb[nb++] = 0.0;
    double ta = tx < ty ? tx : ty, tc = tx < ty ? ty : tx;
    if (ta <= 1.0) tb[nb++] = ta;
    if (tc <= 1.0) tb[nb++] = tc;
    tb[nb++] = 1.0;
    for (int k = 0; k + 1 < nb; ++k) {
        double t0 = tb[k], t1 = tb[k + 1];
        if (!(t1 > t0)) continue;
        double tm = 0.5 * (t0 + t1);
        int cx = (int)floor(x + tm * ddx), cy = (int)floor(y + tm * ddy);
        deposit_segment(s, jt, qp, ix + cx, iy + cy,
                        x + t0 * ddx - cx, y + t0 * ddy - cy,
                        x + t1 * ddx - cx, y + t1 * ddy - cy, t1 - t0, vz);
    }
}

/* Stages 1-3 for particles [q0, q1) of species p: interpolate, push, move,
 * deposit into jt.  The kept particles are written compacted from index q0
 * on; returns how many were kept.  With the moving window, particles whose
 * new position is outside the box are removed. */
static long long advance_range(const orc_sim *s, orc_species *p, double *const *jt,
                               long long q0, long long q1)
{
    long long keep = q0;
    for (long long q = q0; q < q1; ++q) {
        double fl[6];
        orc_gather(s, p->ix[q], p->iy[q], p->x[q], p->y[q], fl);
        double u[3] = {p->ux[q], p->uy[q], p->uz[q]};
        orc_boris(p->qm, s->dt, fl, fl + 3, u);
        double g = sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
        double ddx = s->dt * u[0] / (g * s->dx);
        double ddy = s->dt * u[1] / (g * s->dy);
        deposit_move(s, jt, p->qp, p->ix[q], p->iy[q], p->x[q], p->y[q], ddx, ddy, u[2] / g);
        /* new cell and offset */
        double xn = p->x[q] + ddx, yn = p->y[q] + ddy;
        int di = (int)floor(xn), dj = (int)floor(yn);
        xn -= di;
        yn -= dj;
        int ix = p->ix[q] + di, iy = p->iy[q] + dj;
        if (xn >= 1.0) { xn -= 1.0; ix += 1; }
        if (yn >= 1.0) { yn -= 1.0; iy += 1; }
        iy = imod(iy, s->ny);
        if (s->window) {
            if (ix < 0 || ix >= s->nx) continue; /* left the box: removed */
        } else {
            ix = imod(ix, s->nx);
        }
        p->ix[keep] = ix; p->iy[keep] = iy; p->x[keep] = xn; p->y[keep] = yn;
        p->ux[keep] = u[0]; p->uy[keep] = u[1]; p->uz[keep] = u[2];
        ++keep;
    }
    return keep - q0;
}

static void move_particles(orc_species *p, long long to, long long from, long long n)
{
    if (to == from || n == 0) return;
    memmove(p->ix + to, p->ix + from, n * sizeof(int));
    memmove(p->iy + to, p->iy + from, n * sizeof(int));
    memmove(p->x + to, p->x + from, n * sizeof(double));
    memmove(p->y + to, p->y + from, n * sizeof(double));
    memmove(p->ux + to, p->ux + from, n * sizeof(double));
    memmove(p->uy + to, p->uy + from, n * sizeof(double));
    memmove(p->uz + to, p->uz + from, n * sizeof(double));
}

/* Stages 1-3 for every particle.  The current of the step is accumulated in
 * jr (zeroed first). */
void orc_push_deposit(orc_sim *s)
{
    size_t nc = (size_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) memset(s->jr[c], 0, nc * sizeof(double));
    const int nt = s->nthreads;
    if (nt <= 1) {
        for (int k = 0; k < s->nsp; ++k) {
            orc_species *p = &s->sp[k];
            p->n = advance_range(s, p, s->jr, 0, p->n);
        }
        return;
    }
    /* parallel for (Sec. 3.1): contiguous chunks, private current copies */
    if (s->priv_nt != nt) {
        free(s->priv);
        s->priv = (double *)malloc((size_t)nt * 3 * nc * sizeof(double));
        s->priv_nt = nt;
    }
    double *priv = s->priv;
#pragma omp parallel for num_threads(nt) schedule(static, 1)
    for (int t = 0; t < nt; ++t) memset(priv + (size_t)t * 3 * nc, 0, 3 * nc * sizeof(double));
    long long *kept = (long long *)calloc((size_t)nt, sizeof(long long));
    for (int k = 0; k < s->nsp; ++k) {
        orc_species *p = &s->sp[k];
        const long long n = p->n;
#pragma omp parallel for num_threads(nt) schedule(static, 1)
        for (int t = 0; t < nt; ++t) {
            double *jt[3] = {priv + ((size_t)t * 3 + 0) * nc, priv + ((size_t)t * 3 + 1) * nc,
                             priv + ((size_t)t * 3 + 2) * nc};
            kept[t] = advance_range(s, p, jt, n * t / nt, n * (t + 1) / nt);
        }
        long long to = 0;
        for (int t = 0; t < nt; ++t) {
            move_particles(p, to, n * t / nt, kept[t]);
            to += kept[t];
        }
        p->n = to;
    }
    /* reduction of the private copies, in thread order */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (long long q = 0; q < (long long)nc; ++q)
        for (int c = 0; c < 3; ++c) {
            double v = 0.0;
            for (int t = 0; t < nt; ++t) v += priv[((size_t)t * 3 + c) * nc + q];
            s->jr[c][q] = v;
        }
    free(kept);
}

void orc_set_threads(orc_sim *s, int n) { s->nthreads = n < 1 ? 1 : n; }

/* ------------------------------------------------------------------ */
/* digital filter: 3-point stencil (w0, w1, w2) along one axis         */
/* ------------------------------------------------------------------ */
static void stencil_x(const orc_sim *s, double *f, double w0, double w1, double w2)
{
    size_t nc = (size_t)s->nx * s->ny;
    double *t = (double *)malloc(nc * sizeof(double));
    memcpy(t, f, nc * sizeof(double));
#pragma omp parallel for num_threads(s->nthreads) if (s->nthreads > 1)
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i)
            f[i + (size_t)j * s->nx] = w0 * fget(s, t, i - 1, j) + w1 * fget(s, t, i, j) +
                                       w2 * fget(s, t, i + 1, j);
    free(t);
}

static void stencil_y(const orc_sim *s, double *f, double w0, double w1, double w2)
{
    size_t nc = (size_t)s->nx * s->ny;
    double *t = (double *)malloc(nc * sizeof(double));
    memcpy(t, f, nc * sizeof(double));
#pragma omp parallel for num_threads(s->nthreads) if (s->nthreads > 1)
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i)
            f[i + (size_t)j * s->nx] = w0 * fget(s, t, i, j - 1) + w1 * fget(s, t, i, j) +
                                       w2 * fget(s, t, i, j + 1);
    free(t);
}

/* Apply the filter F in place to one plane: N binomial passes along x, the
 * compensator along x, then the same along y. */
void orc_filter_plane(const orc_sim *s, double *f)
{
    double N = (double)s->npass;
    for (int k = 0; k < s->npass; ++k) stencil_x(s, f, 0.25, 0.5, 0.25);
    if (s->compensate && s->npass > 0) stencil_x(s, f, -N / 4.0, (4.0 + 2.0 * N) / 4.0, -N / 4.0);
    for (int k = 0; k < s->npass; ++k) stencil_y(s, f, 0.25, 0.5, 0.25);
    if (s->compensate && s->npass > 0) stencil_y(s, f, -N / 4.0, (4.0 + 2.0 * N) / 4.0, -N / 4.0);
}

void orc_filter(orc_sim *s)
{
    size_t nc = (size_t)s->nx * s->ny;
    for (int c = 0; c < 3; ++c) {
        memcpy(s->jf[c], s->jr[c], nc * sizeof(double));
        orc_filter_plane(s, s->jf[c]);
    }
}

/* ------------------------------------------------------------------ */
/* stage 4: Yee FDTD, B half step, E full step, B half step            */
/* ------------------------------------------------------------------ */
static void b_half(orc_sim *s)
{
    double h = 0.5 * s->dt;
#pragma omp parallel for num_threads(s->nthreads) if (s->nthreads > 1)
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            size_t q = i + (size_t)j * s->nx;
            double dEz_dy = (fget(s, s->e[2], i, j + 1) - fget(s, s->e[2], i, j)) / s->dy;
            double dEz_dx = (fget(s, s->e[2], i + 1, j) - fget(s, s->e[2], i, j)) / s->dx;
            double dEy_dx = (fget(s, s->e[1], i + 1, j) - fget(s, s->e[1], i, j)) / s->dx;
            double dEx_dy = (fget(s, s->e[0], i, j + 1) - fget(s, s->e[0], i, j)) / s->dy;
            s->b[0][q] -= h * dEz_dy;
            s->b[1][q] += h * dEz_dx;
            s->b[2][q] -= h * (dEy_dx - dEx_dy);
        }
}

static void e_full(orc_sim *s)
{
    double dt = s->dt;
#pragma omp parallel for num_threads(s->nthreads) if (s->nthreads > 1)
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i) {
            size_t q = i + (size_t)j * s->nx;
            double dBz_dy = (fget(s, s->b[2], i, j) - fget(s, s->b[2], i, j - 1)) / s->dy;
            double dBz_dx = (fget(s, s->b[2], i, j) - fget(s, s->b[2], i - 1, j)) / s->dx;
            double dBy_dx = (fget(s, s->b[1], i, j) - fget(s, s->b[1], i - 1, j)) / s->dx;
            double dBx_dy = (fget(s, s->b[0], i, j) - fget(s, s->b[0], i, j - 1)) / s->dy;
            s->e[0][q] += dt * (dBz_dy - s->jf[0][q]);
            s->e[1][q] += dt * (-dBz_dx - s->jf[1][q]);
            s->e[2][q] += dt * (dBy_dx - dBx_dy - s->jf[2][q]);
        }
}

void orc_yee(orc_sim *s)
{
    b_half(s);
    e_full(s);
    b_half(s);
}

/* ------------------------------------------------------------------ */
/* moving window (Sec. 4.1): the box follows the laser at c            */
/* ------------------------------------------------------------------ */
static void window_shift(orc_sim *s)
{
    for (int c = 0; c < 6; ++c) {
        double *f = c < 3 ? s->e[c] : s->b[c - 3];
#pragma omp parallel for num_threads(s->nthreads) if (s->nthreads > 1)
        for (int j = 0; j < s->ny; ++j) {
            double *row = f + (size_t)j * s->nx;
            for (int i = 0; i + 1 < s->nx; ++i) row[i] = row[i + 1];
            row[s->nx - 1] = 0.0;
        }
    }
    for (int k = 0; k < s->nsp; ++k) {
        orc_species *p = &s->sp[k];
        long long keep = 0;
        for (long long q = 0; q < p->n; ++q) {
            int ix = p->ix[q] - 1;
            if (ix < 0) continue;
            p->ix[keep] = ix; p->iy[keep] = p->iy[q]; p->x[keep] = p->x[q]; p->y[keep] = p->y[q];
            p->ux[keep] = p->ux[q]; p->uy[keep] = p->uy[q]; p->uz[keep] = p->uz[q];
            ++keep;
        }
        p->n = keep;
    }
    s->nshift += 1;
    for (int k = 0; k < s->nsp; ++k)
        for (int j = 0; j < s->ny; ++j) load_cell(s, k, s->nx - 1, j);
}

/* Filter, field advance, step count and (if due) window shift.  The window
 * moves one cell when the light travelled since t = 0 has passed the next
 * cell boundary: iter*dt >= (nshift+1)*dx, evaluated in double. */
void orc_field_advance(orc_sim *s)
{
    orc_filter(s);
    orc_yee(s);
    s->iter += 1;
    if (s->window && (double)s->iter * s->dt >= (double)(s->nshift + 1) * s->dx) window_shift(s);
}

void orc_step(orc_sim *s, int nsteps)
{
    for (int n = 0; n < nsteps; ++n) {
        orc_push_deposit(s);
        orc_field_advance(s);
    }
}

/* ------------------------------------------------------------------ */
/* diagnostics                                                         */
/* ------------------------------------------------------------------ */
/* charge density on the nodes: bilinear (area) weights, sum over species */
void orc_charge(const orc_sim *s, double *rho)
{
    size_t nc = (size_t)s->nx * s->ny;
    memset(rho, 0, nc * sizeof(double));
    for (int k = 0; k < s->nsp; ++k) {
        const orc_species *p = &s->sp[k];
        for (long long q = 0; q < p->n; ++q) {
            double x = p->x[q], y = p->y[q];
            fadd(s, rho, p->ix[q], p->iy[q], p->qp * (1 - x) * (1 - y));
            fadd(s, rho, p->ix[q] + 1, p->iy[q], p->qp * x * (1 - y));
            fadd(s, rho, p->ix[q], p->iy[q] + 1, p->qp * (1 - x) * y);
            fadd(s, rho, p->ix[q] + 1, p->iy[q] + 1, p->qp * x * y);
        }
    }
}

/* discrete divergence at the nodes of a staggered (Ex-like, Ey-like) pair */
void orc_divergence(const orc_sim *s, const double *fx, const double *fy, double *div)
{
    for (int j = 0; j < s->ny; ++j)
        for (int i = 0; i < s->nx; ++i)
            div[i + (size_t)j * s->nx] = (fget(s, fx, i, j) - fget(s, fx, i - 1, j)) / s->dx +
                                         (fget(s, fy, i, j) - fget(s, fy, i, j - 1)) / s->dy;
}

/* out[0] = electric energy, out[1] = magnetic energy, out[2 + k] = kinetic
 * energy of species k (k < ORC_MAX_SPECIES), out[2 + ORC_MAX_SPECIES] = total
 * charge.  Kinetic energy at time n uses u^- = u^{n-1/2} + (q/m)(dt/2)E^n:
 * m_p |u^-|^2 / (gamma^- + 1), with m_p = q_p / (q/m). */
void orc_energy(const orc_sim *s, double *out)
{
    size_t nc = (size_t)s->nx * s->ny;
    double area = s->dx * s->dy;
    double we = 0, wb = 0;
    for (size_t q = 0; q < nc; ++q) {
        we += s->e[0][q] * s->e[0][q] + s->e[1][q] * s->e[1][q] + s->e[2][q] * s->e[2][q];
        wb += s->b[0][q] * s->b[0][q] + s->b[1][q] * s->b[1][q] + s->b[2][q] * s->b[2][q];
    }
    out[0] = 0.5 * we * area;
    out[1] = 0.5 * wb * area;
    double charge = 0;
    for (int k = 0; k < ORC_MAX_SPECIES; ++k) out[2 + k] = 0.0;
    for (int k = 0; k < s->nsp; ++k) {
        const orc_species *p = &s->sp[k];
        double tau = 0.5 * s->dt * p->qm, mp = p->qp / p->qm, ke = 0;
        for (long long q = 0; q < p->n; ++q) {
            double fl[6];
            orc_gather(s, p->ix[q], p->iy[q], p->x[q], p->y[q], fl);
            double a = p->ux[q] + tau * fl[0], b = p->uy[q] + tau * fl[1], c = p->uz[q] + tau * fl[2];
            double u2 = a * a + b * b + c * c;
            ke += mp * u2 / (sqrt(1.0 + u2) + 1.0);
        }
        out[2 + k] = ke * area;
        charge += p->qp * (double)p->n * area;
    }
    out[2 + ORC_MAX_SPECIES] = charge;
}
