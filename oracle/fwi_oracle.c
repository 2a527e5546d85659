/*
 * fwi_oracle.c -- plain FP64 CPU oracle for the acoustic FWI hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
 * Python binding) includes, links or calls this file; only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark do.  It shares no
 * source, header or table with the GPU path.
 *
 * What it computes (the paper, Section 3):
 *   - Eq. 2: constant-density acoustic wave equation P_tt = v^2 lap(P) + s.
 *   - Eq. 3: second-order leapfrog in time,
 *       P^{n+1} = -P^{n-1} + 2 P^n + v^2 dt^2 lap(P^n) + dt^2 s^n,
 *     here with a sponge (damping term 2*eta*P_t, centred in time), so that
 *       P^{n+1} = alpha*(2 P^n + kappa*lap(P^n) + dt^2 s^n) - beta*P^{n-1},
 *     alpha = 1/(1+eta dt), beta = (1-eta dt)/(1+eta dt), kappa = v^2 dt^2.
 *     eta == 0 gives alpha == beta == 1, i.e. exactly Eq. 3.
 *   - The spatial Laplacian is the central 2M-th order star stencil (Fig. 3,
 *     "order >= 8") with zero field values outside the grid:
 *       lap(p)_i = (1/dx^2) sum_axes [ c_0 p_i + sum_{m=1..M} c_m (p_{i+m} + p_{i-m}) ]
 *     The weights c_0..c_M are an input (computed exactly in Python).
 *   - Eq. 1: least-squares misfit; the adjoint (discrete, exact transpose of
 *     the recurrence above) and the velocity gradient are computed in the
 *     scaled variable psi = kappa*alpha*lambda, for which the adjoint
 *     recurrence is the forward recurrence itself.
 *
 * Arrays are C-contiguous [nz][ny][nx] float64 over the padded grid (model
 * plus sponge); a 2-D problem uses ny == 1 and no y-term.  No blocking, no
 * fusion: each time step is "Laplacian, then update, then source, then
 * record", in that order, written as plain loops.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int ndim;       /* 2 or 3 */
    long nz, ny, nx;
    int M;          /* stencil half width, order = 2M */
    const double *c;/* c[0..M] */
    double dx;
} orc_grid;

static long ncell(const orc_grid *g) { return g->nz * g->ny * g->nx; }

/* Field value with zero outside the grid (Dirichlet ghost cells). */
static double val(const orc_grid *g, const double *p, long z, long y, long x)
{
    if (z < 0 || z >= g->nz || y < 0 || y >= g->ny || x < 0 || x >= g->nx)
        return 0.0;
    return p[(z * g->ny + y) * g->nx + x];
}

/* out = lap(p), the definition above, cell by cell. */
void orc_laplacian(int ndim, long nz, long ny, long nx, int M, const double *c,
                   double dx, const double *p, double *out)
{
    orc_grid g = {ndim, nz, ny, nx, M, c, dx};
    const double inv_dx2 = 1.0 / (dx * dx);
#pragma omp parallel for schedule(static)
    for (long z = 0; z < nz; ++z) {
        for (long y = 0; y < ny; ++y) {
            for (long x = 0; x < nx; ++x) {
                double pc = p[(z * ny + y) * nx + x];
                double s = 0.0;
                /* every neighbour of an interior cell is inside the grid, so
                   val() reduces to a plain array read; same sum, same order */
                int interior = z >= M && z < nz - M && x >= M && x < nx - M &&
                               (ndim == 2 || (y >= M && y < ny - M));
                if (interior) {
                    const double *q = p + (z * ny + y) * nx + x;
                    const long sz = ny * nx, sy = nx;
                    s += c[0] * pc;
                    for (int m = 1; m <= M; ++m) s += c[m] * (q[m * sz] + q[-m * sz]);
                    if (ndim == 3) {
                        s += c[0] * pc;
                        for (int m = 1; m <= M; ++m) s += c[m] * (q[m * sy] + q[-m * sy]);
                    }
                    s += c[0] * pc;
                    for (int m = 1; m <= M; ++m) s += c[m] * (q[m] + q[-m]);
                    out[(z * ny + y) * nx + x] = s * inv_dx2;
                    continue;
                }
                /* z axis */
                s += c[0] * pc;
                for (int m = 1; m <= M; ++m)
                    s += c[m] * (val(&g, p, z + m, y, x) + val(&g, p, z - m, y, x));
                /* y axis (3-D only) */
                if (ndim == 3) {
                    s += c[0] * pc;
                    for (int m = 1; m <= M; ++m)
                        s += c[m] * (val(&g, p, z, y + m, x) + val(&g, p, z, y - m, x));
                }
                /* x axis */
                s += c[0] * pc;
                for (int m = 1; m <= M; ++m)
                    s += c[m] * (val(&g, p, z, y, x + m) + val(&g, p, z, y, x - m));
                out[(z * ny + y) * nx + x] = s * inv_dx2;
            }
        }
    }
}

/* One leapfrog update: out = alpha*(2 cur + kappa*lap) - beta*prev. */
static void leapfrog(long n, const double *alpha, const double *beta,
                     const double *kappa, const double *cur, const double *lap,
                     const double *prev, double *out)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; ++i)
        out[i] = alpha[i] * (2.0 * cur[i] + kappa[i] * lap[i]) - beta[i] * prev[i];
}

/*
 * Forward modelling of one shot.
 *   p^0 = p^{-1} = 0;  for n = 0..nt-1:
 *     p^{n+1} = alpha*(2p^n + kappa*lap p^n + dt^2 s^n) - beta*p^{n-1},
 *     s^n = w[n] / dx^ndim at cell src (a discrete point source),
 *     traces[n][r] = p^{n+1}[rec[r]].
 * states (optional, may be NULL): (nt+1) fields, states[n] = p^n.
 * Returns 0, or -1 if scratch allocation fails.
 */
int orc_forward(int ndim, long nz, long ny, long nx, int M, const double *c,
                double dx, double dt, const double *kappa, const double *alpha,
                const double *beta, long nt, long src, const double *w,
                long nrec, const long *rec, double *traces, double *states)
{
    orc_grid g = {ndim, nz, ny, nx, M, c, dx};
    const long n = ncell(&g);
    double *prev = calloc((size_t)n, sizeof(double));
    double *cur = calloc((size_t)n, sizeof(double));
    double *next = calloc((size_t)n, sizeof(double));
    double *lap = calloc((size_t)n, sizeof(double));
    if (!prev || !cur || !next || !lap) {
        free(prev); free(cur); free(next); free(lap);
        return -1;
    }
    double cell_vol = 1.0;
    for (int a = 0; a < ndim; ++a) cell_vol *= dx;
    if (states) memset(states, 0, (size_t)n * sizeof(double)); /* p^0 */

    for (long it = 0; it < nt; ++it) {
        orc_laplacian(ndim, nz, ny, nx, M, c, dx, cur, lap);
        leapfrog(n, alpha, beta, kappa, cur, lap, prev, next);
        next[src] += alpha[src] * dt * dt * w[it] / cell_vol;
        for (long r = 0; r < nrec; ++r)
            traces[it * nrec + r] = next[rec[r]];
        if (states) memcpy(states + (size_t)(it + 1) * n, next, (size_t)n * sizeof(double));
        double *t = prev; prev = cur; cur = next; next = t;
    }
    free(prev); free(cur); free(next); free(lap);
    return 0;
}

/*
 * Adjoint of orc_forward's map (kappa -> traces) for adjoint source res[n][r]
 * (res = d(misfit)/d(traces)), in the scaled variable psi = kappa*alpha*lambda:
 *   psi^{nt+1} = psi^{nt+2} = 0;  for k = nt..1:
 *     psi^k = alpha*(2 psi^{k+1} + kappa*lap psi^{k+1}) - beta*psi^{k+2},
 *     psi^k[rec[r]] += kappa*alpha*res[k-1][r]   (r in order),
 * and, when states (p^0..p^nt from orc_forward) and g are given,
 *     g += psi^{n+1} * lap(p^n)   for n = 1..nt-1,
 * so that d(misfit)/d(kappa) = g / kappa.
 * probe (optional): probe[k] = psi^k[probe_cell] for k = 1..nt (probe[0] unused).
 */
int orc_adjoint(int ndim, long nz, long ny, long nx, int M, const double *c,
                double dx, double dt, const double *kappa, const double *alpha,
                const double *beta, long nt, long nrec, const long *rec,
                const double *res, const double *states, double *g,
                long probe_cell, double *probe)
{
    (void)dt;
    orc_grid gr = {ndim, nz, ny, nx, M, c, dx};
    const long n = ncell(&gr);
    double *psi2 = calloc((size_t)n, sizeof(double)); /* psi^{k+2} */
    double *psi1 = calloc((size_t)n, sizeof(double)); /* psi^{k+1} */
    double *psi0 = calloc((size_t)n, sizeof(double)); /* psi^{k}   */
    double *lap = calloc((size_t)n, sizeof(double));
    double *lapp = calloc((size_t)n, sizeof(double));
    if (!psi2 || !psi1 || !psi0 || !lap || !lapp) {
        free(psi2); free(psi1); free(psi0); free(lap); free(lapp);
        return -1;
    }
    for (long k = nt; k >= 1; --k) {
        orc_laplacian(ndim, nz, ny, nx, M, c, dx, psi1, lap);
        leapfrog(n, alpha, beta, kappa, psi1, lap, psi2, psi0);
        for (long r = 0; r < nrec; ++r) {
            long i = rec[r];
            psi0[i] += kappa[i] * alpha[i] * res[(k - 1) * nrec + r];
        }
        if (probe) probe[k] = psi0[probe_cell];
        if (states && g && k - 1 >= 1) {
            /* term n = k-1 of sum_n psi^{n+1} * lap(p^n) */
            orc_laplacian(ndim, nz, ny, nx, M, c, dx, states + (size_t)(k - 1) * n, lapp);
            for (long i = 0; i < n; ++i) g[i] += psi0[i] * lapp[i];
        }
        double *t = psi2; psi2 = psi1; psi1 = psi0; psi0 = t;
    }
    free(psi2); free(psi1); free(psi0); free(lap); free(lapp);
    return 0;
}
