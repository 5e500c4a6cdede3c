/*
 * FP64 CPU oracle for the OS-LALM CT hot path -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * use this file.  It shares no code with the GPU library.
 *
 * What it computes: the system matrix A of the PWLS problem (Sec. IV,
 * eq. "ct_recon").  The paper names no projector; the reading used here is a
 * ray-driven Joseph interpolator with one ray per detector-cell centre:
 *
 *   For a ray with source S and unit direction u, the in-plane dominant axis
 *   is x when |u_x| >= |u_y| (ties go to x), else y.  For x-dominance, every
 *   image column i (centre X_i) is sampled at t_i = (X_i - S_x) / u_x; the
 *   sample has fractional row index eta = (S_y + t_i u_y - Y_0) / dy and (3D)
 *   fractional slice index zeta = (S_z + t_i u_z - Z_0) / dz.  With
 *   j0 = floor(eta), f = eta - j0 (and k0, h for zeta) the sample puts weight
 *   L (1-f)(1-h), L f (1-h), L (1-f) h, L f h on voxels (i,j0,k0), (i,j0+1,k0),
 *   (i,j0,k0+1), (i,j0+1,k0+1), where L = dx / |u_x| is the ray length per
 *   column.  Taps outside the volume are dropped (zero padding).  In 2D only
 *   the eta interpolation exists.  y-dominance swaps the roles of x and y.
 *
 * The forward projection marches each ray (plain loops, FP64); the
 * back-projection scatters the same weights (the exact transpose).  The dense
 * builder evaluates every matrix entry on its own, as the hat function
 * max(0, 1 - |eta - j|) max(0, 1 - |zeta - k|) L of the sampled position, for
 * brute-force checks on tiny geometries.
 *
 * Geometry (scanner model, a reading): voxel centres X_i = (i - (nx-1)/2) dx;
 * view angle beta = start + 2 pi v / views_per_turn; source
 * (dso cos beta, dso sin beta, z_s); equiangular channels
 * gamma_b = (b - (nb-1)/2 - offset) ds / dsd, in-plane direction at angle
 * beta + pi + gamma_b; cylindrical rows at height v_r = (r - (nr-1)/2) dt at
 * distance dsd; helical z_s = (v - (n_views-1)/2) feed / views_per_turn with
 * feed = pitch n_rows dt dso / dsd.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int kind; /* 0 fan 2D, 1 cone axial, 2 cone helical */
    int nx, ny, nz;
    double dx, dy, dz;
    int n_views, n_views_per_turn, n_bins, n_rows;
    double ds, dt, dso, dsd, start_angle, pitch, channel_offset;
    int detector; /* 0 = arc (equiangular, cylindrical); the only one here */
} og_geom;

/* Source point and unit direction of ray (view v, row r, bin b). */
void og_ray(const og_geom *g, int v, int r, int b, double *S, double *u)
{
    const double PI = 3.14159265358979323846;
    double beta = g->start_angle + 2.0 * PI * (double)v / (double)g->n_views_per_turn;
    double zs = 0.0;
    if (g->kind == 2) {
        double feed = g->pitch * g->n_rows * g->dt * g->dso / g->dsd;
        zs = ((double)v - (g->n_views - 1) / 2.0) * feed / (double)g->n_views_per_turn;
    }
    double gam = ((double)b - (g->n_bins - 1) / 2.0 - g->channel_offset) * g->ds / g->dsd;
    double vr = (g->kind == 0) ? 0.0 : ((double)r - (g->n_rows - 1) / 2.0) * g->dt;
    double th = beta + PI + gam;
    double ex = cos(th), ey = sin(th);
    double n = sqrt(g->dsd * g->dsd + vr * vr);
    S[0] = g->dso * cos(beta);
    S[1] = g->dso * sin(beta);
    S[2] = zs;
    u[0] = g->dsd * ex / n;
    u[1] = g->dsd * ey / n;
    u[2] = vr / n;
}

static double vox_centre0(int n, double d) { return -(n - 1) / 2.0 * d; }

/* Voxel value with zero padding outside the volume; x is [z][y][x]. */
static double vox(const og_geom *g, const double *x, int i, int j, int k)
{
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || k < 0 || k >= g->nz) return 0.0;
    return x[((size_t)k * g->ny + j) * g->nx + i];
}

static void vox_add(const og_geom *g, double *x, int i, int j, int k, double val)
{
    if (i < 0 || i >= g->nx || j < 0 || j >= g->ny || k < 0 || k >= g->nz) return;
    x[((size_t)k * g->ny + j) * g->nx + i] += val;
}

/*
 * One Joseph sample of a ray at slice s of its dominant axis.
 * Returns the 4 taps (voxel indices) and weights; in 2D the k taps are 0 and
 * the weights for k0+1 are zero.
 */
typedef struct { int i[4], j[4], k[4]; double w[4]; } og_sample;

static void og_sample_at(const og_geom *g, const double *S, const double *u,
                         int xdom, int s, og_sample *out)
{
    double X0 = vox_centre0(g->nx, g->dx), Y0 = vox_centre0(g->ny, g->dy);
    double Z0 = vox_centre0(g->nz, g->dz);
    double t, L, other, zeta = 0.0;
    if (xdom) {
        double Xs = X0 + s * g->dx;
        t = (Xs - S[0]) / u[0];
        L = g->dx / fabs(u[0]);
        other = (S[1] + t * u[1] - Y0) / g->dy;
    } else {
        double Ys = Y0 + s * g->dy;
        t = (Ys - S[1]) / u[1];
        L = g->dy / fabs(u[1]);
        other = (S[0] + t * u[0] - X0) / g->dx;
    }
    double o0 = floor(other), f = other - o0;
    int io = (int)o0;
    double h = 0.0;
    int k0 = 0;
    if (g->kind != 0) {
        zeta = (S[2] + t * u[2] - Z0) / g->dz;
        double z0 = floor(zeta);
        h = zeta - z0;
        k0 = (int)z0;
    }
    double wo[2] = {1.0 - f, f};
    double wz[2] = {1.0 - h, h};
    for (int a = 0; a < 2; ++a)
        for (int c = 0; c < 2; ++c) {
            int q = a + 2 * c;
            if (xdom) { out->i[q] = s; out->j[q] = io + a; }
            else      { out->j[q] = s; out->i[q] = io + a; }
            out->k[q] = k0 + c;
            out->w[q] = L * wo[a] * ((g->kind != 0) ? wz[c] : (c == 0 ? 1.0 : 0.0));
        }
}

static int og_xdom(const double *u) { return fabs(u[0]) >= fabs(u[1]); }

/* Joseph line integral of one ray through image x ([z][y][x]). */
double og_ray_integral(const og_geom *g, const double *x, int v, int r, int b)
{
    double S[3], u[3];
    og_ray(g, v, r, b, S, u);
    int xdom = og_xdom(u);
    int ns = xdom ? g->nx : g->ny;
    double acc = 0.0;
    for (int s = 0; s < ns; ++s) {
        og_sample sm;
        og_sample_at(g, S, u, xdom, s, &sm);
        for (int q = 0; q < 4; ++q)
            if (sm.w[q] != 0.0) acc += sm.w[q] * vox(g, x, sm.i[q], sm.j[q], sm.k[q]);
    }
    return acc;
}

/* out[kv][r][b] = (A x) for the listed views, in listed order. */
void og_forward(const og_geom *g, const double *x, const int *views, int nv, double *out)
{
    long long nray = (long long)nv * g->n_rows * g->n_bins;
#pragma omp parallel for schedule(dynamic, 64)
    for (long long q = 0; q < nray; ++q) {
        int b = (int)(q % g->n_bins);
        int r = (int)((q / g->n_bins) % g->n_rows);
        int kv = (int)(q / ((long long)g->n_bins * g->n_rows));
        out[q] = og_ray_integral(g, x, views[kv], r, b);
    }
}

/* Scatter one ray's value along its Joseph weights into img. */
static void og_scatter_ray(const og_geom *g, double *img, int v, int r, int b, double val)
{
    if (val == 0.0) return;
    double S[3], u[3];
    og_ray(g, v, r, b, S, u);
    int xdom = og_xdom(u);
    int ns = xdom ? g->nx : g->ny;
    for (int s = 0; s < ns; ++s) {
        og_sample sm;
        og_sample_at(g, S, u, xdom, s, &sm);
        for (int q = 0; q < 4; ++q)
            if (sm.w[q] != 0.0) vox_add(g, img, sm.i[q], sm.j[q], sm.k[q], sm.w[q] * val);
    }
}

/*
 * img = A' sino over the listed views (sino is [kv][r][b]).  Views are split
 * into a fixed number of contiguous chunks, each scattered into its own
 * buffer and summed in chunk order, so the result does not depend on the
 * number of threads.
 */
void og_back(const og_geom *g, const double *sino, const int *views, int nv, double *img)
{
    size_t nvox = (size_t)g->nx * g->ny * g->nz;
    int nchunk = nv < 16 ? nv : 16;
    if (nchunk <= 0) { memset(img, 0, nvox * sizeof(double)); return; }
    double *part = (double *)calloc((size_t)nchunk * nvox, sizeof(double));
    size_t per_view = (size_t)g->n_rows * g->n_bins;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < nchunk; ++c) {
        int lo = (int)((long long)nv * c / nchunk), hi = (int)((long long)nv * (c + 1) / nchunk);
        double *dst = part + (size_t)c * nvox;
        for (int kv = lo; kv < hi; ++kv)
            for (int r = 0; r < g->n_rows; ++r)
                for (int b = 0; b < g->n_bins; ++b)
                    og_scatter_ray(g, dst, views[kv], r, b,
                                   sino[(size_t)kv * per_view + (size_t)r * g->n_bins + b]);
    }
    for (size_t p = 0; p < nvox; ++p) {
        double s = 0.0;
        for (int c = 0; c < nchunk; ++c) s += part[(size_t)c * nvox + p];
        img[p] = s;
    }
    free(part);
}

/* Per-entry system matrix weight a(ray, voxel), evaluated on its own. */
double og_weight(const og_geom *g, int v, int r, int b, int i, int j, int k)
{
    double S[3], u[3];
    og_ray(g, v, r, b, S, u);
    double X0 = vox_centre0(g->nx, g->dx), Y0 = vox_centre0(g->ny, g->dy);
    double Z0 = vox_centre0(g->nz, g->dz);
    double t, L, d_other;
    if (og_xdom(u)) {
        t = (X0 + i * g->dx - S[0]) / u[0];
        L = g->dx / fabs(u[0]);
        d_other = (S[1] + t * u[1] - Y0) / g->dy - j;
    } else {
        t = (Y0 + j * g->dy - S[1]) / u[1];
        L = g->dy / fabs(u[1]);
        d_other = (S[0] + t * u[0] - X0) / g->dx - i;
    }
    double w = 1.0 - fabs(d_other);
    if (w <= 0.0) return 0.0;
    if (g->kind != 0) {
        double dz = (S[2] + t * u[2] - Z0) / g->dz - k;
        double wz = 1.0 - fabs(dz);
        if (wz <= 0.0) return 0.0;
        w *= wz;
    } else if (k != 0) {
        return 0.0;
    }
    return w * L;
}

/* Selected entries of A' sino: out[n] = sum over the rays of the listed
 * views of a(ray, voxel n) * sino(ray), each entry summed on its own in ray
 * order (voxel n = (k, j, i) = vox[3n .. 3n+2]). */
void og_back_at(const og_geom *g, const double *sino, const int *views, int nv, const int *vox, int nvox,
                double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int n = 0; n < nvox; ++n) {
        const int k = vox[3 * n], j = vox[3 * n + 1], i = vox[3 * n + 2];
        double acc = 0.0;
        for (int kv = 0; kv < nv; ++kv)
            for (int r = 0; r < g->n_rows; ++r)
                for (int b = 0; b < g->n_bins; ++b) {
                    const double s = sino[((long long)kv * g->n_rows + r) * g->n_bins + b];
                    if (s != 0.0) acc += og_weight(g, views[kv], r, b, i, j, k) * s;
                }
        out[n] = acc;
    }
}

/* Dense A for tiny geometries: A[(kv, r, b)][(k, j, i)]. */
void og_dense(const og_geom *g, const int *views, int nv, double *A)
{
    long long nray = (long long)nv * g->n_rows * g->n_bins;
    long long nvox = (long long)g->nx * g->ny * g->nz;
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < nray; ++q) {
        int b = (int)(q % g->n_bins);
        int r = (int)((q / g->n_bins) % g->n_rows);
        int kv = (int)(q / ((long long)g->n_bins * g->n_rows));
        for (long long p = 0; p < nvox; ++p) {
            int i = (int)(p % g->nx), j = (int)((p / g->nx) % g->ny), k = (int)(p / ((long long)g->nx * g->ny));
            A[q * nvox + p] = og_weight(g, views[kv], r, b, i, j, k);
        }
    }
}

/*
 * Number of Joseph samples of the listed views: (ray, slice) pairs whose
 * lower tap index along each interpolated axis lies in [-1, n-1], i.e. at
 * least one tap of the sample falls inside the volume.
 */
long long og_count_samples(const og_geom *g, const int *views, int nv)
{
    long long nray = (long long)nv * g->n_rows * g->n_bins;
    long long total = 0;
#pragma omp parallel for reduction(+ : total) schedule(dynamic, 256)
    for (long long q = 0; q < nray; ++q) {
        int b = (int)(q % g->n_bins);
        int r = (int)((q / g->n_bins) % g->n_rows);
        int kv = (int)(q / ((long long)g->n_bins * g->n_rows));
        double S[3], u[3];
        og_ray(g, views[kv], r, b, S, u);
        int xdom = og_xdom(u);
        int ns = xdom ? g->nx : g->ny, no = xdom ? g->ny : g->nx;
        for (int s = 0; s < ns; ++s) {
            og_sample sm;
            og_sample_at(g, S, u, xdom, s, &sm);
            int lo = xdom ? sm.j[0] : sm.i[0];
            if (lo < -1 || lo > no - 1) continue;
            if (g->kind != 0 && (sm.k[0] < -1 || sm.k[0] > g->nz - 1)) continue;
            ++total;
        }
    }
    return total;
}
