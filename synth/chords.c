/*
 * Analytic line integrals of ellipse/ellipsoid phantoms for the synthetic
 * input generator (same recipe as synth/phantom.py, compiled for speed on
 * large cone-beam workloads).  For every ray (view, row, bin) of the scanner
 * model the sum over objects of amplitude x chord length is written to out.
 * This is data synthesis, not part of the reconstruction method.
 */
#include <math.h>
#include <omp.h>

/* geometry: kind nx ny nz dx dy dz n_views n_views_per_turn n_bins n_rows ds
 *           dt dso dsd start_angle pitch channel_offset (doubles)  */
void synth_chords(const double *geo, int n_obj, const double *cx, const double *cy,
                  const double *cz, const double *ax, const double *ay, const double *az,
                  const double *phi, const double *amp, int is2d, const int *views, int nv,
                  double *out, int n_threads)
{
    /* n_threads <= 0: the OpenMP default */
    const int nt = n_threads > 0 ? n_threads : omp_get_max_threads();
    const double PI = 3.14159265358979323846;
    int kind = (int)geo[0];
    int n_views = (int)geo[7], vpt = (int)geo[8], nb = (int)geo[9], nr = (int)geo[10];
    double ds = geo[11], dt = geo[12], dso = geo[13], dsd = geo[14];
    double start = geo[15], pitch = geo[16], off = geo[17];
    double feed = (kind == 2) ? pitch * nr * dt * dso / dsd : 0.0;
    long long nray = (long long)nv * nr * nb;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (long long q = 0; q < nray; ++q) {
        int b = (int)(q % nb);
        int r = (int)((q / nb) % nr);
        int kv = (int)(q / ((long long)nb * nr));
        int v = views[kv];
        double beta = start + 2.0 * PI * v / vpt;
        double zs = (kind == 2) ? (v - (n_views - 1) / 2.0) * feed / vpt : 0.0;
        double gam = (b - (nb - 1) / 2.0 - off) * ds / dsd;
        double vr = (kind == 0) ? 0.0 : (r - (nr - 1) / 2.0) * dt;
        double th = beta + PI + gam;
        double n = sqrt(dsd * dsd + vr * vr);
        double ux = dsd * cos(th) / n, uy = dsd * sin(th) / n, uz = vr / n;
        double sx = dso * cos(beta), sy = dso * sin(beta), sz = zs;
        double acc = 0.0;
        for (int e = 0; e < n_obj; ++e) {
            double c = cos(phi[e]), s = sin(phi[e]);
            double px = sx - cx[e], py = sy - cy[e];
            double P0 = (c * px + s * py) / ax[e], P1 = (-s * px + c * py) / ay[e];
            double D0 = (c * ux + s * uy) / ax[e], D1 = (-s * ux + c * uy) / ay[e];
            double A = D0 * D0 + D1 * D1, B = P0 * D0 + P1 * D1, C = P0 * P0 + P1 * P1 - 1.0;
            if (!is2d) {
                double P2 = (sz - cz[e]) / az[e], D2 = uz / az[e];
                A += D2 * D2;
                B += P2 * D2;
                C += P2 * P2;
            }
            double disc = B * B - A * C;
            if (disc > 0.0) acc += amp[e] * 2.0 * sqrt(disc) / A;
        }
        out[q] = acc;
    }
}
