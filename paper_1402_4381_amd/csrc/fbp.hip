// Filtered back-projection for the 2D equiangular fan beam over one full
// turn: the initial image the paper's experiments start from (figure
// captions).  Textbook equiangular fan-beam reconstruction: the data are
// weighted by D cos(gamma), filtered along the channels with the fan-beam
// Ram-Lak kernel g(n dg) = 1/2 (n dg / sin(n dg))^2 h(n dg), which is
// 1/(8 dg^2) at n = 0, -1/(2 pi^2 sin^2(n dg)) at odd n and 0 at even n,
// and back-projected with the weight 1/L^2 (L: distance from the source)
// and linear interpolation in channel.
#include "lalm_internal.h"

namespace lalm {
namespace {

constexpr int FBP_NBMAX = 4096;   // channels per view held in LDS

// Q[slot][b] = dg sum_k q[k] g(b - k), q[k] = y[slot][k] D cos(gamma_k);
// one block per view, the weighted row and the kernel table in LDS, each
// output summed over k in increasing order.
__global__ void __launch_bounds__(256) fbp_filter_kernel(const float *y, float *Q, int nb, double dg, double D,
                                                         double center)
{
    __shared__ float q[FBP_NBMAX];
    __shared__ float gk[FBP_NBMAX];
    const long long base = (long long)blockIdx.x * nb;
    const double pi = 3.14159265358979323846;
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        q[k] = (float)((double)y[base + k] * D * cos(((double)k - center) * dg));
        double g = 0.0;
        if (k == 0) {
            g = 1.0 / (8.0 * dg * dg);
        } else if (k & 1) {
            const double sn = sin((double)k * dg);
            g = -1.0 / (2.0 * pi * pi * sn * sn);
        }
        gk[k] = (float)g;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        float acc = 0.0f;
        for (int k = 0; k < nb; ++k) {
            const int d = b > k ? b - k : k - b;
            acc = fmaf(q[k], gk[d], acc);
        }
        Q[base + b] = (float)dg * acc;
    }
}

// x[j][i] = dbeta sum_views Q(gamma'(P)) / L(P)^2
__global__ void __launch_bounds__(256) fbp_backproject_kernel(GeoK K, const ViewRec *views, int nview,
                                                              const float *Q, float dbeta, float *x)
{
    const int i = blockIdx.x * 32 + threadIdx.x, j = blockIdx.y * 8 + threadIdx.y;
    if (i >= K.nx || j >= K.ny) return;
    const float X = fmaf((float)i, K.dx, K.x0), Y = fmaf((float)j, K.dy, K.y0);
    float acc = 0.0f;
    for (int v = 0; v < nview; ++v) {
        const ViewRec V = views[v];
        const float ddx = X - V.sx, ddy = Y - V.sy;
        const float dc = -(ddx * V.cb + ddy * V.sb);
        const float dp = ddx * V.sb - ddy * V.cb;
        const float bc = fmaf(atan2f(dp, dc), K.dsd_over_ds, K.bin_center);
        const float fl = floorf(bc);
        const int b0 = (int)fl;
        const float t = bc - fl;
        const float *row = Q + (long long)v * K.nb;
        float val = 0.0f;
        if (b0 >= 0 && b0 < K.nb) val = (1.0f - t) * row[b0];
        if (b0 + 1 >= 0 && b0 + 1 < K.nb) val = fmaf(t, row[b0 + 1], val);
        acc += val / fmaf(ddx, ddx, ddy * ddy);
    }
    x[(long long)j * K.nx + i] = dbeta * acc;
}

}  // namespace

hipError_t launch_fbp(const lalm_plan *p, const float *y, float *x, hipStream_t st)
{
    const lalm_geometry &g = p->g;
    const double dg = g.ds / g.dsd;
    const double center = (p->nb - 1) / 2.0 + g.channel_offset;
    hipLaunchKernelGGL(fbp_filter_kernel, dim3(p->nv), dim3(256), 0, st, y, p->d_fbpq, p->nb, dg, g.dso, center);
    const float dbeta = (float)(2.0 * 3.14159265358979323846 / g.n_views_per_turn);
    dim3 blk(32, 8), grd((p->nx + 31) / 32, (p->ny + 7) / 8);
    hipLaunchKernelGGL(fbp_backproject_kernel, grd, blk, 0, st, p->k, (const ViewRec *)p->d_views, p->nv,
                       (const float *)p->d_fbpq, dbeta, x);
    return hipGetLastError();
}

int fbp_max_bins() { return FBP_NBMAX; }

}  // namespace lalm
