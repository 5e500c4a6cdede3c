// Geometry planning, plan lifetime and error reporting.
//
// The per-view and per-ray Joseph tables are derived in FP64 on the host from
// the scanner model stated in lalm.h and stored as FP32.  Every GPU kernel
// that needs the fractional position of a sample evaluates it from the same
// FP32 table entries with the same fused multiply-adds, so the forward and
// back-projectors see bit-identical interpolation positions (matched pair).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>

#include "lalm_internal.h"

namespace {
thread_local std::string g_err;

// Integers s in [0, ns) with lo <= alpha + beta*s < hi.
void linear_range(double alpha, double beta, double lo, double hi, int ns, long long *s0,
                  long long *s1)
{
    double a, b;  // real interval of s
    if (beta == 0.0) {
        if (alpha >= lo && alpha < hi) { *s0 = 0; *s1 = ns - 1; }
        else { *s0 = 1; *s1 = 0; }
        return;
    }
    long long first, last;
    if (beta > 0.0) {
        a = (lo - alpha) / beta;  // s >= a
        b = (hi - alpha) / beta;  // s <  b
        first = (long long)std::ceil(a);
        last = (long long)std::ceil(b) - 1;
    } else {
        a = (hi - alpha) / beta;  // s >  a
        b = (lo - alpha) / beta;  // s <= b
        first = (long long)std::floor(a) + 1;
        last = (long long)std::floor(b);
    }
    *s0 = std::max<long long>(first, 0);
    *s1 = std::min<long long>(last, ns - 1);
}

std::vector<int32_t> bit_reversal(int M)
{
    int B = 0;
    while ((1 << B) < M) ++B;
    std::vector<int32_t> out;
    for (int j = 0; j < (1 << B); ++j) {
        int r = 0;
        for (int t = 0; t < B; ++t)
            if (j & (1 << t)) r |= 1 << (B - 1 - t);
        if (r < M) out.push_back(r);
    }
    return out;
}

template <class T>
hipError_t dev_alloc(T **p, size_t n)
{
    return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

}  // namespace

void lalm::set_error(const std::string &msg) { g_err = msg; }

bool lalm::prof_pair(const lalm_plan *p, hipEvent_t *start, hipEvent_t *stop)
{
    if (!p->prof || p->prof_cls < 0) return false;
    if (p->prof_used + 2 > p->prof_ev.size()) {
        const size_t n = p->prof_ev.size();
        p->prof_ev.resize(std::max<size_t>(64, 2 * n));
        for (size_t i = n; i < p->prof_ev.size(); ++i)
            if (hipEventCreate(&p->prof_ev[i]) != hipSuccess) p->prof_ev[i] = nullptr;
    }
    *start = p->prof_ev[p->prof_used];
    *stop = p->prof_ev[p->prof_used + 1];
    if (!*start || !*stop) return false;
    p->prof_used += 2;
    p->prof_kind.push_back(p->prof_cls);
    return true;
}

extern "C" const char *lalm_last_error(void) { return g_err.c_str(); }

extern "C" const char *lalm_version(void) { return "lalm-gfx950 0.1"; }

static lalm_status invalid(const char *msg)
{
    lalm::set_error(msg);
    return LALM_E_INVALID;
}

static void free_plan(lalm_plan *p)
{
    if (!p) return;
    (void)hipFree(p->d_rays);
    (void)hipFree(p->d_raysz);
    (void)hipFree(p->d_views);
    (void)hipFree(p->d_rowv);
    (void)hipFree(p->d_rowf);
    (void)hipFree(p->d_xt);
    (void)hipFree(p->d_xn);
    (void)hipFree(p->d_gradR);
    (void)hipFree(p->d_v);
    (void)hipFree(p->d_fbpq);
    (void)hipFree(p->d_xt1);
    (void)hipFree(p->d_xn1);
    (void)hipFree(p->d_xc);
    (void)hipFree(p->d_r);
    (void)hipFree(p->d_part);
    (void)hipFree(p->d_part2);
    (void)hipFree(p->d_partials);
    (void)hipFree(p->d_sc);
    (void)hipFree(p->d_tmp);
    if (p->h_sc) (void)hipHostFree(p->h_sc);
    for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
    delete p;
}

extern "C" lalm_status lalm_plan_geometry(const lalm_geometry *geom, int32_t n_subsets, int32_t batch,
                                          lalm_plan **out)
{
    if (!geom || !out) return invalid("lalm_plan_geometry: null argument");
    *out = nullptr;
    const lalm_geometry &g = *geom;
    if (g.kind < 0 || g.kind > 2) return invalid("geometry: unknown kind");
    if (g.nx < 1 || g.ny < 1 || g.nz < 1 || g.nx > 32767 || g.ny > 32767 || g.nz > 32767)
        return invalid("geometry: image sizes must lie in [1, 32767]");
    if (g.kind == LALM_FAN2D && (g.nz != 1 || g.n_rows != 1))
        return invalid("geometry: fan-beam 2D needs nz = 1 and n_rows = 1");
    if (!(g.dx > 0 && g.dy > 0 && g.dz > 0 && g.ds > 0 && g.dt > 0))
        return invalid("geometry: voxel and detector sizes must be positive");
    if (g.n_views < 1 || g.n_views_per_turn < 1 || g.n_bins < 1 || g.n_rows < 1)
        return invalid("geometry: view, bin and row counts must be positive");
    if (!(g.dso > 0 && g.dsd > g.dso)) return invalid("geometry: need 0 < dso < dsd");
    double half_diag = 0.5 * std::sqrt((double)g.nx * g.dx * g.nx * g.dx + (double)g.ny * g.dy * g.ny * g.dy);
    if (!(g.dso > half_diag + 2.0 * std::max(g.dx, g.dy)))
        return invalid("geometry: source inside (or within two pixels of) the image's circumscribed cylinder");
    if (g.detector != 0) return invalid("geometry: only the arc detector (0) is implemented");
    if (g.kind == LALM_CONE_HELICAL && !(g.pitch >= 0)) return invalid("geometry: negative pitch");
    if (n_subsets < 1 || n_subsets > g.n_views) return invalid("n_subsets must lie in [1, n_views]");
    // kernels index the images of a batch along a grid dimension with the slices
    if (batch < 1 || (int64_t)batch * g.nz > 65535) return invalid("batch must lie in [1, 65535 / nz]");
    if (g.n_rows > 256) return invalid("geometry: at most 256 detector rows");
    // the cone back-projector forms row offsets row * n_bins with 24-bit
    // multiplies and gathers a subset's residual by 32-bit byte offsets
    if (g.n_bins > (1 << 20)) return invalid("geometry: at most 2^20 detector channels");
    if (g.kind != LALM_FAN2D &&
        4.0 * ((g.n_views + n_subsets - 1) / n_subsets) * g.n_rows * g.n_bins >= 4294967296.0)
        return invalid("geometry: a subset's sinogram must stay below 4 GiB");
    double half_fan = 0.5 * g.n_bins * g.ds / g.dsd;
    if (!(half_fan < 0.75)) return invalid("geometry: fan angle too wide (half fan must stay below 0.75 rad)");

    lalm_plan *p = new lalm_plan();
    p->g = g;
    p->M = n_subsets;
    p->B = batch;
    p->nx = g.nx; p->ny = g.ny; p->nz = g.nz; p->nb = g.n_bins; p->nr = g.n_rows; p->nv = g.n_views;
    p->is3d = g.kind != LALM_FAN2D;
    (void)hipGetDevice(&p->device);
    const int M = n_subsets, nv = g.n_views, nb = g.n_bins, nr = g.n_rows;
    const bool is3d = p->is3d;

    // subsets: views v with v mod M == m, increasing; visited in bit-reversal order
    p->order = bit_reversal(M);
    p->slot_offset.assign(M + 1, 0);
    p->view_of_slot.clear();
    for (int m = 0; m < M; ++m) {
        p->slot_offset[m] = (int64_t)p->view_of_slot.size();
        for (int v = m; v < nv; v += M) p->view_of_slot.push_back(v);
    }
    p->slot_offset[M] = nv;
    p->rays_per_view = (int64_t)nr * nb;
    int64_t max_views = 0;
    for (int m = 0; m < M; ++m) max_views = std::max(max_views, p->slot_offset[m + 1] - p->slot_offset[m]);
    p->max_subset_rays = max_views * p->rays_per_view;

    // FP64 geometry
    const double PI = 3.14159265358979323846;
    const double X0 = -(g.nx - 1) / 2.0 * g.dx, Y0 = -(g.ny - 1) / 2.0 * g.dy;
    const double Z0 = -(g.nz - 1) / 2.0 * g.dz;
    const double feed = (g.kind == LALM_CONE_HELICAL) ? g.pitch * g.n_rows * g.dt * g.dso / g.dsd : 0.0;
    std::vector<double> vr(nr);
    std::vector<float> rowv(nr), rowf(nr);
    for (int r = 0; r < nr; ++r) {
        vr[r] = is3d ? (r - (nr - 1) / 2.0) * g.dt : 0.0;
        rowv[r] = (float)vr[r];
        rowf[r] = (float)std::sqrt(1.0 + (vr[r] / g.dsd) * (vr[r] / g.dsd));
    }
    std::vector<lalm::RayRec> rays((size_t)nv * nb);
    std::vector<lalm::RayRecZ> raysz(is3d ? (size_t)nv * nb : 0);
    std::vector<lalm::ViewRec> views(nv);
    std::vector<long long> slot_samples(nv, 0);
    std::vector<char> slot_split(nv, 0);   // dominance classes not contiguous

    auto work = [&](int slot_lo, int slot_hi) {
        for (int slot = slot_lo; slot < slot_hi; ++slot) {
            int v = p->view_of_slot[slot];
            double beta = g.start_angle + 2.0 * PI * v / g.n_views_per_turn;
            double Sx = g.dso * std::cos(beta), Sy = g.dso * std::sin(beta);
            double Sz = (g.kind == LALM_CONE_HELICAL) ? (v - (g.n_views - 1) / 2.0) * feed / g.n_views_per_turn : 0.0;
            double z0 = (Sz - Z0) / g.dz;
            lalm::ViewRec vw{};
            vw.sx = (float)Sx; vw.sy = (float)Sy;
            vw.cb = (float)std::cos(beta); vw.sb = (float)std::sin(beta);
            vw.z0 = (float)z0;
            vw.bx0 = vw.by0 = nb;
            vw.bx1 = vw.by1 = 0;
            long long nsamp = 0;
            int nxdom = 0;
            for (int b = 0; b < nb; ++b) {
                double gam = (b - (nb - 1) / 2.0 - g.channel_offset) * g.ds / g.dsd;
                double th = beta + PI + gam;
                double ex = std::cos(th), ey = std::sin(th);
                bool xdom = std::fabs(ex) >= std::fabs(ey);
                double a, c, sc, m = 0, k = 0;
                int ns, no;
                if (xdom) {
                    a = (Sy + (X0 - Sx) * ey / ex - Y0) / g.dy;
                    c = g.dx * ey / (ex * g.dy);
                    sc = g.dx / std::fabs(ex);
                    m = (X0 - Sx) / (ex * g.dsd * g.dz);
                    k = g.dx / (ex * g.dsd * g.dz);
                    ns = g.nx; no = g.ny;
                } else {
                    a = (Sx + (Y0 - Sy) * ex / ey - X0) / g.dx;
                    c = g.dy * ex / (ey * g.dx);
                    sc = g.dy / std::fabs(ey);
                    m = (Y0 - Sy) / (ey * g.dsd * g.dz);
                    k = g.dy / (ey * g.dsd * g.dz);
                    ns = g.ny; no = g.nx;
                }
                long long s0, s1;
                linear_range(a, c, -1.0, (double)no, ns, &s0, &s1);
                // conservative range for the kernels (one extra slice each side)
                long long k0 = std::max<long long>(s0 - 1, 0), k1 = std::min<long long>(s1 + 1, ns - 1);
                if (s0 > s1) { k0 = 1; k1 = 0; }
                lalm::RayRec rr;
                rr.a = (float)a; rr.c = (float)c; rr.sc = (float)sc;
                rr.meta = (uint32_t)(k0 & 0xFFFF) | ((uint32_t)(k1 & 0x7FFF) << 16) | (xdom ? 0u : lalm::kYDom);
                rays[(size_t)slot * nb + b] = rr;
                if (xdom) { vw.bx0 = std::min(vw.bx0, b); vw.bx1 = std::max(vw.bx1, b + 1); ++nxdom; }
                else { vw.by0 = std::min(vw.by0, b); vw.by1 = std::max(vw.by1, b + 1); }
                if (is3d) {
                    raysz[(size_t)slot * nb + b] = lalm::RayRecZ{(float)m, (float)k};
                    for (int r = 0; r < nr; ++r) {
                        if (s0 > s1) break;
                        long long t0, t1;
                        // zeta(s) = z0 + v_r (m + s k) in [-1, nz)
                        linear_range(z0 + vr[r] * m, vr[r] * k, -1.0, (double)g.nz, ns, &t0, &t1);
                        long long lo = std::max(s0, t0), hi = std::min(s1, t1);
                        if (hi >= lo) nsamp += hi - lo + 1;
                    }
                } else if (s1 >= s0) {
                    nsamp += s1 - s0 + 1;
                }
            }
            if (vw.bx0 > vw.bx1) { vw.bx0 = 0; vw.bx1 = 0; }
            if (vw.bx1 - vw.bx0 != nxdom || (nxdom > 0 && nxdom < nb && vw.bx0 != 0 && vw.bx1 != nb))
                slot_split[slot] = 1;
            if (vw.by0 > vw.by1) { vw.by0 = 0; vw.by1 = 0; }
            views[slot] = vw;
            slot_samples[slot] = nsamp;
        }
    };
    unsigned nthr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (nv < 64) nthr = 1;
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nthr; ++t)
        pool.emplace_back(work, (int)((long long)nv * t / nthr), (int)((long long)nv * (t + 1) / nthr));
    for (auto &th : pool) th.join();

    for (int slot = 0; slot < nv; ++slot)
        if (slot_split[slot]) {
            free_plan(p);
            return invalid("geometry: a view's rays switch dominant axis more than once");
        }
    p->subset_samples.assign(M, 0);
    for (int m = 0; m < M; ++m)
        for (int64_t s = p->slot_offset[m]; s < p->slot_offset[m + 1]; ++s) p->subset_samples[m] += slot_samples[s];

    lalm::GeoK &K = p->k;
    K.nx = g.nx; K.ny = g.ny; K.nz = g.nz; K.nb = nb; K.nr = nr; K.is3d = is3d;
    K.dx = (float)g.dx; K.dy = (float)g.dy; K.dz = (float)g.dz;
    K.x0 = (float)X0; K.y0 = (float)Y0;
    K.dsd_over_ds = (float)(g.dsd / g.ds);
    K.bin_center = (float)((nb - 1) / 2.0 + g.channel_offset);
    K.dmax = (float)std::max(g.dx, g.dy);
    K.inv_dt = (float)(1.0 / g.dt);
    K.row_center = (float)((nr - 1) / 2.0);
    K.bin_margin = (float)(0.05 + (g.dsd / g.ds) * 4e-6);
    K.zreach = (float)(((nr - 1) / 2.0 * g.dt) / (g.dsd * g.dz) * 1.0001);
    K.dso = (float)g.dso;
    // helical: the views of a subset are in increasing order, so their
    // source heights never decrease; checked on the stored values
    K.z_sorted = 0;
    if (g.kind == LALM_CONE_HELICAL) {
        bool sorted = true;
        for (int m = 0; m < M && sorted; ++m)
            for (int64_t s = p->slot_offset[m] + 1; s < p->slot_offset[m + 1]; ++s)
                if (views[s].z0 < views[s - 1].z0) { sorted = false; break; }
        K.z_sorted = sorted ? 1 : 0;
    }
    K.ldT = g.ny + 4;
    K.ldN = g.nx + 4;
    K.slabT = is3d ? (long long)(g.nz + 4) * K.ldT : K.ldT;
    K.slabN = is3d ? (long long)(g.nz + 4) * K.ldN : K.ldN;

    // FP launch shape: split rays into slice segments when a subset has too
    // few rays to fill the chip (256 CUs x 4 SIMDs, several waves each)
    int64_t waves = (p->max_subset_rays + 63) / 64;
    p->fp_nseg = 1;
    while (p->fp_nseg < 8 && waves * p->fp_nseg < 8192) p->fp_nseg *= 2;

    const size_t nvox = (size_t)g.nx * g.ny * g.nz;
    p->nvox = (int64_t)nvox;
    p->layT = (int64_t)g.nx * K.slabT;
    p->layN = (int64_t)g.ny * K.slabN;
    const size_t Bn = (size_t)batch;          // every per-image buffer holds the batch's images
    const int64_t bp_blocks = (int64_t)((g.nx + 31) / 32) * ((g.ny + 7) / 8) * ((g.nz + 7) / 8);
    p->n_partials = std::max<int64_t>({65536, bp_blocks + 16, (p->max_subset_rays + 63) / 64 + 16,
                                       (int64_t)M + 16});
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t r) { if (e == hipSuccess) e = r; };
    chk(dev_alloc(&p->d_rays, rays.size()));
    if (is3d) chk(dev_alloc(&p->d_raysz, raysz.size()));
    chk(dev_alloc(&p->d_views, views.size()));
    chk(dev_alloc(&p->d_rowv, (size_t)nr));
    chk(dev_alloc(&p->d_rowf, (size_t)nr));
    chk(dev_alloc(&p->d_xt, Bn * p->layT));
    chk(dev_alloc(&p->d_xn, Bn * p->layN));
    chk(dev_alloc(&p->d_gradR, Bn * nvox));
    chk(dev_alloc(&p->d_r, Bn * (size_t)p->max_subset_rays));
    chk(dev_alloc(&p->d_part, Bn * nvox));
    chk(dev_alloc(&p->d_part2, Bn * nvox));
    chk(dev_alloc(&p->d_v, Bn * nvox));
    // filtered sinogram of the initial image (fan-beam FBP, axial FDK)
    if (!is3d || (g.kind == LALM_CONE_AXIAL && g.n_views == g.n_views_per_turn))
        chk(dev_alloc(&p->d_fbpq, Bn * (size_t)p->nv * nr * p->nb));
    if (!is3d) {
        chk(dev_alloc(&p->d_xt1, Bn * p->layT));
        chk(dev_alloc(&p->d_xn1, Bn * p->layN));
        chk(dev_alloc(&p->d_xc, 4 * Bn * nvox));      // [step pair][candidate][image]
    }
    chk(dev_alloc(&p->d_partials, Bn * (size_t)p->n_partials));
    chk(dev_alloc(&p->d_sc, 2 * Bn));
    chk(dev_alloc(&p->d_tmp, Bn * (size_t)(64 + M)));
    if (e == hipSuccess)
        e = hipHostMalloc((void **)&p->h_sc, Bn * sizeof(lalm::DevScalars), hipHostMallocDefault);
    if (e != hipSuccess) {
        lalm::set_error(std::string("plan allocation failed: ") + hipGetErrorString(e));
        free_plan(p);
        return LALM_E_NOMEM;
    }
    chk(hipMemcpy(p->d_rays, rays.data(), rays.size() * sizeof(lalm::RayRec), hipMemcpyHostToDevice));
    if (is3d) chk(hipMemcpy(p->d_raysz, raysz.data(), raysz.size() * sizeof(lalm::RayRecZ), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->d_views, views.data(), views.size() * sizeof(lalm::ViewRec), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->d_rowv, rowv.data(), nr * sizeof(float), hipMemcpyHostToDevice));
    chk(hipMemcpy(p->d_rowf, rowf.data(), nr * sizeof(float), hipMemcpyHostToDevice));
    // the layouts' zero borders are written once, here, and never again
    chk(hipMemset(p->d_xt, 0, Bn * p->layT * sizeof(float)));
    chk(hipMemset(p->d_xn, 0, Bn * p->layN * sizeof(float)));
    if (!is3d) {
        chk(hipMemset(p->d_xt1, 0, Bn * p->layT * sizeof(float)));
        chk(hipMemset(p->d_xn1, 0, Bn * p->layN * sizeof(float)));
    }
    chk(hipMemset(p->d_gradR, 0, Bn * nvox * sizeof(float)));
    chk(hipMemset(p->d_sc, 0, 2 * Bn * sizeof(lalm::DevScalars)));
    chk(hipDeviceSynchronize());
    if (e != hipSuccess) {
        lalm::set_error(std::string("plan upload failed: ") + hipGetErrorString(e));
        free_plan(p);
        return LALM_E_HIP;
    }
    *out = p;
    return LALM_OK;
}

extern "C" lalm_status lalm_plan_info(const lalm_plan *p, int64_t *image_elems, int64_t *sino_elems,
                                      int64_t *subset_ray_offset, int32_t *order,
                                      int32_t *view_of_slot, int64_t *subset_samples)
{
    if (!p) return invalid("lalm_plan_info: null plan");
    if (image_elems) *image_elems = (int64_t)p->nx * p->ny * p->nz;
    if (sino_elems) *sino_elems = (int64_t)p->nv * p->rays_per_view;
    if (subset_ray_offset)
        for (int m = 0; m <= p->M; ++m) subset_ray_offset[m] = p->slot_offset[m] * p->rays_per_view;
    if (order) std::copy(p->order.begin(), p->order.end(), order);
    if (view_of_slot) std::copy(p->view_of_slot.begin(), p->view_of_slot.end(), view_of_slot);
    if (subset_samples) std::copy(p->subset_samples.begin(), p->subset_samples.end(), subset_samples);
    return LALM_OK;
}

extern "C" lalm_status lalm_plan_destroy(lalm_plan *p)
{
    if (!p) return invalid("lalm_plan_destroy: null plan");
    (void)hipDeviceSynchronize();
    free_plan(p);
    return LALM_OK;
}
