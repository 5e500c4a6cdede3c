// C ABI entry points: projections, SQS denominator, the OS-LALM iteration
// and the FP64 monitors.  Argument validation happens before any work is
// queued; launch failures map to LALM_E_HIP with the HIP error text.
#include <algorithm>
#include <cmath>
#include <string>

#include "lalm_internal.h"

using namespace lalm;

namespace {

lalm_status fail(lalm_status code, const std::string &msg)
{
    set_error(msg);
    return code;
}

lalm_status hip_fail(const char *where, hipError_t e)
{
    return fail(LALM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(where, expr)                                  \
    do {                                                     \
        hipError_t e_ = (expr);                              \
        if (e_ != hipSuccess) return hip_fail(where, e_);    \
    } while (0)

int64_t subset_slot0(const lalm_plan *p, int m) { return p->slot_offset[m]; }

// Opens a kernel class of lalm_iterate while profiling: the kernels that
// are launched until it closes are timed and attributed to it.
struct ProfScope {
    lalm_plan *p;
    ProfScope(lalm_plan *p_, int kind, hipStream_t) : p(p_)
    {
        if (!p->prof) return;
        p->prof_cls = kind;
        p->prof_n[kind] += 1;
    }
    ~ProfScope() { p->prof_cls = -1; }
};

// After a stream synchronization: fold recorded pairs into the totals.
void prof_collect(lalm_plan *p)
{
    if (!p->prof) return;
    for (size_t k = 0; k < p->prof_kind.size(); ++k) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p->prof_ev[2 * k], p->prof_ev[2 * k + 1]) == hipSuccess)
            p->prof_ms[p->prof_kind[k]] += ms;
    }
    p->prof_kind.clear();
    p->prof_used = 0;
}
int subset_nview(const lalm_plan *p, int m) { return (int)(p->slot_offset[m + 1] - p->slot_offset[m]); }
int64_t subset_ray0(const lalm_plan *p, int m) { return p->slot_offset[m] * p->rays_per_view; }
int64_t sino_elems(const lalm_plan *p) { return (int64_t)p->nv * p->rays_per_view; }

}  // namespace

extern "C" lalm_status lalm_project_subset(lalm_plan *p, int32_t m, const float *x, float *out_sub,
                                           const float *y_sub, const float *w_sub, hipStream_t st)
{
    if (!p || !x || !out_sub) return fail(LALM_E_INVALID, "lalm_project_subset: null argument");
    if (m < 0 || m >= p->M) return fail(LALM_E_INVALID, "lalm_project_subset: subset out of range");
    HIPCHK("project layout", launch_update(p, UPD_LAYOUT, const_cast<float *>(x), nullptr, nullptr,
                                           nullptr, 0.0f, 0, nullptr, st));
    // image b's subset arrays follow each other: stride = the subset's rays
    const int64_t n_m = subset_nview(p, m) * p->rays_per_view;
    HIPCHK("project", launch_fp(p, subset_slot0(p, m), subset_nview(p, m), y_sub, w_sub, out_sub, 0, 0,
                                nullptr, 0, st, 0, n_m, n_m));
    return LALM_OK;
}

extern "C" lalm_status lalm_backproject_subset(lalm_plan *p, int32_t m, const float *r_sub, float *x_out,
                                               float scale, int32_t accumulate, hipStream_t st)
{
    if (!p || !r_sub || !x_out) return fail(LALM_E_INVALID, "lalm_backproject_subset: null argument");
    if (m < 0 || m >= p->M) return fail(LALM_E_INVALID, "lalm_backproject_subset: subset out of range");
    BpEpi e{};
    e.scale = scale;
    e.accumulate = accumulate ? 1 : 0;
    e.out = x_out;
    e.r_stride = subset_nview(p, m) * p->rays_per_view;
    HIPCHK("backproject", launch_bp(p, subset_slot0(p, m), subset_nview(p, m), r_sub, BP_PLAIN, e, st));
    return LALM_OK;
}

extern "C" lalm_status lalm_sqs_denom(lalm_plan *p, const float *w_full, float *denom, hipStream_t st)
{
    if (!p || !w_full || !denom) return fail(LALM_E_INVALID, "lalm_sqs_denom: null argument");
    HIPCHK("sqs ones", launch_update(p, UPD_ONES, nullptr, nullptr, nullptr, nullptr, 0.0f, 0, nullptr, st));
    for (int m = 0; m < p->M; ++m) {
        // the library's own residuals carry each ray's scale (3D)
        HIPCHK("sqs project", launch_fp(p, subset_slot0(p, m), subset_nview(p, m), nullptr,
                                        w_full + subset_ray0(p, m), p->d_r, 0, 0, nullptr, 0, st, 1,
                                        sino_elems(p), p->max_subset_rays));
        BpEpi e{};
        e.scale = 1.0f;
        e.accumulate = m > 0;
        e.out = denom;
        e.ray_scaled = 1;
        e.r_stride = p->max_subset_rays;
        HIPCHK("sqs backproject", launch_bp(p, subset_slot0(p, m), subset_nview(p, m), p->d_r, BP_PLAIN, e, st));
    }
    return LALM_OK;
}

extern "C" lalm_status lalm_fbp(lalm_plan *p, const float *y_full, float *x_out, hipStream_t st)
{
    if (!p || !y_full || !x_out) return fail(LALM_E_INVALID, "lalm_fbp: null argument");
    if (p->g.kind == LALM_CONE_HELICAL || p->g.n_views != p->g.n_views_per_turn || !p->d_fbpq)
        return fail(LALM_E_INVALID, "lalm_fbp: 2D fan beam or axial cone beam over one full turn only");
    if (p->nb > fbp_max_bins()) return fail(LALM_E_INVALID, "lalm_fbp: too many channels");
    HIPCHK("fbp", launch_fbp(p, y_full, x_out, st));
    return LALM_OK;
}

extern "C" lalm_status lalm_iterate(lalm_plan *p, const lalm_problem *prob, lalm_state *s,
                                    int64_t n_steps, const lalm_options *opt, const lalm_stats *stats,
                                    hipStream_t st)
{
    if (!p || !prob || !s || !opt) return fail(LALM_E_INVALID, "lalm_iterate: null argument");
    if (!prob->y || !prob->w || !prob->denom) return fail(LALM_E_INVALID, "lalm_iterate: null problem array");
    if (!s->x || !s->g || !s->grad) return fail(LALM_E_INVALID, "lalm_iterate: null state array");
    if (opt->n_inner < 1 || opt->n_inner > LALM_MAX_INNER)
        return fail(LALM_E_INVALID, "lalm_iterate: n_inner must lie in [1, LALM_MAX_INNER]");
    if (n_steps < 0) return fail(LALM_E_INVALID, "lalm_iterate: negative step count");
    if (!(prob->beta >= 0.0) || !(prob->delta > 0.0)) return fail(LALM_E_INVALID, "lalm_iterate: need beta >= 0, delta > 0");
    if (!(opt->rho_min > 0.0 && opt->rho_min <= 1.0)) return fail(LALM_E_INVALID, "lalm_iterate: rho_min must lie in (0, 1]");
    if (!opt->continuation && !(opt->rho_fixed > 0.0)) return fail(LALM_E_INVALID, "lalm_iterate: rho_fixed must be positive");
    if (s->step < 0) return fail(LALM_E_STATE, "lalm_iterate: negative state step");
    const int B = p->B;
    if (B > 1 && (!s->l_b || !s->rho_b || !s->alpha_b))
        return fail(LALM_E_INVALID, "lalm_iterate: a batch needs state.l_b, rho_b and alpha_b");
    // continuation scalars of image b (the scalar fields for a single image)
    auto l_of = [&](int b) { return B > 1 ? s->l_b[b] : s->l; };
    auto rho_of = [&](int b) { return B > 1 ? s->rho_b[b] : s->rho; };
    auto alpha_of = [&](int b) { return B > 1 ? s->alpha_b[b] : s->alpha; };
    for (int b = 0; b < B; ++b)
        if (s->step > 0 && (l_of(b) < 0 || !(rho_of(b) > 0.0) || !std::isfinite(rho_of(b))))
            return fail(LALM_E_STATE, "lalm_iterate: inconsistent continuation state");
    if (opt->bb) {
        if (!s->x_prev || !s->grad_prev) return fail(LALM_E_INVALID, "lalm_iterate: bb needs state.x_prev and state.grad_prev");
        if (!(opt->bb_alpha_min > 0.0 && opt->bb_alpha_min <= 1.0))
            return fail(LALM_E_INVALID, "lalm_iterate: bb_alpha_min must lie in (0, 1]");
        for (int b = 0; b < B; ++b)
            if (s->step > 0 && !(alpha_of(b) > 0.0 && alpha_of(b) <= 1.0))
                return fail(LALM_E_STATE, "lalm_iterate: inconsistent Barzilai-Borwein state");
    }
    if (p->n_partials < p->bp_nblocks + 2 * 1024 || p->n_partials < 4096)
        return fail(LALM_E_STATE, "lalm_iterate: reduction workspace too small");

    const int M = p->M;
    const float beta = (float)prob->beta;
    const float dl = (float)prob->delta;
    const float inv_delta2 = 1.0f / (dl * dl);
    BpEpi e{};
    e.scale = (float)M;
    e.ray_scaled = 1;      // the residuals below come from launch_fp with ray_scaled
    e.r_stride = p->max_subset_rays;
    const int64_t S = sino_elems(p), R = p->max_subset_rays;
    e.G = s->grad;
    e.g = s->g;
    e.x = s->x;
    e.beta = beta;
    e.inv_delta2 = inv_delta2;
    e.cont.continuation = opt->continuation ? 1 : 0;
    e.cont.rho_fixed = opt->rho_fixed;
    e.cont.rho_min = opt->rho_min;
    e.cont.forced = opt->forced_restart;
    e.cont.forced_len = opt->forced_restart ? opt->forced_len : 0;
    if (stats) {
        e.cont.st_rho = stats->rho;
        e.cont.st_xi = stats->xi;
        e.cont.st_restart = stats->restart;
        e.cont.st_cap = stats->capacity;
    }

    if (s->step == 0) {
        for (int b = 0; b < B; ++b)
            HIPCHK("iterate scalars", launch_set_scalars(p, b, 0, opt->continuation ? 1.0 : opt->rho_fixed, 0, 1.0, st));
        HIPCHK("iterate layout", launch_update(p, UPD_LAYOUT, s->x, nullptr, nullptr, nullptr, 0.0f, 0, nullptr, st));
        const int m0 = p->order[0];
        HIPCHK("iterate init project", launch_fp(p, subset_slot0(p, m0), subset_nview(p, m0),
                                                 prob->y + subset_ray0(p, m0), prob->w + subset_ray0(p, m0),
                                                 p->d_r, 0, 0, nullptr, 1, st, 1, S, R));
        HIPCHK("iterate init backproject", launch_bp(p, subset_slot0(p, m0), subset_nview(p, m0), p->d_r,
                                                     BP_INIT, e, st));
    } else {
        for (int b = 0; b < B; ++b) {
            const double rho = opt->continuation ? rho_of(b) : opt->rho_fixed;
            HIPCHK("iterate scalars", launch_set_scalars(p, b, l_of(b), rho, s->step, opt->bb ? alpha_of(b) : 1.0, st));
        }
        HIPCHK("iterate resume", launch_reg_grad(p, s->x, beta, inv_delta2, st));
    }
    // The continuation decision after a step's back-projection is taken by
    // a one-block kernel, or in 2D by the next step's x-update kernel
    // (fused: every wave reduces the epilogue's partials; 3D has too many
    // partials for that).  No decision stays pending between calls.
    //
    // 2D with n = 1 and no Barzilai-Borwein scaling, within a call: the
    // step kernel after the back-projection also computes the next x for
    // both values the pending decision can give rho (restart or continue),
    // into one of two candidate pairs; the next forward projection takes
    // the decision and reads the chosen candidate's layouts, and the next
    // step kernel reads that candidate (and copies it to the caller's x).
    // Same arithmetic as the unfused path, one kernel fewer per step.
    const bool fused = !p->is3d && opt->n_inner == 1 && !opt->bb && n_steps >= 2;
    const size_t nvox = (size_t)p->nx * p->ny * p->nz;
    bool pending = false;
    for (int64_t t = 0; t < n_steps; ++t) {
        const int64_t j = s->step + t;
        const int m = p->order[(size_t)((j + 1) % M)];
        const bool f_in = fused && t > 0;             // x of this step is a candidate
        const bool f_out = fused && t + 1 < n_steps;  // this step makes the next candidates
        if (opt->bb && j % M == 0)
            HIPCHK("iterate bb", launch_bb(p, s->x, s->grad, s->x_prev, s->grad_prev, prob->denom, j > 0,
                                           opt->bb_alpha_min, st));
        if (!f_in) {
            ProfScope ps(p, 0, st);
            const int n = opt->n_inner;
            // FISTA on the inner problem: iteration 1 is the projected step
            // from x (its momentum is zero); z ping-pongs between the two
            // partial images, which the back-projector needs only later
            float *zb[2] = {p->d_part, p->d_part2};
            HIPCHK("iterate update", launch_update(p, UPD_STEP, s->x, s->grad, s->g, prob->denom, beta,
                                                   prob->nonneg, pending ? &e.cont : nullptr, st,
                                                   n > 1 ? p->d_v : nullptr, n > 1 ? zb[0] : nullptr));
            pending = false;
            double tk = 0.5 * (1.0 + std::sqrt(5.0));     // t_2 (t_1 = 1)
            for (int it = 2; it <= n; ++it) {
                const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * tk * tk));
                const float mom = (float)((tk - 1.0) / tn);
                HIPCHK("iterate inner", launch_inner(p, zb[it % 2], p->d_v, zb[(it + 1) % 2], s->x, s->grad, s->g,
                                                     prob->denom, beta, inv_delta2, mom, prob->nonneg, it == n, st));
                tk = tn;
            }
        }
        {
            ProfScope ps(p, 1, st);
            if (f_in)
                HIPCHK("iterate project", launch_fp_decide(p, subset_slot0(p, m), subset_nview(p, m),
                                                           prob->y + subset_ray0(p, m),
                                                           prob->w + subset_ray0(p, m), p->d_r, e.cont, st, S, R));
            else
                HIPCHK("iterate project", launch_fp(p, subset_slot0(p, m), subset_nview(p, m),
                                                    prob->y + subset_ray0(p, m), prob->w + subset_ray0(p, m),
                                                    p->d_r, 0, 0, nullptr, 1, st, 1, S, R));
        }
        if (!fused) {
            ProfScope ps(p, 2, st);
            HIPCHK("iterate backproject", launch_bp(p, subset_slot0(p, m), subset_nview(p, m), p->d_r,
                                                    BP_STEP, e, st));
            if (p->is3d) HIPCHK("iterate finalize", launch_finalize(p, e.cont, st));
            else pending = true;
            continue;
        }
        {
            ProfScope ps(p, 2, st);
            HIPCHK("iterate backproject", launch_bp(p, subset_slot0(p, m), subset_nview(p, m), p->d_r,
                                                    BP_LINES, e, st));
        }
        {
            ProfScope ps(p, 0, st);
            // candidates: [step pair][candidate][image of the batch]
            const size_t cand = (size_t)B * nvox;
            const float *xs = f_in ? p->d_xc + (size_t)((t - 1) % 2) * 2 * cand : s->x;
            float *xo = p->d_xc + (size_t)(t % 2) * 2 * cand;
            HIPCHK("iterate step", launch_step2d(p, xs, f_in ? xs + cand : s->x, f_in ? s->x : nullptr,
                                                 f_out ? xo : nullptr, f_out ? xo + cand : nullptr, e,
                                                 prob->denom, prob->nonneg, !f_out, st));
        }
        pending = true;
    }
    if (pending) HIPCHK("iterate finalize", launch_finalize(p, e.cont, st));
    HIPCHK("iterate readback", hipMemcpyAsync(p->h_sc, cur_sc(p), (size_t)B * sizeof(DevScalars),
                                              hipMemcpyDeviceToHost, st));
    HIPCHK("iterate sync", hipStreamSynchronize(st));
    prof_collect(p);
    bool nonfinite = false;
    int64_t step = 0;
    for (int b = 0; b < B; ++b) {
        const DevScalars &h = p->h_sc[b];
        nonfinite = nonfinite || h.status;
        step = std::max<int64_t>(step, h.step);
        if (s->l_b) s->l_b[b] = h.l;
        if (s->rho_b) s->rho_b[b] = h.rho;
        if (s->alpha_b) s->alpha_b[b] = h.alpha;
    }
    s->step = step;
    s->l = p->h_sc[0].l;
    s->rho = p->h_sc[0].rho;
    s->alpha = p->h_sc[0].alpha;
    if (nonfinite)
        return fail(LALM_E_NONFINITE, "lalm_iterate: non-finite restart indicator; later steps skipped");
    return LALM_OK;
}

extern "C" lalm_status lalm_cost_f64(lalm_plan *p, const lalm_problem *prob, const float *x,
                                     double *out_dev, hipStream_t st)
{
    if (!p || !prob || !x || !out_dev || !prob->y || !prob->w)
        return fail(LALM_E_INVALID, "lalm_cost_f64: null argument");
    if (!(prob->delta > 0.0)) return fail(LALM_E_INVALID, "lalm_cost_f64: need delta > 0");
    HIPCHK("cost layout", launch_update(p, UPD_LAYOUT, const_cast<float *>(x), nullptr, nullptr, nullptr,
                                        0.0f, 0, nullptr, st));
    const int64_t ntmp = 64 + p->M;        // FP64 scratch per image
    for (int m = 0; m < p->M; ++m) {
        int64_t nblk = 0;
        HIPCHK("cost project", launch_fp(p, subset_slot0(p, m), subset_nview(p, m), prob->y + subset_ray0(p, m),
                                         prob->w + subset_ray0(p, m), nullptr, 1, 0, &nblk, 0, st, 0,
                                         sino_elems(p), 0));
        for (int b = 0; b < p->B; ++b)
            HIPCHK("cost sum", launch_sum_partials(p->d_partials + b * p->n_partials, nblk,
                                                   p->d_tmp + b * ntmp + 8 + m, 1.0, st));
    }
    for (int b = 0; b < p->B; ++b) {
        double *t = p->d_tmp + b * ntmp;
        HIPCHK("cost data", launch_sum_partials(t + 8, p->M, t + 0, 1.0, st));
        HIPCHK("cost reg", launch_reg_value(p, x + b * p->nvox, prob->beta, prob->delta, t + 1, st));
        HIPCHK("cost combine", launch_combine_cost(out_dev + 3 * b, t + 0, t + 1, st));
    }
    return LALM_OK;
}

extern "C" lalm_status lalm_dot_f64(lalm_plan *p, const float *a, const float *b, int64_t n,
                                    double *out_dev, hipStream_t st)
{
    if (!p || !a || !b || !out_dev || n < 0) return fail(LALM_E_INVALID, "lalm_dot_f64: bad argument");
    HIPCHK("dot", launch_dot(p, a, b, n, out_dev, st));
    return LALM_OK;
}

extern "C" lalm_status lalm_roi_rmsd_f64(lalm_plan *p, const float *a, const float *b, double radius_mm,
                                         double *out_dev, hipStream_t st)
{
    if (!p || !a || !b || !out_dev || !(radius_mm >= 0.0))
        return fail(LALM_E_INVALID, "lalm_roi_rmsd_f64: bad argument");
    for (int k = 0; k < p->B; ++k)
        HIPCHK("rmsd", launch_rmsd(p, a + k * p->nvox, b + k * p->nvox, radius_mm, out_dev + k, st));
    return LALM_OK;
}

extern "C" lalm_status lalm_profile_begin(lalm_plan *p)
{
    if (!p) return fail(LALM_E_INVALID, "lalm_profile_begin: null plan");
    p->prof = true;
    p->prof_kind.clear();
    p->prof_used = 0;
    for (int k = 0; k < 3; ++k) { p->prof_ms[k] = 0.0; p->prof_n[k] = 0; }
    return LALM_OK;
}

extern "C" lalm_status lalm_profile_read(lalm_plan *p, double *ms, int64_t *counts)
{
    if (!p || !ms || !counts) return fail(LALM_E_INVALID, "lalm_profile_read: null argument");
    for (int k = 0; k < 3; ++k) { ms[k] = p->prof_ms[k]; counts[k] = p->prof_n[k]; }
    return LALM_OK;
}

extern "C" lalm_status lalm_profile_end(lalm_plan *p)
{
    if (!p) return fail(LALM_E_INVALID, "lalm_profile_end: null plan");
    p->prof = false;
    for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
    p->prof_ev.clear();
    p->prof_kind.clear();
    p->prof_used = 0;
    return LALM_OK;
}
