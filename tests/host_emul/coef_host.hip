// TEST FIXTURE: runs the library's coefficient-pass routines (the per-element
// bodies of coef_radial_kernel / coef_theta_kernel / coef_point_kernel) in
// plain host loops, so CPU-only tests can check them against the oracle.
// The library itself never runs these on the host.
#include <vector>

#include "prec_impl.hpp"

using namespace lwk;

template <class T>
static int run(CoefJob &J, double *ch, double *cf, double *wt) {
    constexpr int W = words_of<T>::value;
    const int n = 2 * J.nr - 1, nth = J.nth;
    CoefSetup<T> S = coef_setup<T>(J);
    std::vector<double> r((size_t)W * n), d((size_t)W * n), c((size_t)W * nth), s2((size_t)W * nth);
    for (int t = 0; t < n; ++t) coef_radial_one<T>(S.RP, t, S.rsmin, S.h, S.rp, S.dpm, S.A, S.B, r.data(), d.data());
    for (int j = 0; j < nth; ++j) coef_theta_one<T>(S.TP, j, S.dth, c.data(), s2.data(), wt);
    if constexpr (W == 1) {
        // FP64: the kernel rebuilds the coefficients per point from radial rows (as on the device)
        const double sh = S.hdt, sih = mp_mul(S.hdt, S.ih), sf = S.dt, sif = mp_mul(S.dt, S.ih);
        std::vector<double> row(kRadRow);
        for (int t = 0; t < n; ++t) {
            const bool half = t >= J.nr;
            const int i = half ? t - J.nr : t, ni = half ? J.nr - 1 : J.nr;
            coef_fp64_radial_row(J.s, J.m, J.mass, J.a_over_M * J.mass, r[t], d[t], half ? sh : sf, half ? sih : sif,
                                 row.data());
            for (int j = 0; j < nth; ++j) {
                double cc[8];
                coef_fp64_point(row.data(), c[j], s2[j], cc);
                for (int k = 0; k < 8; ++k) (half ? ch : cf)[(size_t)k * ni * nth + (size_t)i * nth + j] = cc[k];
            }
        }
    } else {
        for (int t = 0; t < n; ++t)
            for (int j = 0; j < nth; ++j)
                coef_point_one<T>(S.PP, t, j, r.data(), d.data(), c.data(), s2.data(), S.hdt, mp_mul(S.hdt, S.ih),
                                  S.dt, mp_mul(S.dt, S.ih), ch, cf);
    }
    return 0;
}

// ch: [8*W][n_r-1][n_theta], cf: [8*W][n_r][n_theta], wt: [(2R+1)*W][n_theta] (device layout)
extern "C" int coef_host(int words, int s, int m, double a_over_M, int nr, int nth, double rsmin, double rsmax,
                         double cfl, double mass, int order, double *ch, double *cf, double *wt, double *scal) {
    CoefJob J{};
    J.s = s; J.m = m; J.nr = nr; J.nth = nth; J.reach = order / 2;
    J.a_over_M = a_over_M; J.mass = mass; J.rstar_min = rsmin; J.rstar_max = rsmax; J.cfl = cfl;
    int rc = words == 1 ? run<double>(J, ch, cf, wt) : words == 2 ? run<dd>(J, ch, cf, wt) : run<qd>(J, ch, cf, wt);
    for (int k = 0; k < kMaxWords; ++k) { scal[k] = J.hdt[k]; scal[kMaxWords + k] = J.dt[k]; }
    return rc;
}

// Double-double per-point mode: the planes the step kernel forms per point
// from double-double radial rows (coef_radial_row_mp + coef_dd_point), same
// layouts as coef_host.
extern "C" int coef_host_dd_rows(int s, int m, double a_over_M, int nr, int nth, double rsmin, double rsmax,
                                 double cfl, double mass, int order, double *ch, double *cf, double *wt, double *scal) {
    CoefJob J{};
    J.s = s; J.m = m; J.nr = nr; J.nth = nth; J.reach = order / 2;
    J.a_over_M = a_over_M; J.mass = mass; J.rstar_min = rsmin; J.rstar_max = rsmax; J.cfl = cfl;
    constexpr int W = 2;
    const int n = 2 * J.nr - 1;
    CoefSetup<dd> S = coef_setup<dd>(J);
    std::vector<double> r((size_t)W * n), d((size_t)W * n), c((size_t)W * nth), s2((size_t)W * nth);
    for (int t = 0; t < n; ++t) coef_radial_one<dd>(S.RP, t, S.rsmin, S.h, S.rp, S.dpm, S.A, S.B, r.data(), d.data());
    for (int j = 0; j < nth; ++j) coef_theta_one<dd>(S.TP, j, S.dth, c.data(), s2.data(), wt);
    std::vector<double> rows((size_t)kRadRow * W * n);
    for (int t = 0; t < n; ++t) {
        const bool half = t >= J.nr;
        dd row[kRadRow];
        coef_radial_row_mp<dd>(J.s, J.m, J.mass, J.a_over_M * J.mass, ld<dd>(r.data(), (size_t)n, (size_t)t),
                               ld<dd>(d.data(), (size_t)n, (size_t)t), half ? S.hdt : S.dt,
                               half ? mp_mul(S.hdt, S.ih) : mp_mul(S.dt, S.ih), row);
        const int i = half ? t - J.nr : t, ni = half ? J.nr - 1 : J.nr;
        for (int k = 0; k < kRadRow; ++k) {
            rows[(size_t)t * kRadRow * W + 2 * k] = row[k].x0;
            rows[(size_t)t * kRadRow * W + 2 * k + 1] = row[k].x1;
        }
        for (int j = 0; j < nth; ++j) {
            dd cc[8];
            coef_dd_point(rows.data() + (size_t)t * kRadRow * W, ld<dd>(c.data(), (size_t)nth, (size_t)j),
                          ld<dd>(s2.data(), (size_t)nth, (size_t)j), cc);
            double *out = half ? ch : cf;
            const size_t plane = (size_t)ni * nth;
            for (int k = 0; k < 8; ++k) st(out + (size_t)k * W * plane, plane, (size_t)i * nth + j, cc[k]);
        }
    }
    for (int k = 0; k < kMaxWords; ++k) { scal[k] = J.hdt[k]; scal[kMaxWords + k] = J.dt[k]; }
    return 0;
}

// One full step of the scheme on the host with the kernel's own stage routines
// (lw_stage, pt_avg, pt_diff) and the device data layout; the angular operator
// is applied with the same folded weights and reflected row index.
template <class T>
static void step_host(int nr, int nth, int R, const double *ch, const double *cf, const double *wt, const double *hdtw,
                      const double *dtw, const double *uin, double *uout) {
    constexpr int W = words_of<T>::value;
    const size_t plane = (size_t)nr * nth, hplane = (size_t)(nr - 1) * nth;
    const T hdt = from_words<T>(hdtw), dt = from_words<T>(dtw);
    auto theta = [&](const std::vector<cx<T>> &col, int j) {
        Acc<T> re, im;
        for (int k = -R; k <= R; ++k) {
            int q = j + k;
            q = q < 0 ? -1 - q : (q >= nth ? 2 * nth - 1 - q : q);
            const T w = ld<T>(wt + (size_t)(k + R) * W * nth, (size_t)nth, (size_t)j);
            re.prod(w, col[q].re);
            im.prod(w, col[q].im);
        }
        return cx<T>{re.result(), im.result()};
    };
    std::vector<Pt<T>> u((size_t)nr * nth), uh((size_t)(nr - 1) * nth);
    std::vector<cx<T>> L((size_t)nr * nth), Lh((size_t)(nr - 1) * nth), col(nth);
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nth; ++j) u[(size_t)i * nth + j] = ld_pt<T>(uin, plane, (size_t)i * nth + j);
    for (int i = 0; i < nr; ++i) {
        for (int j = 0; j < nth; ++j) col[j] = u[(size_t)i * nth + j].phi;
        for (int j = 0; j < nth; ++j) L[(size_t)i * nth + j] = theta(col, j);
    }
    for (int i = 0; i + 1 < nr; ++i)
        for (int j = 0; j < nth; ++j) {
            T c[8];
            for (int q = 0; q < 8; ++q) c[q] = ld<T>(ch + (size_t)q * W * hplane, hplane, (size_t)i * nth + j);
            const Pt<T> &a = u[(size_t)i * nth + j], &b = u[(size_t)(i + 1) * nth + j];
            const Pt<T> bar = pt_avg(a, b);
            uh[(size_t)i * nth + j] = lw_stage(bar, bar, pt_diff(a, b),
                                               c_avg(L[(size_t)i * nth + j], L[(size_t)(i + 1) * nth + j]), c, hdt);
        }
    for (int i = 0; i + 1 < nr; ++i) {
        for (int j = 0; j < nth; ++j) col[j] = uh[(size_t)i * nth + j].phi;
        for (int j = 0; j < nth; ++j) Lh[(size_t)i * nth + j] = theta(col, j);
    }
    const Pt<T> z = {{mp_from<T>(0.0), mp_from<T>(0.0)}, {mp_from<T>(0.0), mp_from<T>(0.0)}};
    for (int j = 0; j < nth; ++j) {
        st_pt(uout, plane, (size_t)j, z);
        st_pt(uout, plane, (size_t)(nr - 1) * nth + j, z);
    }
    for (int i = 1; i + 1 < nr; ++i)
        for (int j = 0; j < nth; ++j) {
            T c[8];
            for (int q = 0; q < 8; ++q) c[q] = ld<T>(cf + (size_t)q * W * plane, plane, (size_t)i * nth + j);
            const Pt<T> &a = uh[(size_t)(i - 1) * nth + j], &b = uh[(size_t)i * nth + j];
            const Pt<T> un = lw_stage(u[(size_t)i * nth + j], pt_avg(a, b), pt_diff(a, b),
                                      c_avg(Lh[(size_t)(i - 1) * nth + j], Lh[(size_t)i * nth + j]), c, dt);
            st_pt(uout, plane, (size_t)i * nth + j, un);
        }
}

// u: device-layout state [4*W][n_r][n_theta], advanced nsteps in place
extern "C" int step_host(int words, int nr, int nth, int order, const double *ch, const double *cf, const double *wt,
                         const double *scal, double *u, int nsteps) {
    const size_t n = 4 * (size_t)words * nr * nth;
    std::vector<double> tmp(n);
    for (int s = 0; s < nsteps; ++s) {
        if (words == 1) step_host<double>(nr, nth, order / 2, ch, cf, wt, scal, scal + kMaxWords, u, tmp.data());
        else if (words == 2) step_host<dd>(nr, nth, order / 2, ch, cf, wt, scal, scal + kMaxWords, u, tmp.data());
        else step_host<qd>(nr, nth, order / 2, ch, cf, wt, scal, scal + kMaxWords, u, tmp.data());
        for (size_t k = 0; k < n; ++k) u[k] = tmp[k];
    }
    return 0;
}
