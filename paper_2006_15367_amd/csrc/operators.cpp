// FP64 host precompute of the per-level tables (setup; not in the matvec).
//
// Per level l >= 3 (Sec. 3.2.3 "translation operators", precomputed once):
//   * truncation order L = ceil(k d + 1.8 digits^(2/3) (k d)^(1/3)),
//     d = sqrt(3) a_l (the box diagonal);
//   * samples: L+1 Gauss-Legendre nodes in cos(theta) x 2L+2 uniform phi;
//   * translation operators of every offset used by the far lists,
//       T(khat) = sum_{l<=L} i^l (2l+1) h_l^(1)(k|X|) P_l(khat . X/|X|);
//   * shift phases exp(-i k khat.(c_c - c_p)) for the 8 child octants;
//   * the exact band-limited interpolation child -> parent (Sec. 3.2.2,
//     global interpolation) as real DFT x per-order Legendre map x real
//     synthesis, and its weighted adjoint (anterpolation, Sec. 3.2.4).
#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <thread>

#include "internal.h"

namespace mlfma {

using cplx = std::complex<double>;

int truncation_order(double k, double a, int digits)
{
    const double kd = k * std::sqrt(3.0) * a;
    return (int)std::ceil(kd + 1.8 * std::pow((double)digits, 2.0 / 3.0) *
                                   std::pow(kd, 1.0 / 3.0));
}

// n-point Gauss-Legendre rule, nodes descending; Newton on P_n in long double.
static void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.resize(n);
    w.resize(n);
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) {
        long double z = std::cos(pi * (i + 0.75L) / (n + 0.5L));
        long double dp = 1;
        for (int it = 0; it < 100; ++it) {
            long double p0 = 1, p1 = z;
            for (int l = 2; l <= n; ++l) {
                long double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p0 = 1; p1 = z; }
            dp = n * (z * p1 - p0) / (z * z - 1);
            long double dz = p1 / dp;
            z -= dz;
            if (std::fabs((double)dz) < 1e-19) break;
        }
        long double p0 = 1, p1 = z;
        for (int l = 2; l <= n; ++l) {
            long double p2 = ((2 * l - 1) * z * p1 - (l - 1) * p0) / l;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p0 = 1; p1 = z; }
        dp = n * (z * p1 - p0) / (z * z - 1);
        x[i] = (double)z;
        w[i] = (double)(2.0L / ((1 - z) * (1 + z) * dp * dp));
    }
}

// Pbar_l^m(x_i) for l = m..lmax (unit L2 norm on [-1,1], no Condon-Shortley
// sign); out[(l-m)*nx + i].
static void pbar_order(int lmax, int m, const std::vector<double> &x, std::vector<double> &out)
{
    const int nx = (int)x.size();
    out.assign((size_t)(lmax - m + 1) * nx, 0.0);
    for (int i = 0; i < nx; ++i) {
        const double s = std::sqrt((1.0 - x[i]) * (1.0 + x[i]));
        double pmm = std::sqrt(0.5);
        for (int mm = 1; mm <= m; ++mm) pmm *= std::sqrt((2.0 * mm + 1.0) / (2.0 * mm)) * s;
        double lm2 = 0, lm1 = pmm;
        out[i] = pmm;
        if (lmax > m) {
            double v = std::sqrt(2.0 * m + 3.0) * x[i] * pmm;
            out[(size_t)nx + i] = v;
            lm2 = pmm;
            lm1 = v;
        }
        for (int l = m + 2; l <= lmax; ++l) {
            const double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
            const double b = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) /
                                       (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
            const double v = a * (x[i] * lm1 - b * lm2);
            out[(size_t)(l - m) * nx + i] = v;
            lm2 = lm1;
            lm1 = v;
        }
    }
}

// spherical Hankel functions of the first kind, l = 0..L, upward recurrence
static void hankel1(int L, double z, std::vector<cplx> &h)
{
    h.resize(L + 1);
    const cplx e = std::exp(cplx(0.0, z));
    h[0] = cplx(0.0, -1.0) * e / z;
    if (L >= 1) h[1] = -e * cplx(z, 1.0) / (z * z);
    for (int l = 1; l < L; ++l) h[l + 1] = (2.0 * l + 1.0) / z * h[l] - h[l - 1];
}

static void run_parallel(int n, const std::function<void(int)> &fn)
{
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int nth = (int)std::min<unsigned>(hw, (unsigned)std::max(1, n));
    std::vector<std::thread> th;
    for (int t = 0; t < nth; ++t)
        th.emplace_back([&, t]() {
            for (int i = t; i < n; i += nth) fn(i);
        });
    for (auto &x : th) x.join();
}

static void real_dft(int nphi_in, int M, std::vector<float> &F)
{
    // F[j][col]: col 0 -> 1/N, col 2m-1 -> cos(m phi_j)/N, col 2m -> sin(m phi_j)/N
    F.assign((size_t)nphi_in * M, 0.f);
    for (int j = 0; j < nphi_in; ++j) {
        const double ph = 2.0 * M_PI * j / nphi_in;
        F[(size_t)j * M] = (float)(1.0 / nphi_in);
        for (int m = 1; 2 * m <= M - 1; ++m) {
            F[(size_t)j * M + 2 * m - 1] = (float)(std::cos(m * ph) / nphi_in);
            F[(size_t)j * M + 2 * m] = (float)(std::sin(m * ph) / nphi_in);
        }
    }
}

static void real_synthesis(int M, int nphi_out, std::vector<float> &G)
{
    // G[col][j]: col 0 -> 1, col 2m-1 -> 2cos(m phi_j), col 2m -> 2sin(m phi_j)
    G.assign((size_t)M * nphi_out, 0.f);
    for (int j = 0; j < nphi_out; ++j) {
        const double ph = 2.0 * M_PI * j / nphi_out;
        G[j] = 1.f;
        for (int m = 1; 2 * m <= M - 1; ++m) {
            G[(size_t)(2 * m - 1) * nphi_out + j] = (float)(2.0 * std::cos(m * ph));
            G[(size_t)(2 * m) * nphi_out + j] = (float)(2.0 * std::sin(m * ph));
        }
    }
}

// maps[m][i_from][i_to] = sum_{l=m}^{Lband} Pbar_l^m(x_to) Pbar_l^m(x_from) w_from
// (stored with the input index first: it is the K index of the contraction)
static void legendre_maps(int Lband, const std::vector<double> &xf, const std::vector<double> &wf,
                          const std::vector<double> &xt, std::vector<float> &maps)
{
    const int nf = (int)xf.size(), nt = (int)xt.size();
    maps.assign((size_t)(Lband + 1) * nt * nf, 0.f);
    run_parallel(Lband + 1, [&](int m) {
        std::vector<double> Pf, Pt;
        pbar_order(Lband, m, xf, Pf);
        pbar_order(Lband, m, xt, Pt);
        for (int a = 0; a < nt; ++a)
            for (int b = 0; b < nf; ++b) {
                double s = 0;
                for (int l = m; l <= Lband; ++l)
                    s += Pt[(size_t)(l - m) * nt + a] * Pf[(size_t)(l - m) * nf + b];
                maps[((size_t)m * nf + b) * nt + a] = (float)(s * wf[b]);
            }
    });
}

int build_level_tables(const Tree &t, double k, int digits, std::vector<LevelTables> &out,
                       bool sampled)
{
    out.clear();
    out.resize(t.n_lev + 1);
    if (t.n_lev < 3) return MLFMA_OK;
    try {
        for (int l = 3; l <= t.n_lev; ++l) {
            LevelTables &T = out[l];
            T.L = truncation_order(k, t.lev[l].a, digits);
            T.nth = T.L + 1;
            T.nph = 2 * T.L + 2;
            T.K = (int64_t)T.nth * T.nph;
            gauss_legendre(T.nth, T.x, T.wx);
            T.khat_w.resize(4 * T.K);
            for (int i = 0; i < T.nth; ++i) {
                const double st = std::sqrt((1.0 - T.x[i]) * (1.0 + T.x[i]));
                for (int j = 0; j < T.nph; ++j) {
                    const double ph = 2.0 * M_PI * j / T.nph;
                    float *o = &T.khat_w[4 * ((size_t)i * T.nph + j)];
                    o[0] = (float)(st * std::cos(ph));
                    o[1] = (float)(st * std::sin(ph));
                    o[2] = (float)T.x[i];
                    o[3] = (float)(T.wx[i] * 2.0 * M_PI / T.nph);
                }
            }
            // translation operators of the offsets in use
            const HostLevel &HL = t.lev[l];
            T.code_to_type.assign(343, -1);
            std::vector<int> codes;
            for (int16_t c : HL.far_code)
                if (T.code_to_type[c] < 0) {
                    T.code_to_type[c] = 0;
                    codes.push_back(c);
                }
            std::sort(codes.begin(), codes.end());
            for (size_t i = 0; i < codes.size(); ++i) T.code_to_type[codes[i]] = (int16_t)i;
            T.ntypes = (int)codes.size();
            T.far_type.resize(HL.far_code.size());
            for (size_t e = 0; e < HL.far_code.size(); ++e)
                T.far_type[e] = T.code_to_type[HL.far_code[e]];
            const double a = HL.a;
            if (sampled) {
                // Sec. 3.2.3 "Translation Operators": sampled operators.  T
                // depends on the direction only through the angle gamma to
                // the offset and is a cosine polynomial of degree L in it;
                // tabulate it per distinct offset length at M + 1 angles,
                // M = 8 L, for interpolation at the grid directions.
                std::vector<int> rad_of_n2(28, -1), n2_of_rad;
                for (int code : codes) {
                    const int dx = code / 49 - 3, dy = (code / 7) % 7 - 3, dz = code % 7 - 3;
                    const int n2 = dx * dx + dy * dy + dz * dz;
                    if (rad_of_n2[n2] < 0) {
                        rad_of_n2[n2] = (int)n2_of_rad.size();
                        n2_of_rad.push_back(n2);
                    }
                }
                T.nrad = (int)n2_of_rad.size();
                T.Msamp = kSampledOversample * T.L;
                const int Ms = T.Msamp;
                T.Tsamp.assign((size_t)T.nrad * (Ms + 1) * 2, 0.f);
                run_parallel(T.nrad, [&](int ri) {
                    const double r = a * std::sqrt((double)n2_of_rad[ri]);
                    std::vector<cplx> h;
                    hankel1(T.L, k * r, h);
                    std::vector<cplx> coef(T.L + 1);
                    cplx il(1.0, 0.0);
                    for (int ll = 0; ll <= T.L; ++ll) {
                        coef[ll] = il * (2.0 * ll + 1.0) * h[ll];
                        il *= cplx(0.0, 1.0);
                    }
                    for (int m = 0; m <= Ms; ++m) {
                        const double u = std::cos(M_PI * m / Ms);
                        double p0 = 1.0, p1 = u;
                        cplx sum = coef[0];
                        if (T.L >= 1) sum += coef[1] * u;
                        for (int ll = 1; ll < T.L; ++ll) {
                            const double p2 = ((2.0 * ll + 1.0) * u * p1 - ll * p0) / (ll + 1.0);
                            p0 = p1;
                            p1 = p2;
                            sum += coef[ll + 1] * p2;
                        }
                        float *o = &T.Tsamp[2 * ((size_t)ri * (Ms + 1) + m)];
                        o[0] = (float)sum.real();
                        o[1] = (float)sum.imag();
                    }
                });
                T.xr.assign((size_t)T.ntypes * 4, 0.f);
                for (int ti = 0; ti < T.ntypes; ++ti) {
                    const int code = codes[ti];
                    const int dx = code / 49 - 3, dy = (code / 7) % 7 - 3, dz = code % 7 - 3;
                    T.xr[4 * ti + 0] = (float)dx;
                    T.xr[4 * ti + 1] = (float)dy;
                    T.xr[4 * ti + 2] = (float)dz;
                    T.xr[4 * ti + 3] = (float)rad_of_n2[dx * dx + dy * dy + dz * dz];
                }
                T.trig64.resize((size_t)2 * (T.nth + T.nph));
                for (int i = 0; i < T.nth; ++i) {
                    T.trig64[2 * i] = T.x[i];
                    T.trig64[2 * i + 1] = std::sqrt((1.0 - T.x[i]) * (1.0 + T.x[i]));
                }
                for (int j = 0; j < T.nph; ++j) {
                    const double ph = 2.0 * M_PI * j / T.nph;
                    T.trig64[2 * (T.nth + j)] = std::cos(ph);
                    T.trig64[2 * (T.nth + j) + 1] = std::sin(ph);
                }
                continue;
            }
            T.T.assign((size_t)T.ntypes * T.K * 2, 0.f);
            run_parallel(T.ntypes, [&](int ti) {
                const int code = codes[ti];
                const double dx = code / 49 - 3, dy = (code / 7) % 7 - 3, dz = code % 7 - 3;
                const double X[3] = {a * dx, a * dy, a * dz};
                const double r = std::sqrt(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
                std::vector<cplx> h;
                hankel1(T.L, k * r, h);
                std::vector<cplx> coef(T.L + 1);
                cplx il(1.0, 0.0);
                for (int ll = 0; ll <= T.L; ++ll) {
                    coef[ll] = il * (2.0 * ll + 1.0) * h[ll];
                    il *= cplx(0.0, 1.0);
                }
                for (int i = 0; i < T.nth; ++i) {
                    const double st = std::sqrt((1.0 - T.x[i]) * (1.0 + T.x[i]));
                    for (int j = 0; j < T.nph; ++j) {
                        const double ph = 2.0 * M_PI * j / T.nph;
                        const double u = (st * std::cos(ph) * X[0] + st * std::sin(ph) * X[1] +
                                          T.x[i] * X[2]) / r;
                        double p0 = 1.0, p1 = u;
                        cplx s = coef[0];
                        if (T.L >= 1) s += coef[1] * u;
                        for (int ll = 1; ll < T.L; ++ll) {
                            const double p2 = ((2.0 * ll + 1.0) * u * p1 - ll * p0) / (ll + 1.0);
                            p0 = p1;
                            p1 = p2;
                            s += coef[ll + 1] * p2;
                        }
                        float *o = &T.T[2 * ((size_t)ti * T.K + (size_t)i * T.nph + j)];
                        o[0] = (float)s.real();
                        o[1] = (float)s.imag();
                    }
                }
            });
        }
        // level pairs: this level p = l (parent), child l+1
        for (int l = 3; l < t.n_lev; ++l) {
            LevelTables &P = out[l];
            const LevelTables &C = out[l + 1];
            P.Lc = C.L;
            P.Mc = 2 * C.L + 1;
            const double q = t.lev[l].a / 4.0;
            P.shift.resize((size_t)8 * P.K * 2);
            for (int o = 0; o < 8; ++o) {
                const double d[3] = {q * (2 * ((o >> 2) & 1) - 1), q * (2 * ((o >> 1) & 1) - 1),
                                     q * (2 * (o & 1) - 1)};
                for (int i = 0; i < P.nth; ++i) {
                    const double st = std::sqrt((1.0 - P.x[i]) * (1.0 + P.x[i]));
                    for (int j = 0; j < P.nph; ++j) {
                        const double ph = 2.0 * M_PI * j / P.nph;
                        const double kd = k * (st * std::cos(ph) * d[0] + st * std::sin(ph) * d[1] +
                                               P.x[i] * d[2]);
                        float *e = &P.shift[2 * ((size_t)o * P.K + (size_t)i * P.nph + j)];
                        e[0] = (float)std::cos(kd);
                        e[1] = (float)(-std::sin(kd));
                    }
                }
            }
            // axis factors of the shift: the octant's shift is their product,
            // each conjugated where the octant bit is 0
            P.shift_axis.resize((size_t)2 * (2 * P.K + P.nth));
            for (int i = 0; i < P.nth; ++i) {
                const double st = std::sqrt((1.0 - P.x[i]) * (1.0 + P.x[i]));
                for (int j = 0; j < P.nph; ++j) {
                    const double ph = 2.0 * M_PI * j / P.nph;
                    const size_t e = (size_t)i * P.nph + j;
                    const double ax = k * q * st * std::cos(ph), ay = k * q * st * std::sin(ph);
                    P.shift_axis[2 * e] = (float)std::cos(ax);
                    P.shift_axis[2 * e + 1] = (float)(-std::sin(ax));
                    P.shift_axis[2 * (P.K + e)] = (float)std::cos(ay);
                    P.shift_axis[2 * (P.K + e) + 1] = (float)(-std::sin(ay));
                }
                const double az = k * q * P.x[i];
                P.shift_axis[2 * (2 * P.K + i)] = (float)std::cos(az);
                P.shift_axis[2 * (2 * P.K + i) + 1] = (float)(-std::sin(az));
            }
            real_dft(C.nph, P.Mc, P.iF);
            legendre_maps(C.L, C.x, C.wx, P.x, P.iA);
            real_synthesis(P.Mc, P.nph, P.iG);
            real_dft(P.nph, P.Mc, P.aF);
            legendre_maps(C.L, P.x, P.wx, C.x, P.aB);
            real_synthesis(P.Mc, C.nph, P.aG);
        }
    } catch (const std::bad_alloc &) {
        return fail(MLFMA_ENOMEM, "precompute: out of host memory");
    }
    return MLFMA_OK;
}

}  // namespace mlfma
