/*
 * Plain O(N^2) Helmholtz potential and its gradient, FP64 (oracle; test
 * infrastructure only -- the product path never links this file).
 *
 * Definition followed: the pair-potential sum of the paper's problem
 * statement (Sec. 2, Eq. for Phi(r)), evaluated at target points, with the
 * kernel G(r) = exp(i k |r|) / |r| (the sign and 1/(4 pi) scale reading
 * recorded in the design notes; the paper's own exp(-jkr)/(4 pi r) is the
 * complex conjugate over 4 pi for real k).
 *
 *   phi[t][c]  = sum_{s : src_s != tgt_t} G(tgt_t - src_s) q[s][c]
 *   grad[t][c] = sum_{s : src_s != tgt_t} grad G(tgt_t - src_s) q[s][c],
 *   grad G(r)  = G(r) (i k - 1/|r|) r / |r|
 *
 * A source whose three coordinates equal the target's bit for bit is
 * skipped: that removes the singular self term when targets are a subset of
 * the sources, and coincident points in general.
 *
 * Layouts: coordinates [n][3] row-major; complex values interleaved
 * (re, im) doubles; q is [ns][nrhs]; phi is [nt][nrhs]; grad is
 * [nt][nrhs][3].  OpenMP over targets; each target's sum runs over sources
 * in index order.
 */
#include <math.h>
#include <stdint.h>

static int same_point(const double *a, const double *b)
{
    return a[0] == b[0] && a[1] == b[1] && a[2] == b[2];
}

void oracle_dense_potential(int64_t ns, const double *src, const double *q,
                            int64_t nt, const double *tgt, int64_t nrhs,
                            double k, double *phi)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const double *rt = tgt + 3 * t;
        double *out = phi + 2 * nrhs * t;
        for (int64_t c = 0; c < 2 * nrhs; ++c) out[c] = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            const double *rs = src + 3 * s;
            if (same_point(rt, rs)) continue;
            double dx = rt[0] - rs[0], dy = rt[1] - rs[1], dz = rt[2] - rs[2];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double gre = cos(k * r) / r, gim = sin(k * r) / r;
            const double *qs = q + 2 * nrhs * s;
            for (int64_t c = 0; c < nrhs; ++c) {
                double qre = qs[2 * c], qim = qs[2 * c + 1];
                out[2 * c] += gre * qre - gim * qim;
                out[2 * c + 1] += gre * qim + gim * qre;
            }
        }
    }
}

void oracle_dense_field(int64_t ns, const double *src, const double *q,
                        int64_t nt, const double *tgt, int64_t nrhs,
                        double k, double *grad)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < nt; ++t) {
        const double *rt = tgt + 3 * t;
        double *out = grad + 6 * nrhs * t;
        for (int64_t c = 0; c < 6 * nrhs; ++c) out[c] = 0.0;
        for (int64_t s = 0; s < ns; ++s) {
            const double *rs = src + 3 * s;
            if (same_point(rt, rs)) continue;
            double d[3] = {rt[0] - rs[0], rt[1] - rs[1], rt[2] - rs[2]};
            double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            double gre = cos(k * r) / r, gim = sin(k * r) / r;
            /* G (i k - 1/r) / r : (gre + i gim)(-1/r + i k) / r */
            double fre = (-gre / r - gim * k) / r;
            double fim = (gre * k - gim / r) / r;
            const double *qs = q + 2 * nrhs * s;
            for (int64_t c = 0; c < nrhs; ++c) {
                double qre = qs[2 * c], qim = qs[2 * c + 1];
                double pre = fre * qre - fim * qim;
                double pim = fre * qim + fim * qre;
                for (int a = 0; a < 3; ++a) {
                    out[6 * c + 2 * a] += pre * d[a];
                    out[6 * c + 2 * a + 1] += pim * d[a];
                }
            }
        }
    }
}
