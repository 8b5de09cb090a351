// Important-term truncation of a Wick-term table (Sec. 5, "distributions of
// terms in determinants and blocks", and App. D).
//
// The paper finds that the values of the deduplicated terms, summed over the
// volume at a time slice, are concentrated near zero with a thin tail of large
// contributions; the correlator is carried by the tail, and which terms form it
// depends on the operator rather than on the ensemble, so it can be fixed once
// on a small calibration lattice and the full computation then uses only
// those terms with the same kernels.
//
// Selection (documented in the header):
//   v_n(s)  = coef_n * prod_a Bcal[s][kidx_{a,n}]          (calibration slice s)
//   m_s     = max_n |v_n(s)|
//   score_n = max over s with m_s > 0 of |v_n(s)| / m_s     (0 if no such s)
//   M       = clamp(ceil(keep * N - 1e-6), 1, N)
//   keep the M largest scores, equal scores in table order; kept terms stay
//   in table order, so the kept table is a sub-table of the input one.
// |v| is formed as |coef| * prod |B| (the magnitude of the complex product).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "internal.hpp"

namespace wick {
namespace {

constexpr int64_t kChunk = 1 << 16;  // terms per work unit (fixed: results do not depend on threads)

template <class F>
void for_chunks(int64_t n_chunks, F &&body)
{
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (n_chunks <= 1 || nth == 1) {
        for (int64_t c = 0; c < n_chunks; ++c) body(c);
        return;
    }
    std::vector<std::thread> th;
    std::atomic<int64_t> next{0};
    for (unsigned t = 0; t < std::min<int64_t>(nth, n_chunks); ++t)
        th.emplace_back([&]() {
            for (int64_t c; (c = next.fetch_add(1)) < n_chunks;) body(c);
        });
    for (auto &t : th) t.join();
}

}  // namespace

int64_t truncation_count(int64_t n_terms, double keep)
{
    if (n_terms <= 0) return 0;
    double m = std::ceil(keep * (double)n_terms - 1e-6);
    if (m < 1.0) m = 1.0;
    if (m > (double)n_terms) m = (double)n_terms;
    return (int64_t)m;
}

wick_status truncate_plan(const wick_plan_s *p, const double *B_cal, int32_t n_slices, double keep,
                          wick_plan_t *out, double *dropped)
{
    if (!p || !B_cal || !out) return fail(WICK_EINVAL, "wick_plan_truncate: null argument");
    *out = nullptr;
    if (n_slices < 1) return fail(WICK_EINVAL, "wick_plan_truncate: n_slices must be >= 1");
    if (!(keep > 0.0 && keep <= 1.0)) return fail(WICK_EINVAL, "wick_plan_truncate: keep_fraction must lie in (0, 1]");
    const int A = p->A;
    const int64_t N = p->n_terms;
    const size_t L = p->kinds.size() * (size_t)kBlockLen;
    const int64_t M = truncation_count(N, keep);
    const int64_t n_chunks = (N + kChunk - 1) / kChunk;

    // |B| per slice and entry
    std::vector<double> mag((size_t)n_slices * L);
    for (size_t e = 0; e < mag.size(); ++e) {
        mag[e] = std::hypot(B_cal[2 * e], B_cal[2 * e + 1]);
        if (!std::isfinite(mag[e])) return fail(WICK_EINVAL, "wick_plan_truncate: non-finite calibration blocks");
    }
    std::vector<double> cmag((size_t)N);
    for (int64_t n = 0; n < N; ++n) cmag[n] = std::hypot(p->coef_re[n], p->coef_im[n]);
    auto term_mag = [&](int64_t n, int s) {
        const double *ms = mag.data() + (size_t)s * L;
        double v = cmag[n];
        for (int a = 0; a < A; ++a) v *= ms[p->kidx[(size_t)a * N + n]];
        return v;
    };

    // 1. per-slice maxima
    std::vector<double> cmax((size_t)n_chunks * n_slices, 0.0);
    for_chunks(n_chunks, [&](int64_t c) {
        const int64_t lo = c * kChunk, hi = std::min(N, lo + kChunk);
        double *mx = cmax.data() + (size_t)c * n_slices;
        for (int64_t n = lo; n < hi; ++n)
            for (int s = 0; s < n_slices; ++s) mx[s] = std::max(mx[s], term_mag(n, s));
    });
    std::vector<double> inv(n_slices, 0.0);
    for (int s = 0; s < n_slices; ++s) {
        double m = 0.0;
        for (int64_t c = 0; c < n_chunks; ++c) m = std::max(m, cmax[(size_t)c * n_slices + s]);
        if (!std::isfinite(m))
            return fail(WICK_EINVAL, "wick_plan_truncate: a term overflows on the calibration blocks (rescale them)");
        inv[s] = m > 0.0 ? 1.0 / m : 0.0;
    }

    // 2. scores
    std::vector<double> score((size_t)N);
    for_chunks(n_chunks, [&](int64_t c) {
        const int64_t lo = c * kChunk, hi = std::min(N, lo + kChunk);
        for (int64_t n = lo; n < hi; ++n) {
            double sc = 0.0;
            for (int s = 0; s < n_slices; ++s)
                if (inv[s] > 0.0) sc = std::max(sc, term_mag(n, s) * inv[s]);
            score[n] = sc;
        }
    });

    // 3. the M-th largest score; every larger one is kept, equal ones in table order
    std::vector<uint8_t> kept((size_t)N, 0);
    if (M > 0) {
        std::vector<double> tmp(score);
        std::nth_element(tmp.begin(), tmp.begin() + (M - 1), tmp.end(), std::greater<double>());
        const double tau = tmp[M - 1];
        std::vector<double>().swap(tmp);
        int64_t k = 0;
        for (int64_t n = 0; n < N; ++n)
            if (score[n] > tau) { kept[n] = 1; ++k; }
        for (int64_t n = 0; n < N && k < M; ++n)
            if (score[n] == tau) { kept[n] = 1; ++k; }
    }

    // 4. sum of |v| over the dropped terms per slice (chunk partials added in chunk order)
    if (dropped) {
        std::vector<double> part((size_t)n_chunks * n_slices, 0.0);
        for_chunks(n_chunks, [&](int64_t c) {
            const int64_t lo = c * kChunk, hi = std::min(N, lo + kChunk);
            double *ps = part.data() + (size_t)c * n_slices;
            for (int64_t n = lo; n < hi; ++n)
                if (!kept[n])
                    for (int s = 0; s < n_slices; ++s) ps[s] += term_mag(n, s);
        });
        for (int s = 0; s < n_slices; ++s) {
            double t = 0.0;
            for (int64_t c = 0; c < n_chunks; ++c) t += part[(size_t)c * n_slices + s];
            dropped[s] = t;
        }
    }

    // 5. the kept sub-table, in table order
    auto q = new wick_plan_s();
    q->A = A;
    q->kinds = p->kinds;
    q->n_enumerated = p->n_enumerated;
    q->n_groups = p->n_groups;
    q->bound = p->bound;
    q->scale = p->scale;
    q->n_terms = M;
    try {
        q->kidx.resize((size_t)A * M);
        q->coef_re.resize(M);
        q->coef_im.resize(M);
    } catch (const std::bad_alloc &) {
        delete q;
        return fail(WICK_ENOMEM, "wick_plan_truncate: out of host memory");
    }
    bool real = true;
    int64_t o = 0;
    for (int64_t n = 0; n < N; ++n) {
        if (!kept[n]) continue;
        for (int a = 0; a < A; ++a) q->kidx[(size_t)a * M + o] = p->kidx[(size_t)a * N + n];
        q->coef_re[o] = p->coef_re[n];
        q->coef_im[o] = p->coef_im[n];
        if (p->coef_im[n] != 0.0) real = false;
        ++o;
    }
    q->coef_real = real;
    factor_kinds(q);
    *out = q;
    return WICK_OK;
}

}  // namespace wick
