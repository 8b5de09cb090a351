// Point-sink planner for the determinant method (Sec. 3.1 Eq. 2.9; the
// improved method B of Sec. 3.3; the minimal sets zeta_u, zeta_d and weights
// Theta of App. A Eq. A1).
//
// 1. Antisymmetrise the sink and the source coefficient tensors per flavor:
//    every index tuple of an operator pattern (a product of kind weights) is
//    reordered to (u indices ascending, then d indices ascending); the sign
//    of that reordering of quark positions (which holds the flavor-grouping
//    sign eta of Eq. 2.8) multiplies the pattern coefficient and the weights.
//    Tuples that repeat an index within a flavor vanish (Pauli). Equal
//    (U, D) lists add up exactly (Gaussian integers); zero groups are dropped.
//    Reordering the rows (columns) of a determinant multiplies it by the sign
//    of that reordering (redundancy R.1 of Sec. 3.2), which is what the sign
//    carries.
// 2. The determinants needed at a site are det S_f[R; K] for every sink row
//    set R and source column set K of each flavor. A given (R, K) appears in
//    many (sink group, source group) pairs (redundancy R.2) and is computed
//    once per site. Two different (R, K) of one flavor are different
//    polynomials of the propagator entries (their monomials have different
//    supports), so no randomised identity test can merge them further: the
//    distinct pairs are the minimal set.
// 3. Tables: sink groups sorted by (row set of u, row set of d) with range
//    starts per u row set; source column sets as colex ranks of k-subsets of
//    {0..11} (rank = sum_i binom(c_i, i + 1) for c_0 < c_1 < ...).
#include <algorithm>
#include <cstring>
#include <map>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace wick {
namespace {

constexpr int kMaxPointQuarks = 6;  // per flavor: binom(12, 6) = 924 minors per row set

struct Acc {
    __int128 re = 0, im = 0;
};

int64_t binom(int n, int k)
{
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 0; i < k; ++i) r = r * (n - i) / (i + 1);
    return r;
}

// Antisymmetrise one side of the operator; key = (u list, d list) packed in
// 4-bit fields (u first). Returns the flavor counts through nu, nd.
wick_status antisymmetrise(const wick_nucleus_desc *d, bool sink, int *nu_out, int *nd_out,
                           std::map<uint64_t, Acc> &groups)
{
    const int A = d->A;
    const int n_pat = sink ? d->n_snk : d->n_src;
    const int32_t *pk = sink ? d->snk_kind : d->src_kind;
    const int64_t *cre = sink ? d->snk_re : d->src_re;
    const int64_t *cim = sink ? d->snk_im : d->src_im;
    const char *side = sink ? "sink" : "source";
    int nu = -1, nd = -1;
    for (int p = 0; p < n_pat; ++p) {
        const int32_t *ks = pk + (size_t)p * A;
        int fl[3 * kMaxA];
        int64_t count = 1;
        for (int a = 0; a < A; ++a) {
            if (ks[a] < 0 || ks[a] >= d->n_kinds) return fail(WICK_EINVAL, std::string("wick_point_plan: bad kind in ") + side);
            const wick_kind &k = d->kinds[ks[a]];
            for (int s = 0; s < 3; ++s) fl[3 * a + s] = k.flavor[s];
            count *= k.n_w;
        }
        int cu = 0, cd = 0;
        for (int q = 0; q < 3 * A; ++q) {
            if (fl[q] != 0 && fl[q] != 1) return fail(WICK_EINVAL, "wick_point_plan: flavors must be 0 (u) or 1 (d)");
            (fl[q] == 0 ? cu : cd)++;
        }
        if (nu < 0) { nu = cu; nd = cd; }
        if (cu != nu || cd != nd) return fail(WICK_EINVAL, std::string("wick_point_plan: ") + side + " patterns differ in flavor content");
        if (cre[p] == 0 && cim[p] == 0) continue;
        std::vector<int> ctr(A, 0);
        for (int64_t t = 0; t < count; ++t) {
            int idx[3 * kMaxA];
            __int128 wr = cre[p], wi = cim[p];
            for (int a = 0; a < A; ++a) {
                const wick_kind &k = d->kinds[ks[a]];
                const int e = ctr[a];
                for (int s = 0; s < 3; ++s) idx[3 * a + s] = k.j[3 * e + s];
                const __int128 xr = k.w_re[e], xi = k.w_im[e];
                const __int128 nr = wr * xr - wi * xi, ni = wr * xi + wi * xr;
                wr = nr;
                wi = ni;
            }
            for (int a = A - 1; a >= 0; --a) {
                if (++ctr[a] < d->kinds[ks[a]].n_w) break;
                ctr[a] = 0;
            }
            // canonical position of every quark; parity of the position map
            int pos[3 * kMaxA];
            bool pauli = false;
            for (int q = 0; q < 3 * A && !pauli; ++q) {
                int rank = 0;
                for (int r = 0; r < 3 * A; ++r) {
                    if (r == q || fl[r] != fl[q]) continue;
                    if (idx[r] == idx[q]) { pauli = true; break; }
                    rank += idx[r] < idx[q];
                }
                pos[q] = (fl[q] == 0 ? 0 : nu) + rank;
            }
            if (pauli) continue;
            int canon[3 * kMaxA], inv = 0;
            for (int q = 0; q < 3 * A; ++q) canon[pos[q]] = idx[q];
            for (int q = 0; q < 3 * A; ++q)
                for (int r = q + 1; r < 3 * A; ++r) inv += pos[q] > pos[r];
            uint64_t key = 0;
            for (int q = 0; q < 3 * A; ++q) key = (key << 4) | (uint64_t)canon[q];
            Acc &g = groups[key];
            if (inv & 1) { g.re -= wr; g.im -= wi; }
            else { g.re += wr; g.im += wi; }
        }
    }
    for (auto it = groups.begin(); it != groups.end();) {
        if (it->second.re == 0 && it->second.im == 0) it = groups.erase(it);
        else ++it;
    }
    *nu_out = nu < 0 ? 0 : nu;
    *nd_out = nd < 0 ? 0 : nd;
    return WICK_OK;
}

void unpack(uint64_t key, int n, int *v)
{
    for (int q = n - 1; q >= 0; --q) { v[q] = (int)(key & 15); key >>= 4; }
}

int colex_rank(const int *c, int k)
{
    int r = 0;
    for (int i = 0; i < k; ++i) r += (int)binom(c[i], i + 1);
    return r;
}

}  // namespace

wick_status build_point_plan(const wick_nucleus_desc *d, wick_point_t *out)
{
    if (!d || !out) return fail(WICK_EINVAL, "wick_point_plan: null argument");
    *out = nullptr;
    if (d->A < 1 || d->A > kMaxA) return fail(WICK_EINVAL, "wick_point_plan: A must be 1..5");
    if (d->n_kinds < 1 || !d->kinds) return fail(WICK_EINVAL, "wick_point_plan: no kinds");
    if (d->n_snk < 1 || d->n_src < 1 || !d->snk_kind || !d->src_kind || !d->snk_re || !d->snk_im ||
        !d->src_re || !d->src_im)
        return fail(WICK_EINVAL, "wick_point_plan: missing patterns");
    for (int k = 0; k < d->n_kinds; ++k) {
        const wick_kind &kd = d->kinds[k];
        if (kd.n_w < 0 || kd.n_w > 1728 || (kd.n_w > 0 && (!kd.j || !kd.w_re || !kd.w_im)))
            return fail(WICK_EINVAL, "wick_point_plan: bad kind weights");
        for (int e = 0; e < 3 * kd.n_w; ++e)
            if (kd.j[e] < 0 || kd.j[e] >= 12) return fail(WICK_EINVAL, "wick_point_plan: index outside [0, 12)");
    }
    std::map<uint64_t, Acc> snk, src;
    int nu, nd, nu2, nd2;
    wick_status st = antisymmetrise(d, true, &nu, &nd, snk);
    if (st != WICK_OK) return st;
    st = antisymmetrise(d, false, &nu2, &nd2, src);
    if (st != WICK_OK) return st;
    if (nu != nu2 || nd != nd2) return fail(WICK_EINVAL, "wick_point_plan: sink and source differ in flavor content");
    if (nu > kMaxPointQuarks || nd > kMaxPointQuarks)
        return fail(WICK_EUNSUPPORTED, "wick_point_plan: more than 6 quarks of one flavor");
    const __int128 lim = ((__int128)1) << 52;
    for (auto *m : {&snk, &src})
        for (auto &g : *m)
            if (g.second.re > lim || g.second.re < -lim || g.second.im > lim || g.second.im < -lim)
                return fail(WICK_ETOOBIG, "wick_point_plan: antisymmetrised weight above 2^52");

    auto p = new wick_point_s();
    p->n_u = nu;
    p->n_d = nd;
    p->scale = d->scale;
    // distinct sink row sets (map keys are sorted, so u lists come out in order)
    std::map<uint64_t, int> ru, rd;
    const int n = nu + nd;
    for (auto &g : snk) {
        int v[16];
        unpack(g.first, n, v);
        uint64_t ku = 0, kd = 0;
        for (int q = 0; q < nu; ++q) ku = (ku << 4) | (uint64_t)v[q];
        for (int q = 0; q < nd; ++q) kd = (kd << 4) | (uint64_t)v[nu + q];
        ru.emplace(ku, 0);
        rd.emplace(kd, 0);
    }
    for (auto *m : {&ru, &rd}) {
        int i = 0;
        for (auto &e : *m) e.second = i++;
    }
    auto rows_of = [](const std::map<uint64_t, int> &m, int k, std::vector<std::array<int8_t, 8>> &out) {
        out.assign(m.size(), {});
        for (auto &e : m) {
            int v[16];
            unpack(e.first, k, v);
            for (int q = 0; q < k; ++q) out[e.second][q] = (int8_t)v[q];
        }
    };
    rows_of(ru, nu, p->rows_u);
    rows_of(rd, nd, p->rows_d);
    // sink groups in (u row set, d row set) order: the map key order is exactly that
    p->u_beg.assign(p->rows_u.size() + 1, 0);
    for (auto &g : snk) {
        int v[16];
        unpack(g.first, n, v);
        uint64_t ku = 0, kd = 0;
        for (int q = 0; q < nu; ++q) ku = (ku << 4) | (uint64_t)v[q];
        for (int q = 0; q < nd; ++q) kd = (kd << 4) | (uint64_t)v[nu + q];
        const int iu = ru[ku];
        p->g_u.push_back(iu);
        p->g_d.push_back(rd[kd]);
        p->g_w.push_back((double)g.second.re);
        p->g_w.push_back((double)g.second.im);
        p->u_beg[iu + 1]++;
    }
    for (size_t i = 1; i < p->u_beg.size(); ++i) p->u_beg[i] += p->u_beg[i - 1];
    // source groups: column sets as colex ranks
    std::map<int, int> cu, cd;
    for (auto &h : src) {
        int v[16];
        unpack(h.first, n, v);
        const int r_u = colex_rank(v, nu), r_d = colex_rank(v + nu, nd);
        p->h_ru.push_back((uint16_t)r_u);
        p->h_rd.push_back((uint16_t)r_d);
        p->h_w.push_back((double)h.second.re);
        p->h_w.push_back((double)h.second.im);
        cu[r_u] = 1;
        cd[r_d] = 1;
    }
    p->n_cols_u = (int64_t)cu.size();
    p->n_cols_d = (int64_t)cd.size();
    *out = p;
    return WICK_OK;
}

}  // namespace wick

using namespace wick;

wick_point_s::~wick_point_s() { release_point_tables(this); }

extern "C" {

wick_status wick_point_plan(const wick_nucleus_desc *desc, wick_point_t *out)
{
    try {
        return build_point_plan(desc, out);
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_point_plan: out of host memory");
    } catch (...) {
        return fail(WICK_EINVAL, "wick_point_plan: internal error");
    }
}

wick_status wick_point_plan_std(const char *nucleus, int32_t J, wick_point_t *out)
{
    try {
        return std_point_plan(nucleus, J, out);
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_point_plan_std: out of host memory");
    } catch (...) {
        return fail(WICK_EINVAL, "wick_point_plan_std: internal error");
    }
}

wick_status wick_point_info(wick_point_t p, int32_t *n_u, int32_t *n_d, int64_t *n_sink_groups, int64_t *n_src_groups,
                            int64_t *n_rows_u, int64_t *n_cols_u, int64_t *n_rows_d, int64_t *n_cols_d)
{
    if (!p) return fail(WICK_EINVAL, "wick_point_info: null plan");
    if (n_u) *n_u = p->n_u;
    if (n_d) *n_d = p->n_d;
    if (n_sink_groups) *n_sink_groups = (int64_t)p->g_u.size();
    if (n_src_groups) *n_src_groups = (int64_t)p->h_ru.size();
    if (n_rows_u) *n_rows_u = (int64_t)p->rows_u.size();
    if (n_cols_u) *n_cols_u = p->n_cols_u;
    if (n_rows_d) *n_rows_d = (int64_t)p->rows_d.size();
    if (n_cols_d) *n_cols_d = p->n_cols_d;
    return WICK_OK;
}

void wick_point_destroy(wick_point_t p) { delete p; }

}  // extern "C"
