// Correlation matrices for the generalized eigenvalue problem (Sec. "Application
// of the proposed algorithms to the GEVP", Eqs. E1-E3): C_ij(t) with operator
// O_i at the sink and O_j at the source, for a basis of N operators.
//
// Every element is planned like a single correlator (the deduplicated table of
// Sec. 3.2 / App. C, merged exactly in F_p). All elements share the
// propagators, hence the blocks, so the element tables are then united: a term
// of the union is one block-entry monomial (its sorted (kind, index) tuple in a
// common kind numbering) with a coefficient for every element in which it
// occurs. The GPU evaluates each monomial once per time slice and adds it to
// every element (the cross-element common sub-expressions of Eq. E3).
//
// Readings: the operators share A and flavor content; element (i, j) carries
// the normalisation sqrt(scale_i * scale_j) (each scale is the square of an
// operator normalisation, e.g. 1/96 for the helium-4 operator).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

namespace wick {
namespace {

constexpr int kMaxGevpOps = 4;  // N x N <= 16 elements

using KindKey = std::pair<std::array<int, 3>, std::vector<std::array<int64_t, 5>>>;

KindKey key_of(const KindDef &k)
{
    KindKey key;
    for (int s = 0; s < 3; ++s) key.first[s] = k.flav[s];
    for (size_t n = 0; n < k.w.size(); ++n)
        key.second.push_back({k.j[n][0], k.j[n][1], k.j[n][2], k.w[n].re, k.w[n].im});
    std::sort(key.second.begin(), key.second.end());
    return key;
}

KindDef kind_of(const wick_kind &wk)
{
    KindDef k;
    for (int s = 0; s < 3; ++s) k.flav[s] = wk.flavor[s];
    for (int n = 0; n < wk.n_w; ++n) {
        if (wk.w_re[n] == 0 && wk.w_im[n] == 0) continue;
        k.j.push_back({wk.j[3 * n], wk.j[3 * n + 1], wk.j[3 * n + 2]});
        k.w.push_back(GInt{wk.w_re[n], wk.w_im[n]});
    }
    return k;
}

struct TupleHash {
    size_t operator()(const std::array<uint16_t, kMaxA> &t) const
    {
        uint64_t h = 1469598103934665603ULL;
        for (uint16_t v : t) { h ^= v; h *= 1099511628211ULL; }
        return (size_t)h;
    }
};

}  // namespace

wick_status build_gevp(const wick_nucleus_desc *ops, int32_t n_ops, wick_gevp_t *out)
{
    if (!ops || !out) return fail(WICK_EINVAL, "wick_gevp_plan: null argument");
    *out = nullptr;
    if (n_ops < 1 || n_ops > kMaxGevpOps) return fail(WICK_EINVAL, "wick_gevp_plan: n_ops must be 1..4");
    const int A = ops[0].A;
    for (int i = 0; i < n_ops; ++i) {
        const wick_nucleus_desc &d = ops[i];
        if (d.A != A) return fail(WICK_EINVAL, "wick_gevp_plan: operators differ in A");
        if (!(d.scale > 0.0) || !std::isfinite(d.scale)) return fail(WICK_EINVAL, "wick_gevp_plan: scales must be positive");
        if (d.n_kinds < 1 || !d.kinds || d.n_snk < 1 || d.n_src < 1 || !d.snk_kind || !d.src_kind || !d.snk_re ||
            !d.snk_im || !d.src_re || !d.src_im)
            return fail(WICK_EINVAL, "wick_gevp_plan: incomplete operator");
        for (int k = 0; k < d.n_kinds; ++k)
            if (d.kinds[k].n_w < 0 || (d.kinds[k].n_w > 0 && (!d.kinds[k].j || !d.kinds[k].w_re || !d.kinds[k].w_im)))
                return fail(WICK_EINVAL, "wick_gevp_plan: bad kind weights");
        for (int q = 0; q < (d.n_snk + d.n_src) * A; ++q) {
            const int k = q < d.n_snk * A ? d.snk_kind[q] : d.src_kind[q - d.n_snk * A];
            if (k < 0 || k >= d.n_kinds) return fail(WICK_EINVAL, "wick_gevp_plan: pattern kind index out of range");
        }
    }
    // 1. union of the operators' kinds; block kinds = kinds at some sink, by first use
    std::map<KindKey, int> uk;
    std::vector<KindDef> ukinds;
    std::vector<std::vector<int>> umap(n_ops);
    for (int i = 0; i < n_ops; ++i)
        for (int k = 0; k < ops[i].n_kinds; ++k) {
            KindDef kd = kind_of(ops[i].kinds[k]);
            auto it = uk.emplace(key_of(kd), (int)ukinds.size());
            if (it.second) ukinds.push_back(kd);
            umap[i].push_back(it.first->second);
        }
    std::vector<int> block_of(ukinds.size(), -1);
    std::vector<KindDef> bkinds;
    for (int i = 0; i < n_ops; ++i)
        for (int q = 0; q < ops[i].n_snk * A; ++q) {
            const int u = umap[i][ops[i].snk_kind[q]];
            if (block_of[u] < 0) { block_of[u] = (int)bkinds.size(); bkinds.push_back(ukinds[u]); }
        }
    std::map<KindKey, int> bkey;
    for (size_t b = 0; b < bkinds.size(); ++b) bkey[key_of(bkinds[b])] = (int)b;
    if (bkinds.size() * kBlockLen > 65536) return fail(WICK_ETOOBIG, "wick_gevp_plan: too many block kinds");

    // the union kinds as a desc kind array (shared by every element desc)
    std::vector<wick_kind> wk(ukinds.size());
    std::vector<std::vector<int8_t>> wj(ukinds.size());
    std::vector<std::vector<int64_t>> wr(ukinds.size()), wi(ukinds.size());
    for (size_t u = 0; u < ukinds.size(); ++u) {
        for (size_t n = 0; n < ukinds[u].w.size(); ++n) {
            for (int s = 0; s < 3; ++s) wj[u].push_back(ukinds[u].j[n][s]);
            wr[u].push_back(ukinds[u].w[n].re);
            wi[u].push_back(ukinds[u].w[n].im);
        }
        for (int s = 0; s < 3; ++s) wk[u].flavor[s] = ukinds[u].flav[s];
        wk[u].n_w = (int32_t)ukinds[u].w.size();
        wk[u].j = wj[u].data();
        wk[u].w_re = wr[u].data();
        wk[u].w_im = wi[u].data();
    }

    // 2. every element on its own, then the union by monomial
    const int E = n_ops * n_ops;
    auto g = new wick_gevp_s();
    g->n_ops = n_ops;
    g->A = A;
    std::unordered_map<std::array<uint16_t, kMaxA>, int64_t, TupleHash> index;
    std::vector<std::array<uint16_t, kMaxA>> tuples;
    std::vector<double> coef;  // [n][E][2]
    bool real = true;
    for (int i = 0; i < n_ops; ++i)
        for (int j = 0; j < n_ops; ++j) {
            std::vector<int32_t> sk, sc;
            for (int q = 0; q < ops[i].n_snk * A; ++q) sk.push_back(umap[i][ops[i].snk_kind[q]]);
            for (int q = 0; q < ops[j].n_src * A; ++q) sc.push_back(umap[j][ops[j].src_kind[q]]);
            wick_nucleus_desc d{};
            d.A = A;
            d.n_kinds = (int32_t)wk.size();
            d.kinds = wk.data();
            d.n_snk = ops[i].n_snk;
            d.snk_kind = sk.data();
            d.snk_re = ops[i].snk_re;
            d.snk_im = ops[i].snk_im;
            d.n_src = ops[j].n_src;
            d.src_kind = sc.data();
            d.src_re = ops[j].src_re;
            d.src_im = ops[j].src_im;
            d.scale = std::sqrt(ops[i].scale * ops[j].scale);
            d.hash_seed = ops[0].hash_seed;
            d.hash_trials = ops[0].hash_trials;
            d.hash_sites = ops[0].hash_sites;
            wick_plan_t pe = nullptr;
            wick_status st = build_plan(&d, &pe);
            if (st != WICK_OK) { delete g; return st; }
            std::vector<int> kmap(pe->kinds.size());
            for (size_t k = 0; k < pe->kinds.size(); ++k) kmap[k] = bkey.at(key_of(pe->kinds[k]));
            const int e = i * n_ops + j;
            const int64_t N = pe->n_terms;
            g->n_element_terms += N;
            for (int64_t n = 0; n < N; ++n) {
                std::array<uint16_t, kMaxA> t{};
                for (int a = 0; a < A; ++a) {
                    const int v = pe->kidx[(size_t)a * N + n];
                    t[a] = (uint16_t)(kmap[v / kBlockLen] * kBlockLen + v % kBlockLen);
                }
                std::sort(t.begin(), t.begin() + A);
                auto it = index.emplace(t, (int64_t)tuples.size());
                if (it.second) {
                    tuples.push_back(t);
                    coef.resize(coef.size() + 2 * E, 0.0);
                }
                double *c = coef.data() + (size_t)it.first->second * 2 * E + 2 * e;
                c[0] += pe->coef_re[n];
                c[1] += pe->coef_im[n];
                if (pe->coef_im[n] != 0.0) real = false;
            }
            wick_plan_destroy(pe);
        }
    // 3. the union table in tuple order (gather locality)
    const int64_t N = (int64_t)tuples.size();
    std::vector<int64_t> ord(N);
    for (int64_t n = 0; n < N; ++n) ord[n] = n;
    std::sort(ord.begin(), ord.end(), [&](int64_t x, int64_t y) { return tuples[x] < tuples[y]; });
    g->n_terms = N;
    g->kidx.resize((size_t)A * N);
    g->coef.resize((size_t)N * 2 * E);
    for (int64_t n = 0; n < N; ++n) {
        for (int a = 0; a < A; ++a) g->kidx[(size_t)a * N + n] = tuples[ord[n]][a];
        std::memcpy(&g->coef[(size_t)n * 2 * E], &coef[(size_t)ord[n] * 2 * E], sizeof(double) * 2 * E);
    }
    g->coef_real = real;
    // 4. a carrier plan with the block kinds and no terms drives the block kernels
    auto c = new wick_plan_s();
    c->A = A;
    c->kinds = bkinds;
    c->scale = 1.0;
    c->n_terms = 0;
    factor_kinds(c);
    g->carrier = c;
    *out = g;
    return WICK_OK;
}

}  // namespace wick

using namespace wick;

wick_gevp_s::~wick_gevp_s()
{
    release_gevp_tables(this);
    wick_plan_destroy(carrier);  // also drops its device tables and cached batches
}

extern "C" {

wick_status wick_gevp_plan(const wick_nucleus_desc *ops, int32_t n_ops, wick_gevp_t *out)
{
    try {
        return build_gevp(ops, n_ops, out);
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_gevp_plan: out of host memory");
    } catch (const std::exception &ex) {
        return fail(WICK_EINVAL, std::string("wick_gevp_plan: internal: ") + ex.what());
    }
}

wick_status wick_gevp_plan_std(const char *const *names, const int32_t *J, int32_t n_ops, wick_gevp_t *out)
{
    try {
        return std_gevp_plan(names, J, n_ops, out);
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_gevp_plan_std: out of host memory");
    } catch (const std::exception &ex) {
        return fail(WICK_EINVAL, std::string("wick_gevp_plan_std: internal: ") + ex.what());
    }
}

wick_status wick_gevp_info(wick_gevp_t g, int32_t *n_ops, int32_t *A, int32_t *n_kinds, int64_t *n_terms,
                           int64_t *n_element_terms)
{
    if (!g) return fail(WICK_EINVAL, "wick_gevp_info: null plan");
    if (n_ops) *n_ops = g->n_ops;
    if (A) *A = g->A;
    if (n_kinds) *n_kinds = (int32_t)g->carrier->kinds.size();
    if (n_terms) *n_terms = g->n_terms;
    if (n_element_terms) *n_element_terms = g->n_element_terms;
    return WICK_OK;
}

wick_status wick_gevp_table(wick_gevp_t g, uint16_t *kidx, double *coef)
{
    if (!g) return fail(WICK_EINVAL, "wick_gevp_table: null plan");
    if (kidx) std::memcpy(kidx, g->kidx.data(), g->kidx.size() * sizeof(uint16_t));
    if (coef) std::memcpy(coef, g->coef.data(), g->coef.size() * sizeof(double));
    return WICK_OK;
}

wick_status wick_gevp_kinds(wick_gevp_t g, wick_plan_t *carrier)
{
    if (!g || !carrier) return fail(WICK_EINVAL, "wick_gevp_kinds: null argument");
    *carrier = g->carrier;
    return WICK_OK;
}

void wick_gevp_destroy(wick_gevp_t g) { delete g; }

}  // extern "C"
