// Built-in nuclear operators (Sec. 3.3) as exact integer weights.
//
// Basis: gamma_k = [[0, -i sigma_k], [i sigma_k, 0]], gamma_4 = diag(-1,-1,1,1),
// gamma_5 = gamma_1 gamma_2 gamma_3 gamma_4, C = gamma_4 gamma_2 (Sec. 2). In
// it C gamma_5 and P_pm = (1 pm gamma_4)/2 are integer matrices. Spin-color
// index chi = 3*spin + color.
//
// Nucleon kind (Eqs. 2.2-2.3, projected forms of Sec. 3.3): the proton
// p_alpha = eps_abc u^a_alpha u^b_beta (C g5 Q)_{beta eta} d^c_eta, quark
// slots listed as (u^a_alpha, d^c_eta, u^b_beta); the neutron swaps u and d.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <string>

#include "internal.hpp"

namespace wick {
namespace {

using cx = std::complex<int>;
using M4 = std::array<std::array<cx, 4>, 4>;

M4 mat_mul(const M4 &a, const M4 &b)
{
    M4 r{};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            for (int k = 0; k < 4; ++k) r[i][j] += a[i][k] * b[k][j];
    return r;
}

struct Basis {
    M4 g[5];  // g[0..3] = gamma_1..gamma_4, g[4] = gamma_5
    M4 cg5, pp, pm, one;
    Basis()
    {
        const cx I(0, 1), O(0, 0), L(1, 0);
        // Pauli matrices
        cx s[3][2][2] = {{{O, L}, {L, O}}, {{O, -I}, {I, O}}, {{L, O}, {O, -L}}};
        for (int k = 0; k < 3; ++k) {
            M4 m{};
            for (int i = 0; i < 2; ++i)
                for (int j = 0; j < 2; ++j) {
                    m[i][2 + j] = -I * s[k][i][j];
                    m[2 + i][j] = I * s[k][i][j];
                }
            g[k] = m;
        }
        M4 g4{};
        g4[0][0] = g4[1][1] = cx(-1, 0);
        g4[2][2] = g4[3][3] = cx(1, 0);
        g[3] = g4;
        g[4] = mat_mul(mat_mul(mat_mul(g[0], g[1]), g[2]), g[3]);
        M4 C = mat_mul(g[3], g[1]);
        cg5 = mat_mul(C, g[4]);
        one = M4{};
        for (int i = 0; i < 4; ++i) one[i][i] = L;
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                // (1 +- gamma_4)/2: gamma_4 is diagonal with entries -1, 1 here
                cx v = one[i][j];
                pp[i][j] = (v + g4[i][j]) / 2;
                pm[i][j] = (v - g4[i][j]) / 2;
            }
    }
};

const Basis &basis()
{
    static Basis b;
    return b;
}

int eps3(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    int inv = (a > b) + (a > c) + (b > c);
    return (inv & 1) ? -1 : 1;
}

struct OwnedKind {
    int flav[3];
    std::vector<int8_t> j;
    std::vector<int64_t> re, im;
};

// proj: 0 = C g5, +1 = C g5 P_+, -1 = C g5 P_-; ntype: 'p' (u,d,u) or 'n' (d,u,d)
OwnedKind nucleon(char ntype, int proj, int alpha)
{
    const Basis &B = basis();
    M4 M = proj == 0 ? B.cg5 : mat_mul(B.cg5, proj > 0 ? B.pp : B.pm);
    OwnedKind k;
    int f = ntype == 'p' ? 0 : 1;
    k.flav[0] = f; k.flav[1] = 1 - f; k.flav[2] = f;
    for (int c1 = 0; c1 < 3; ++c1)
        for (int s2 = 0; s2 < 4; ++s2)
            for (int c2 = 0; c2 < 3; ++c2)
                for (int s3 = 0; s3 < 4; ++s3)
                    for (int c3 = 0; c3 < 3; ++c3) {
                        cx v = M[s3][s2] * eps3(c1, c3, c2);
                        if (v == cx(0, 0)) continue;
                        k.j.push_back((int8_t)(3 * alpha + c1));
                        k.j.push_back((int8_t)(3 * s2 + c2));
                        k.j.push_back((int8_t)(3 * s3 + c3));
                        k.re.push_back(v.real());
                        k.im.push_back(v.imag());
                    }
    return k;
}

struct OpBuilder {
    std::vector<OwnedKind> kinds;
    std::vector<std::string> keys;
    std::vector<int32_t> pk;
    std::vector<int64_t> re, im;
    int A = 0;
    double scale = 1.0;

    int kind(char t, int proj, int alpha)
    {
        std::string key = std::string(1, t) + std::to_string(proj) + ":" + std::to_string(alpha);
        for (size_t i = 0; i < keys.size(); ++i)
            if (keys[i] == key) return (int)i;
        keys.push_back(key);
        kinds.push_back(nucleon(t, proj, alpha));
        return (int)kinds.size() - 1;
    }
    void pattern(std::initializer_list<int> ks, int64_t c)
    {
        for (int k : ks) pk.push_back(k);
        re.push_back(c);
        im.push_back(0);
    }
    std::vector<wick_kind> wk;
    // The operator as a wick_nucleus_desc (valid while the builder lives and is unchanged).
    wick_nucleus_desc desc()
    {
        wk.assign(kinds.size(), wick_kind{});
        for (size_t i = 0; i < kinds.size(); ++i) {
            for (int s = 0; s < 3; ++s) wk[i].flavor[s] = kinds[i].flav[s];
            wk[i].n_w = (int32_t)kinds[i].re.size();
            wk[i].j = kinds[i].j.data();
            wk[i].w_re = kinds[i].re.data();
            wk[i].w_im = kinds[i].im.data();
        }
        wick_nucleus_desc d{};
        d.A = A;
        d.n_kinds = (int32_t)wk.size();
        d.kinds = wk.data();
        d.n_snk = d.n_src = (int32_t)re.size();
        d.snk_kind = d.src_kind = pk.data();
        d.snk_re = d.src_re = re.data();
        d.snk_im = d.src_im = im.data();
        d.scale = scale;
        return d;
    }
};

int cg5_int(int a, int b) { return basis().cg5[a][b].real(); }

}  // namespace

namespace {

wick_status std_operator(const char *name, int32_t J, OpBuilder &ob)
{
    if (!name) return fail(WICK_EINVAL, "wick_plan_std: null argument");
    std::string n(name);
    if (n == "1H") {
        if (J < 0 || J > 3) return fail(WICK_EINVAL, "wick_plan_std: J must be 0..3");
        ob.A = 1;
        ob.pattern({ob.kind('p', 0, J)}, 1);
    } else if (n == "2H" || n == "2H-" || n == "2H0") {
        // O_2H = n^T (C g5 P_+) p, unprojected nucleons; "2H-" has P_- and "2H0"
        // no projector (the same block kinds: a basis for a correlation matrix)
        ob.A = 2;
        M4 M = n == "2H0" ? basis().cg5 : mat_mul(basis().cg5, n == "2H" ? basis().pp : basis().pm);
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a)
                if (M[b][a] != cx(0, 0)) ob.pattern({ob.kind('n', 0, b), ob.kind('p', 0, a)}, M[b][a].real());
    } else if (n == "3He" || n == "3H") {
        // O_3He = p_-^T (C g5) n_+ p_+^J; the 3H cluster mirrors it
        if (J < 0 || J > 3) return fail(WICK_EINVAL, "wick_plan_std: J must be 0..3");
        char x = n == "3He" ? 'p' : 'n', y = n == "3He" ? 'n' : 'p';
        ob.A = 3;
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                if (cg5_int(a, b)) ob.pattern({ob.kind(x, -1, a), ob.kind(y, +1, b), ob.kind(x, +1, J)}, cg5_int(a, b));
    } else if (n == "4He") {
        // (chibar eta - chi etabar)/sqrt(2); chi, chibar times 2 and sqrt(12);
        // unprojected nucleons, spin up = 0, down = 1; scale 1/96.
        ob.A = 4;
        ob.scale = 1.0 / 96.0;
        const char *cfg[6] = {"udud", "dudu", "uddu", "duud", "uudd", "dduu"};
        const int chi[6] = {1, 1, -1, -1, 0, 0};
        const int chib[6] = {1, 1, 1, 1, -2, -2};
        for (int s = 0; s < 6; ++s)
            for (int i = 0; i < 6; ++i) {
                int c = chib[s] * chi[i] - chi[s] * chib[i];
                if (!c) continue;
                int k[4];
                for (int a = 0; a < 4; ++a) k[a] = ob.kind(cfg[i][a] == 'u' ? 'p' : 'n', 0, cfg[s][a] == 'u' ? 0 : 1);
                ob.pattern({k[0], k[1], k[2], k[3]}, c);
            }
    } else {
        return fail(WICK_EINVAL, "wick_plan_std: unknown nucleus '" + n + "' (1H, 2H, 2H-, 2H0, 3He, 3H, 4He)");
    }
    return WICK_OK;
}

}  // namespace

wick_status std_plan(const char *name, int32_t J, wick_plan_t *out)
{
    if (!out) return fail(WICK_EINVAL, "wick_plan_std: null argument");
    OpBuilder ob;
    wick_status st = std_operator(name, J, ob);
    if (st != WICK_OK) return st;
    const wick_nucleus_desc d = ob.desc();
    return build_plan(&d, out);
}

wick_status std_point_plan(const char *name, int32_t J, wick_point_t *out)
{
    if (!out) return fail(WICK_EINVAL, "wick_point_plan_std: null argument");
    OpBuilder ob;
    wick_status st = std_operator(name, J, ob);
    if (st != WICK_OK) return st;
    const wick_nucleus_desc d = ob.desc();
    return build_point_plan(&d, out);
}

wick_status std_pair_plan(const char *snk, int32_t J_snk, const char *src, int32_t J_src, wick_plan_t *out)
{
    if (!out) return fail(WICK_EINVAL, "wick_plan_std_pair: null argument");
    OpBuilder a, b;
    wick_status st = std_operator(snk, J_snk, a);
    if (st != WICK_OK) return st;
    if ((st = std_operator(src, J_src, b)) != WICK_OK) return st;
    if (a.A != b.A) return fail(WICK_EINVAL, "wick_plan_std_pair: the operators differ in A");
    // the source's kinds joined to the sink's (kinds are keyed by type, projector and spin)
    std::vector<int32_t> src_kind;
    std::vector<int> bmap;
    for (size_t i = 0; i < b.kinds.size(); ++i) {
        auto it = std::find(a.keys.begin(), a.keys.end(), b.keys[i]);
        if (it == a.keys.end()) {
            a.keys.push_back(b.keys[i]);
            a.kinds.push_back(b.kinds[i]);
            bmap.push_back((int)a.kinds.size() - 1);
        } else {
            bmap.push_back((int)(it - a.keys.begin()));
        }
    }
    for (int32_t k : b.pk) src_kind.push_back(bmap[k]);
    wick_nucleus_desc d = a.desc();
    d.n_src = (int32_t)b.re.size();
    d.src_kind = src_kind.data();
    d.src_re = b.re.data();
    d.src_im = b.im.data();
    d.scale = std::sqrt(a.scale * b.scale);
    return build_plan(&d, out);
}

wick_status std_gevp_plan(const char *const *names, const int32_t *J, int32_t n_ops, wick_gevp_t *out)
{
    if (!names || !out || n_ops < 1 || n_ops > 4) return fail(WICK_EINVAL, "wick_gevp_plan_std: bad arguments");
    std::vector<OpBuilder> obs((size_t)n_ops);
    std::vector<wick_nucleus_desc> ds((size_t)n_ops);
    for (int i = 0; i < n_ops; ++i) {
        wick_status st = std_operator(names[i], J ? J[i] : 0, obs[i]);
        if (st != WICK_OK) return st;
    }
    for (int i = 0; i < n_ops; ++i) ds[i] = obs[i].desc();
    return build_gevp(ds.data(), n_ops, out);
}

}  // namespace wick
