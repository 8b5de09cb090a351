// Host planner: nuclear operator -> deduplicated table of Wick terms.
//
// Steps (Sec. 3.2, "computation of non-redundant minimal set"; App. C):
//  1. Antisymmetrise the source per flavor (method A of Sec. 3.3): every
//     source index tuple with distinct same-flavor indices is mapped to its
//     sorted (U, D) lists; W'(U, D) collects the exact integer weights with
//     the sign of the sorting permutation and the flavor-grouping sign eta of
//     Eq. 2.8. Repeated same-flavor indices cancel (Pauli).
//  2. For each (U, D) group and sink pattern, enumerate every assignment of
//     the sorted indices to the blocks' quark slots with its sign (the sum
//     over sigma in Eq. 2.6 / App. D). Blocks are antisymmetric in their two
//     same-flavor slots (Eq. 2.4), so only assignments whose slot-1 index is
//     below the slot-3 index are enumerated; the other half repeats them.
//  3. Evaluate each term on random F_p propagators of a toy lattice with at
//     least A sites (exact integer arithmetic, App. C implementation note 1;
//     Schwartz-Zippel, App. C Thm. 1) and merge terms whose values agree up
//     to sign in every trial, summing integer coefficients exactly (the sign
//     rule R.1 of Sec. 3.2, lifted to block products).
//  4. Emit the table (kind*792 + compact index per block, coefficient).
//
// Merges never cross (U, D) groups: the monomials of different groups have
// different degrees in the source-column variables of S_u and S_d.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <stdexcept>
#include <thread>

#include "internal.hpp"

namespace wick {
namespace {

// ------------------------------------------------------------ F_p, p = 2^61-1
constexpr uint64_t kP = (1ULL << 61) - 1;

inline uint64_t fred(uint64_t x)
{
    x = (x & kP) + (x >> 61);
    return x >= kP ? x - kP : x;
}
inline uint64_t fadd(uint64_t a, uint64_t b) { return fred(a + b); }
inline uint64_t fsub(uint64_t a, uint64_t b) { return a >= b ? a - b : a + kP - b; }
inline uint64_t fmul(uint64_t a, uint64_t b)
{
    unsigned __int128 z = (unsigned __int128)a * b;
    return fred(((uint64_t)z & kP) + (uint64_t)(z >> 61));
}
inline uint64_t fint(int64_t v)
{
    if (v >= 0) return fred((uint64_t)v % kP);
    return fsub(0, fred((uint64_t)(-(v + 1)) % kP + 1));
}

// Field element: F_p (real weights) or F_p[i], i^2 = -1 (Gaussian weights;
// a field because p = 3 mod 4).
struct FR {
    uint64_t a = 0;
    static FR from(GInt g) { return FR{fint(g.re)}; }
    FR operator*(FR o) const { return FR{fmul(a, o.a)}; }
    FR operator+(FR o) const { return FR{fadd(a, o.a)}; }
    FR operator-(FR o) const { return FR{fsub(a, o.a)}; }
    bool zero() const { return a == 0; }
    bool negative() const { return a > (kP - 1) / 2; }
    FR neg() const { return FR{fsub(0, a)}; }
    uint64_t k0() const { return a; }
    uint64_t k1() const { return 0; }
};
struct FC {
    uint64_t a = 0, b = 0;
    static FC from(GInt g) { return FC{fint(g.re), fint(g.im)}; }
    FC operator*(FC o) const
    {
        return FC{fsub(fmul(a, o.a), fmul(b, o.b)), fadd(fmul(a, o.b), fmul(b, o.a))};
    }
    FC operator+(FC o) const { return FC{fadd(a, o.a), fadd(b, o.b)}; }
    FC operator-(FC o) const { return FC{fsub(a, o.a), fsub(b, o.b)}; }
    bool zero() const { return a == 0 && b == 0; }
    bool negative() const { return a ? a > (kP - 1) / 2 : b > (kP - 1) / 2; }
    FC neg() const { return FC{fsub(0, a), fsub(0, b)}; }
    uint64_t k0() const { return a; }
    uint64_t k1() const { return b; }
};

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// --------------------------------------------------------- Gaussian integers
struct GAcc {
    __int128 re = 0, im = 0;
    void add(GInt g, int sgn)
    {
        re += (__int128)sgn * g.re;
        im += (__int128)sgn * g.im;
    }
};
inline GInt gmul(GInt x, GInt y, bool &ovf)
{
    __int128 re = (__int128)x.re * y.re - (__int128)x.im * y.im;
    __int128 im = (__int128)x.re * y.im + (__int128)x.im * y.re;
    const __int128 lim = ((__int128)1) << 62;
    if (re > lim || re < -lim || im > lim || im < -lim) ovf = true;
    return GInt{(int64_t)re, (int64_t)im};
}

inline int pair_index(int i1, int i3) { return i3 * (i3 - 1) / 2 + i1; }  // i1 < i3

struct Pattern {
    std::array<int, kMaxA> k{};
    GInt c;
    int eta = 1;
};

// Sign of the stable sort of a flavor listing (u before d): eta of Eq. 2.8.
int listing_eta(const std::vector<int> &f)
{
    int inv = 0;
    for (size_t q = 0; q < f.size(); ++q)
        for (size_t r = q + 1; r < f.size(); ++r) inv += (f[q] == 1 && f[r] == 0);
    return (inv & 1) ? -1 : 1;
}

struct Group {
    std::array<int8_t, 16> U{}, D{};
    GInt w;
};


// Open-addressing table of the distinct monomials of one group, keyed exactly
// by the sorted (kind*792 + index) tuple of the term (equal tuples are the same
// monomial), accumulating the exact signed coefficients.
struct SynSlot {
    unsigned __int128 key;  // 0 marks an empty slot (tuples are stored + 1)
    __int128 re, im;
};
struct SynTable {
    std::vector<SynSlot> slots;
    size_t n = 0;
    void reset()
    {
        if (slots.size() != (1u << 16)) slots.assign(1u << 16, SynSlot{0, 0, 0});
        else
            for (auto &x : slots) x.key = 0;
        n = 0;
    }
    static uint64_t mix(unsigned __int128 k)
    {
        uint64_t x = (uint64_t)k ^ ((uint64_t)(k >> 64) * 0x9E3779B97F4A7C15ULL);
        x ^= x >> 31;
        x *= 0xBF58476D1CE4E5B9ULL;
        x ^= x >> 27;
        return x;
    }
    void insert(unsigned __int128 key, __int128 re, __int128 im)
    {
        const size_t mask = slots.size() - 1;
        size_t i = mix(key) & mask;
        for (;;) {
            SynSlot &x = slots[i];
            if (x.key == 0) {
                x.key = key;
                x.re = re;
                x.im = im;
                ++n;
                return;
            }
            if (x.key == key) {
                x.re += re;
                x.im += im;
                return;
            }
            i = (i + 1) & mask;
        }
    }
    void add(unsigned __int128 key, GInt c)
    {
        if (2 * (n + 1) > slots.size()) {
            std::vector<SynSlot> old(slots.size() * 2, SynSlot{0, 0, 0});
            old.swap(slots);
            n = 0;
            for (auto &x : old)
                if (x.key) insert(x.key, x.re, x.im);
        }
        insert(key, c.re, c.im);
    }
};

struct Ctx {
    int A = 0, nu = 0, nd = 0, trials = 2;
    std::vector<Pattern> snk;
    std::vector<Group> groups;
    std::vector<KindDef> *kinds = nullptr;
};

template <class F>
struct Enumerator {
    const Ctx &cx;
    const std::vector<std::vector<F>> &bh;        // [trial][kind*792 + c]
    const std::vector<uint8_t> &zero_entry;       // [kind*792 + c] identically zero
    SynTable table;
    int64_t n_enum = 0;

    // current group
    const Group *g = nullptr;
    const Pattern *pat = nullptr;
    GInt coef0;
    std::array<uint16_t, kMaxA> idx{};

    Enumerator(const Ctx &c, const std::vector<std::vector<F>> &b, const std::vector<uint8_t> &z)
        : cx(c), bh(b), zero_entry(z) {}

    int val(int flav, int p) const { return flav == 0 ? g->U[p] : g->D[p]; }

    void rec(int a, uint32_t used_u, uint32_t used_d, int inv)
    {
        if (a == cx.A) {
            ++n_enum;
            std::array<uint16_t, kMaxA> srt = idx;
            std::sort(srt.begin(), srt.begin() + cx.A);
            unsigned __int128 key = 0;
            for (int q = 0; q < cx.A; ++q) key = (key << 16) | (unsigned __int128)(srt[q] + 1);
            const int sg = ((inv & 1) ? -1 : 1) * pat->eta;
            table.add(key, GInt{sg * coef0.re, sg * coef0.im});
            return;
        }
        const int k = pat->k[a];
        const KindDef &kd = (*cx.kinds)[k];
        const int f = kd.flav[0], gfl = kd.flav[1];
        const int nf = f == 0 ? cx.nu : cx.nd, ng = gfl == 0 ? cx.nu : cx.nd;
        uint32_t uf = f == 0 ? used_u : used_d;
        uint32_t ug = gfl == 0 ? used_u : used_d;
        for (int p0 = 0; p0 < nf; ++p0) {
            if ((uf >> p0) & 1) continue;
            uint32_t uf0 = uf | (1u << p0);
            int inv0 = __builtin_popcount(uf >> p0);
            for (int p1 = 0; p1 < ng; ++p1) {
                if ((ug >> p1) & 1) continue;
                uint32_t ug1 = ug | (1u << p1);
                int inv1 = __builtin_popcount(ug >> p1);
                for (int p2 = p0 + 1; p2 < nf; ++p2) {
                    if ((uf0 >> p2) & 1) continue;
                    int inv2 = __builtin_popcount(uf0 >> p2);
                    uint32_t uf2 = uf0 | (1u << p2);
                    int i1 = val(f, p0), i2 = val(gfl, p1), i3 = val(f, p2);
                    int c = pair_index(i1, i3) * 12 + i2;
                    int e = k * kBlockLen + c;
                    if (zero_entry[e]) continue;
                    idx[a] = (uint16_t)e;
                    uint32_t nu_ = f == 0 ? uf2 : ug1, nd_ = f == 0 ? ug1 : uf2;
                    rec(a + 1, nu_, nd_, inv + inv0 + inv1 + inv2);
                }
            }
        }
    }

    void run_group(const Group &grp)
    {
        g = &grp;
        for (const Pattern &p : cx.snk) {
            pat = &p;
            bool ovf = false;
            coef0 = gmul(p.c, grp.w, ovf);
            if (ovf) throw std::runtime_error("coefficient overflow");
            rec(0, 0, 0, 0);
        }
    }
};

struct Term {
    std::array<uint16_t, kMaxA> rep;
    GInt c;
};

// Merge records of one group: equal normalised hashes in every trial.
// Second level: evaluate each distinct monomial on the random F_p propagators
// and merge monomials whose values agree up to sign in every trial (identity
// testing, App. C); the representative is the smallest tuple, with its sign.
template <class F>
void merge(const SynTable &tb, const Ctx &cx, const std::vector<std::vector<F>> &bh, std::vector<Term> &out)
{
    struct R {
        std::array<uint64_t, 2 * kMaxTrials> h;
        std::array<uint16_t, kMaxA> rep;
        __int128 re, im;
        int8_t s;
    };
    std::vector<R> rs;
    rs.reserve(tb.n);
    for (const SynSlot &x : tb.slots) {
        if (!x.key || (x.re == 0 && x.im == 0)) continue;
        R r{};
        unsigned __int128 k = x.key;
        for (int q = cx.A - 1; q >= 0; --q) {
            r.rep[q] = (uint16_t)((uint16_t)(k & 0xFFFF) - 1);
            k >>= 16;
        }
        for (int q = cx.A; q < kMaxA; ++q) r.rep[q] = 0xFFFF;
        F hv[kMaxTrials];
        int first = -1;
        for (int t = 0; t < cx.trials; ++t) {
            F v = bh[t][r.rep[0]];
            for (int q = 1; q < cx.A; ++q) v = v * bh[t][r.rep[q]];
            hv[t] = v;
            if (first < 0 && !v.zero()) first = t;
        }
        if (first < 0) continue;  // identically zero monomial
        const bool neg = hv[first].negative();
        for (int t = 0; t < cx.trials; ++t) {
            F v = neg ? hv[t].neg() : hv[t];
            r.h[2 * t] = v.k0();
            r.h[2 * t + 1] = v.k1();
        }
        r.s = neg ? -1 : 1;
        r.re = x.re * r.s;
        r.im = x.im * r.s;
        rs.push_back(r);
    }
    const int nk = 2 * cx.trials;
    std::sort(rs.begin(), rs.end(), [nk](const R &x, const R &y) {
        for (int t = 0; t < nk; ++t)
            if (x.h[t] != y.h[t]) return x.h[t] < y.h[t];
        return x.rep < y.rep;
    });
    const __int128 lim = ((__int128)1) << 62;
    for (size_t i = 0; i < rs.size();) {
        size_t j = i;
        __int128 re = 0, im = 0;
        while (j < rs.size() && std::equal(rs[j].h.begin(), rs[j].h.begin() + nk, rs[i].h.begin())) {
            re += rs[j].re;
            im += rs[j].im;
            ++j;
        }
        if (re != 0 || im != 0) {
            if (re > lim || re < -lim || im > lim || im < -lim) throw std::runtime_error("merged coefficient overflow");
            Term t;
            t.rep = rs[i].rep;
            t.c = GInt{(int64_t)(rs[i].s * re), (int64_t)(rs[i].s * im)};
            out.push_back(t);
        }
        i = j;
    }
    std::sort(out.begin(), out.end(), [](const Term &x, const Term &y) { return x.rep < y.rep; });
}

template <class F>
void hash_blocks(const Ctx &cx, const std::vector<KindDef> &kinds, int sites, uint64_t seed,
                 std::vector<std::vector<F>> &bh, std::vector<uint8_t> &zero_entry)
{
    const int K = (int)kinds.size();
    bh.assign(cx.trials, std::vector<F>((size_t)K * kBlockLen));
    zero_entry.assign((size_t)K * kBlockLen, 1);
    for (int t = 0; t < cx.trials; ++t) {
        uint64_t st = seed ^ (0xA24BAED4963EE407ULL * (uint64_t)(t + 1));
        std::vector<F> S[2];
        for (int fl = 0; fl < 2; ++fl) {
            S[fl].resize((size_t)sites * 144);
            for (auto &v : S[fl]) {
                GInt gi{(int64_t)(splitmix(st) % kP), 0};
                v = F::from(gi);
            }
        }
        for (int k = 0; k < K; ++k) {
            const KindDef &kd = kinds[k];
            std::vector<F> raw(1728);
            for (int x = 0; x < sites; ++x) {
                const F *s1 = &S[kd.flav[0]][(size_t)x * 144], *s2 = &S[kd.flav[1]][(size_t)x * 144],
                        *s3 = &S[kd.flav[2]][(size_t)x * 144];
                for (size_t n = 0; n < kd.w.size(); ++n) {
                    F w = F::from(kd.w[n]);
                    const F *r1 = s1 + 12 * kd.j[n][0], *r2 = s2 + 12 * kd.j[n][1], *r3 = s3 + 12 * kd.j[n][2];
                    for (int i1 = 0; i1 < 12; ++i1) {
                        F a = w * r1[i1];
                        for (int i2 = 0; i2 < 12; ++i2) {
                            F b = a * r2[i2];
                            for (int i3 = 0; i3 < 12; ++i3) {
                                F &o = raw[i1 * 144 + i2 * 12 + i3];
                                o = o + b * r3[i3];
                            }
                        }
                    }
                }
            }
            for (int i3 = 1; i3 < 12; ++i3)
                for (int i1 = 0; i1 < i3; ++i1)
                    for (int i2 = 0; i2 < 12; ++i2) {
                        F v = raw[i1 * 144 + i2 * 12 + i3] - raw[i3 * 144 + i2 * 12 + i1];
                        size_t e = (size_t)k * kBlockLen + pair_index(i1, i3) * 12 + i2;
                        bh[t][e] = v;
                        if (!v.zero()) zero_entry[e] = 0;
                    }
        }
    }
}

template <class F>
void enumerate_all(const Ctx &cx, const std::vector<std::vector<F>> &bh, const std::vector<uint8_t> &ze,
                   std::vector<std::vector<Term>> &per_group, std::vector<int64_t> &enum_count,
                   std::string &err)
{
    const size_t ng = cx.groups.size();
    per_group.assign(ng, {});
    enum_count.assign(ng, 0);
    std::atomic<size_t> next{0};
    std::atomic<bool> bad{false};
    std::mutex emu;
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    auto work = [&]() {
        Enumerator<F> en(cx, bh, ze);
        for (;;) {
            size_t gi = next.fetch_add(1);
            if (gi >= ng || bad.load()) break;
            try {
                en.table.reset();
                en.n_enum = 0;
                en.run_group(cx.groups[gi]);
                enum_count[gi] = en.n_enum;
                merge(en.table, cx, bh, per_group[gi]);
            } catch (const std::exception &e) {
                std::lock_guard<std::mutex> lk(emu);
                err = e.what();
                bad = true;
            }
        }
    };
    std::vector<std::thread> th;
    for (unsigned i = 0; i < nth; ++i) th.emplace_back(work);
    for (auto &t : th) t.join();
}

}  // namespace

// ---------------------------------------------------------------- build_plan
wick_status build_plan(const wick_nucleus_desc *d, wick_plan_t *out)
{
    if (!d || !out) return fail(WICK_EINVAL, "wick_plan: null argument");
    *out = nullptr;
    const int A = d->A;
    if (A < 1 || A > kMaxA) return fail(WICK_EINVAL, "wick_plan: A must be in 1..5");
    if (d->n_kinds < 1 || !d->kinds) return fail(WICK_EINVAL, "wick_plan: no kinds");
    if (d->n_snk < 1 || !d->snk_kind || !d->snk_re || !d->snk_im)
        return fail(WICK_EINVAL, "wick_plan: no sink patterns");
    if (d->n_src < 1 || !d->src_kind || !d->src_re || !d->src_im)
        return fail(WICK_EINVAL, "wick_plan: no source patterns");
    const int trials = d->hash_trials ? d->hash_trials : 2;
    const int sites = d->hash_sites ? d->hash_sites : 8;
    if (trials < 1 || trials > kMaxTrials) return fail(WICK_EINVAL, "wick_plan: hash_trials must be 1..4");
    if (sites < A || sites > 4096) return fail(WICK_EINVAL, "wick_plan: hash_sites must be >= A and <= 4096");
    const uint64_t seed = d->hash_seed ? d->hash_seed : 0x5EED0F7AB1E5ULL;

    // kinds
    std::vector<KindDef> all((size_t)d->n_kinds);
    bool gauss = false;
    for (int k = 0; k < d->n_kinds; ++k) {
        const wick_kind &wk = d->kinds[k];
        for (int s = 0; s < 3; ++s) {
            if (wk.flavor[s] != 0 && wk.flavor[s] != 1) return fail(WICK_EINVAL, "wick_plan: flavor must be 0 or 1");
            all[k].flav[s] = wk.flavor[s];
        }
        if (wk.n_w < 0 || (wk.n_w > 0 && (!wk.j || !wk.w_re || !wk.w_im)))
            return fail(WICK_EINVAL, "wick_plan: bad kind weights");
        for (int n = 0; n < wk.n_w; ++n) {
            std::array<int8_t, 3> j{wk.j[3 * n], wk.j[3 * n + 1], wk.j[3 * n + 2]};
            for (int s = 0; s < 3; ++s)
                if (j[s] < 0 || j[s] > 11) return fail(WICK_EINVAL, "wick_plan: spin-color index out of range");
            if (wk.w_re[n] == 0 && wk.w_im[n] == 0) continue;
            if (wk.w_im[n] != 0) gauss = true;
            if (std::llabs(wk.w_re[n]) > (1LL << 20) || std::llabs(wk.w_im[n]) > (1LL << 20))
                return fail(WICK_ETOOBIG, "wick_plan: weight magnitude above 2^20");
            all[k].j.push_back(j);
            all[k].w.push_back(GInt{wk.w_re[n], wk.w_im[n]});
        }
    }
    auto check_pat = [&](const int32_t *pk, int n) -> bool {
        for (int i = 0; i < n * A; ++i)
            if (pk[i] < 0 || pk[i] >= d->n_kinds) return false;
        return true;
    };
    if (!check_pat(d->snk_kind, d->n_snk) || !check_pat(d->src_kind, d->n_src))
        return fail(WICK_EINVAL, "wick_plan: pattern kind index out of range");

    // block kinds = kinds used at the sink
    std::vector<int> remap((size_t)d->n_kinds, -1);
    auto plan = new wick_plan_s();
    plan->A = A;
    plan->scale = d->scale;
    Ctx cx;
    cx.A = A;
    cx.trials = trials;
    int nu_ref = -1;
    for (int s = 0; s < d->n_snk; ++s) {
        Pattern p;
        std::vector<int> f;
        for (int a = 0; a < A; ++a) {
            int k = d->snk_kind[s * A + a];
            const KindDef &kd = all[k];
            if (!(kd.flav[0] == kd.flav[2] && kd.flav[0] != kd.flav[1])) {
                delete plan;
                return fail(WICK_EUNSUPPORTED, "wick_plan: sink kinds must have flavors (f, g, f) with f != g");
            }
            if (remap[k] < 0) {
                remap[k] = (int)plan->kinds.size();
                plan->kinds.push_back(kd);
            }
            p.k[a] = remap[k];
            for (int q = 0; q < 3; ++q) f.push_back(kd.flav[q]);
        }
        int nu = (int)std::count(f.begin(), f.end(), 0);
        if (nu_ref < 0) nu_ref = nu;
        if (nu != nu_ref) {
            delete plan;
            return fail(WICK_EINVAL, "wick_plan: sink patterns differ in flavor content");
        }
        p.c = GInt{d->snk_re[s], d->snk_im[s]};
        if (p.c.im) gauss = true;
        if (p.c.re == 0 && p.c.im == 0) continue;
        p.eta = listing_eta(f);
        cx.snk.push_back(p);
    }
    if ((int)plan->kinds.size() * kBlockLen > 65535) {
        delete plan;
        return fail(WICK_ETOOBIG, "wick_plan: more than 82 block kinds");
    }
    cx.nu = nu_ref;
    cx.nd = 3 * A - nu_ref;
    cx.kinds = &plan->kinds;

    // 1. antisymmetrised source groups
    std::map<std::pair<uint64_t, uint64_t>, GAcc> gmap;
    for (int sp = 0; sp < d->n_src; ++sp) {
        GInt cs{d->src_re[sp], d->src_im[sp]};
        if (cs.im) gauss = true;
        if (cs.re == 0 && cs.im == 0) continue;
        std::vector<int> g;
        const int32_t *pk = d->src_kind + sp * A;
        for (int a = 0; a < A; ++a)
            for (int q = 0; q < 3; ++q) g.push_back(all[pk[a]].flav[q]);
        if ((int)std::count(g.begin(), g.end(), 0) != cx.nu) {
            delete plan;
            return fail(WICK_EINVAL, "wick_plan: source and sink differ in flavor content");
        }
        const int eta = listing_eta(g);
        // mixed-radix walk over the nonzero weights of each source nucleon
        std::array<int, kMaxA> ctr{};
        bool empty = false;
        for (int a = 0; a < A; ++a) empty |= all[pk[a]].w.empty();
        if (empty) continue;
        for (;;) {
            int vals[3 * kMaxA];
            GInt w{1, 0};
            bool ovf = false;
            for (int a = 0; a < A; ++a) {
                const KindDef &kd = all[pk[a]];
                for (int q = 0; q < 3; ++q) vals[3 * a + q] = kd.j[ctr[a]][q];
                w = gmul(w, kd.w[ctr[a]], ovf);
            }
            w = gmul(w, cs, ovf);
            if (ovf) {
                delete plan;
                return fail(WICK_ETOOBIG, "wick_plan: source weight overflow");
            }
            int uv[16], dv[16], nu = 0, nd = 0;
            for (int r = 0; r < 3 * A; ++r) {
                if (g[r] == 0) uv[nu++] = vals[r]; else dv[nd++] = vals[r];
            }
            int inv = 0;
            bool pauli = false;
            for (int x = 0; x < nu && !pauli; ++x)
                for (int y = x + 1; y < nu; ++y) {
                    if (uv[x] == uv[y]) { pauli = true; break; }
                    inv += uv[x] > uv[y];
                }
            for (int x = 0; x < nd && !pauli; ++x)
                for (int y = x + 1; y < nd; ++y) {
                    if (dv[x] == dv[y]) { pauli = true; break; }
                    inv += dv[x] > dv[y];
                }
            if (!pauli) {
                std::sort(uv, uv + nu);
                std::sort(dv, dv + nd);
                uint64_t ku = 0, kd = 0;
                for (int x = 0; x < nu; ++x) ku = (ku << 4) | (uint64_t)uv[x];
                for (int x = 0; x < nd; ++x) kd = (kd << 4) | (uint64_t)dv[x];
                gmap[{ku, kd}].add(w, ((inv & 1) ? -1 : 1) * eta);
            }
            int a = A - 1;
            for (; a >= 0; --a) {
                if (++ctr[a] < (int)all[pk[a]].w.size()) break;
                ctr[a] = 0;
            }
            if (a < 0) break;
        }
    }
    for (auto &kv : gmap) {
        if (kv.second.re == 0 && kv.second.im == 0) continue;
        const __int128 lim = ((__int128)1) << 62;
        if (kv.second.re > lim || kv.second.re < -lim || kv.second.im > lim || kv.second.im < -lim) {
            delete plan;
            return fail(WICK_ETOOBIG, "wick_plan: source group weight overflow");
        }
        Group gr;
        uint64_t ku = kv.first.first, kd = kv.first.second;
        for (int x = cx.nu - 1; x >= 0; --x) { gr.U[x] = (int8_t)(ku & 15); ku >>= 4; }
        for (int x = cx.nd - 1; x >= 0; --x) { gr.D[x] = (int8_t)(kd & 15); kd >>= 4; }
        gr.w = GInt{(int64_t)kv.second.re, (int64_t)kv.second.im};
        cx.groups.push_back(gr);
    }
    plan->n_groups = (int64_t)cx.groups.size();

    // 2-3. enumerate and merge, group by group
    std::vector<std::vector<Term>> per_group;
    std::vector<int64_t> enum_count;
    std::string err;
    try {
        if (gauss) {
            std::vector<std::vector<FC>> bh;
            std::vector<uint8_t> ze;
            hash_blocks(cx, plan->kinds, sites, seed, bh, ze);
            enumerate_all(cx, bh, ze, per_group, enum_count, err);
        } else {
            std::vector<std::vector<FR>> bh;
            std::vector<uint8_t> ze;
            hash_blocks(cx, plan->kinds, sites, seed, bh, ze);
            enumerate_all(cx, bh, ze, per_group, enum_count, err);
        }
    } catch (const std::bad_alloc &) {
        delete plan;
        return fail(WICK_ENOMEM, "wick_plan: out of host memory");
    }
    if (!err.empty()) {
        delete plan;
        return fail(WICK_ETOOBIG, "wick_plan: " + err);
    }

    // 4. emit
    int64_t n = 0;
    double bound = 0.0;
    const double per = std::pow(6.0 * A / (double)kP, trials);
    for (size_t gi = 0; gi < per_group.size(); ++gi) {
        n += (int64_t)per_group[gi].size();
        plan->n_enumerated += enum_count[gi];
        double m = (double)enum_count[gi];
        bound += 0.5 * m * (m - 1) * per;
    }
    plan->bound = bound;
    plan->n_terms = n;
    try {
        plan->kidx.resize((size_t)A * (size_t)n);
        plan->coef_re.resize((size_t)n);
        plan->coef_im.resize((size_t)n);
    } catch (const std::bad_alloc &) {
        delete plan;
        return fail(WICK_ENOMEM, "wick_plan: out of host memory for the table");
    }
    int64_t o = 0;
    bool real = true;
    for (auto &vec : per_group) {
        for (const Term &t : vec) {
            for (int a = 0; a < A; ++a) plan->kidx[(size_t)a * n + o] = t.rep[a];
            plan->coef_re[o] = d->scale * (double)t.c.re;
            plan->coef_im[o] = d->scale * (double)t.c.im;
            if (t.c.im) real = false;
            ++o;
        }
        std::vector<Term>().swap(vec);
    }
    plan->coef_real = real;
    factor_kinds(plan);
    *out = plan;
    return WICK_OK;
}

// ------------------------------------------------------- kind factorisation
// Rows of a kind: w(j1, ., .) for each j1 with nonzero weights. Rows equal up
// to sign (across kinds of one flavor pattern) are computed once per site and
// shared (they are the diquark rows eps * (C g5 P) of the nucleon operators).
namespace {
int eps3(int a, int b, int c)
{
    if (a == b || b == c || a == c) return 0;
    return ((a > b) + (a > c) + (b > c)) & 1 ? -1 : 1;
}

// Exact test of the nucleon form; on success alpha and M (row s3, column s2).
bool nucleon_form(const KindDef &kd, int &alpha, int M[4][4])
{
    if (kd.w.empty()) return false;
    int W[12][12][12] = {};
    for (size_t n = 0; n < kd.w.size(); ++n) {
        if (kd.w[n].im != 0 || std::llabs(kd.w[n].re) > 127) return false;
        W[kd.j[n][0]][kd.j[n][1]][kd.j[n][2]] += (int)kd.w[n].re;
    }
    alpha = kd.j[0][0] / 3;
    // read M off the (c1, c2, c3) = (0, 2, 1) entries, where eps[0][1][2] = +1
    for (int s3 = 0; s3 < 4; ++s3)
        for (int s2 = 0; s2 < 4; ++s2) M[s3][s2] = W[3 * alpha][3 * s2 + 2][3 * s3 + 1];
    for (int j1 = 0; j1 < 12; ++j1)
        for (int j2 = 0; j2 < 12; ++j2)
            for (int j3 = 0; j3 < 12; ++j3) {
                int want = j1 / 3 == alpha ? eps3(j1 % 3, j3 % 3, j2 % 3) * M[j3 / 3][j2 / 3] : 0;
                if (W[j1][j2][j3] != want) return false;
            }
    return true;
}
}  // namespace

void factor_kinds(wick_plan_s *p)
{
    p->egroups.clear();
    p->nucgroups.clear();
    {
        // nucleon groups: kinds of one flavor pattern sharing M, at most kMaxKindsPerGroup each
        std::vector<NucGroup> ng;
        std::vector<std::array<int, 16>> keys;
        bool all = true;
        for (int k = 0; k < (int)p->kinds.size() && all; ++k) {
            int alpha, M[4][4];
            if (!nucleon_form(p->kinds[k], alpha, M)) { all = false; break; }
            std::array<int, 16> key;
            for (int i = 0; i < 16; ++i) key[i] = M[i / 4][i % 4];
            int gi = -1;
            for (size_t g = 0; g < ng.size(); ++g)
                if (keys[g] == key && ng[g].f == p->kinds[k].flav[0] && ng[g].g == p->kinds[k].flav[1] &&
                    (int)ng[g].kinds.size() < kMaxKindsPerGroup)
                    gi = (int)g;
            if (gi < 0) {
                NucGroup g;
                g.f = p->kinds[k].flav[0];
                g.g = p->kinds[k].flav[1];
                for (int s3 = 0; s3 < 4; ++s3)
                    for (int s2 = 0; s2 < 4; ++s2)
                        if (M[s3][s2]) g.pairs.push_back({(int8_t)s2, (int8_t)s3, (int8_t)M[s3][s2]});
                ng.push_back(g);
                keys.push_back(key);
                gi = (int)ng.size() - 1;
            }
            ng[gi].kinds.push_back(k);
            ng[gi].alpha.push_back(alpha);
        }
        if (all) p->nucgroups = ng;
    }
    const int K = (int)p->kinds.size();
    using Row = std::vector<std::pair<int, int64_t>>;  // (j2*12+j3, w)
    struct KR { int j1; Row row; int sign; };
    std::vector<std::vector<KR>> krows(K);
    for (int k = 0; k < K; ++k) {
        std::map<int, std::map<int, int64_t>> m;
        const KindDef &kd = p->kinds[k];
        for (size_t n = 0; n < kd.w.size(); ++n) m[kd.j[n][0]][kd.j[n][1] * 12 + kd.j[n][2]] += kd.w[n].re;
        for (auto &r : m) {
            Row row;
            for (auto &e : r.second)
                if (e.second) row.push_back({e.first, e.second});
            if (row.empty()) continue;
            int sign = row[0].second > 0 ? 1 : -1;
            for (auto &e : row) e.second *= sign;
            krows[k].push_back({r.first, row, sign});
        }
    }
    // union kinds of the same flavor pattern that share a row
    std::vector<int> parent(K);
    for (int k = 0; k < K; ++k) parent[k] = k;
    std::function<int(int)> root = [&](int x) { return parent[x] == x ? x : parent[x] = root(parent[x]); };
    std::map<std::pair<std::pair<int, int>, Row>, int> owner;
    for (int k = 0; k < K; ++k)
        for (auto &kr : krows[k]) {
            auto key = std::make_pair(std::make_pair(p->kinds[k].flav[0], p->kinds[k].flav[1]), kr.row);
            auto it = owner.find(key);
            if (it == owner.end()) owner[key] = k;
            else parent[root(k)] = root(it->second);
        }
    std::map<int, std::vector<int>> comps;
    for (int k = 0; k < K; ++k) comps[root(k)].push_back(k);
    for (auto &c : comps) {
        const std::vector<int> &ks = c.second;
        for (size_t s = 0; s < ks.size(); s += kMaxKindsPerGroup) {
            EGroup eg;
            eg.f = p->kinds[ks[s]].flav[0];
            eg.g = p->kinds[ks[s]].flav[1];
            std::vector<Row> rows;
            size_t e = std::min(ks.size(), s + kMaxKindsPerGroup);
            for (size_t q = s; q < e; ++q) eg.kinds.push_back(ks[q]);
            for (int k : eg.kinds)
                for (auto &kr : krows[k])
                    if (std::find(rows.begin(), rows.end(), kr.row) == rows.end()) rows.push_back(kr.row);
            const int R = (int)rows.size();
            for (auto &row : rows) {
                ERow er;
                for (auto &t : row) {
                    er.jj.push_back({(int8_t)(t.first / 12), (int8_t)(t.first % 12)});
                    er.w.push_back((int8_t)std::max<int64_t>(-128, std::min<int64_t>(127, t.second)));
                }
                eg.rows.push_back(er);
            }
            eg.aop.assign((size_t)eg.kinds.size() * R * kMaxAop, {0, 0});
            for (size_t kk = 0; kk < eg.kinds.size(); ++kk)
                for (auto &kr : krows[eg.kinds[kk]]) {
                    int r = (int)(std::find(rows.begin(), rows.end(), kr.row) - rows.begin());
                    auto *slot = &eg.aop[(kk * R + r) * kMaxAop];
                    int u = 0;
                    while (u < kMaxAop && slot[u][1] != 0) ++u;
                    if (u < kMaxAop) slot[u] = {(int8_t)kr.j1, (int8_t)kr.sign};
                    else slot[0] = {slot[0][0], 0};  // marks overflow; checked by the launcher
                }
            p->egroups.push_back(eg);
        }
    }
}

// ----------------------------------------------------------------- plan I/O
namespace {
constexpr char kMagic[8] = {'W', 'I', 'C', 'K', 'P', 'L', 'N', '1'};
constexpr uint32_t kVersion = 1;

uint64_t fnv1a(const std::string &s)
{
    uint64_t h = 1469598103934665603ULL;
    for (unsigned char c : s) { h ^= c; h *= 1099511628211ULL; }
    return h;
}
template <class T> void put(std::string &s, const T &v) { s.append((const char *)&v, sizeof(T)); }
template <class T> bool get(const std::string &s, size_t &o, T &v)
{
    if (o + sizeof(T) > s.size()) return false;
    std::memcpy(&v, s.data() + o, sizeof(T));
    o += sizeof(T);
    return true;
}
}  // namespace

wick_status save_plan(const wick_plan_s *p, const char *path)
{
    if (!p || !path) return fail(WICK_EINVAL, "wick_plan_save: null argument");
    std::string b;
    put(b, kVersion);
    put(b, (int32_t)p->A);
    put(b, p->scale);
    put(b, p->n_enumerated);
    put(b, p->n_groups);
    put(b, p->bound);
    put(b, (int32_t)p->kinds.size());
    for (auto &k : p->kinds) {
        for (int s = 0; s < 3; ++s) put(b, (int32_t)k.flav[s]);
        put(b, (int64_t)k.w.size());
        for (size_t n = 0; n < k.w.size(); ++n) {
            for (int s = 0; s < 3; ++s) put(b, k.j[n][s]);
            put(b, k.w[n].re);
            put(b, k.w[n].im);
        }
    }
    put(b, p->n_terms);
    put(b, (uint8_t)(p->coef_real ? 1 : 0));
    b.append((const char *)p->kidx.data(), p->kidx.size() * sizeof(uint16_t));
    b.append((const char *)p->coef_re.data(), p->coef_re.size() * sizeof(double));
    b.append((const char *)p->coef_im.data(), p->coef_im.size() * sizeof(double));
    uint64_t h = fnv1a(b);
    std::ofstream f(path, std::ios::binary);
    if (!f) return fail(WICK_EINVAL, std::string("wick_plan_save: cannot open ") + path);
    f.write(kMagic, 8);
    f.write(b.data(), (std::streamsize)b.size());
    f.write((const char *)&h, sizeof(h));
    if (!f) return fail(WICK_EINVAL, "wick_plan_save: write failed");
    return WICK_OK;
}

wick_status load_plan(const char *path, wick_plan_t *out)
{
    if (!path || !out) return fail(WICK_EINVAL, "wick_plan_load: null argument");
    *out = nullptr;
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(WICK_EINVAL, std::string("wick_plan_load: cannot open ") + path);
    std::string all((std::istreambuf_iterator<char>(f)), std::istreambuf_iterator<char>());
    if (all.size() < 16 || std::memcmp(all.data(), kMagic, 8) != 0)
        return fail(WICK_ECORRUPT, "wick_plan_load: not a plan file");
    std::string b = all.substr(8, all.size() - 16);
    uint64_t h;
    std::memcpy(&h, all.data() + all.size() - 8, 8);
    if (h != fnv1a(b)) return fail(WICK_ECORRUPT, "wick_plan_load: checksum mismatch");
    size_t o = 0;
    uint32_t ver;
    auto p = new wick_plan_s();
    auto bad = [&]() { delete p; return fail(WICK_ECORRUPT, "wick_plan_load: truncated or inconsistent file"); };
    int32_t A, K;
    if (!get(b, o, ver) || ver != kVersion) { delete p; return fail(WICK_ECORRUPT, "wick_plan_load: version mismatch"); }
    if (!get(b, o, A) || !get(b, o, p->scale) || !get(b, o, p->n_enumerated) || !get(b, o, p->n_groups) ||
        !get(b, o, p->bound) || !get(b, o, K))
        return bad();
    if (A < 1 || A > kMaxA || K < 1 || K > 82) return bad();
    p->A = A;
    p->kinds.resize(K);
    for (auto &k : p->kinds) {
        int64_t nw;
        for (int s = 0; s < 3; ++s) {
            int32_t v;
            if (!get(b, o, v) || (v != 0 && v != 1)) return bad();
            k.flav[s] = v;
        }
        // block kinds are nucleon-like: flavors (f, g, f) with g != f
        if (k.flav[0] != k.flav[2] || k.flav[1] == k.flav[0]) return bad();
        if (!get(b, o, nw) || nw < 0 || nw > 1728) return bad();
        for (int64_t n = 0; n < nw; ++n) {
            std::array<int8_t, 3> j;
            GInt w;
            for (int s = 0; s < 3; ++s)
                if (!get(b, o, j[s]) || j[s] < 0 || j[s] > 11) return bad();
            if (!get(b, o, w.re) || !get(b, o, w.im)) return bad();
            if (std::llabs(w.re) > (1LL << 20) || std::llabs(w.im) > (1LL << 20)) return bad();
            k.j.push_back(j);
            k.w.push_back(w);
        }
    }
    uint8_t real;
    if (!get(b, o, p->n_terms) || !get(b, o, real) || p->n_terms < 0) return bad();
    size_t nt = (size_t)p->n_terms;
    if (o + nt * (A * 2 + 16) != b.size()) return bad();
    p->kidx.resize(nt * A);
    p->coef_re.resize(nt);
    p->coef_im.resize(nt);
    std::memcpy(p->kidx.data(), b.data() + o, nt * A * 2); o += nt * A * 2;
    std::memcpy(p->coef_re.data(), b.data() + o, nt * 8); o += nt * 8;
    std::memcpy(p->coef_im.data(), b.data() + o, nt * 8);
    p->coef_real = real != 0;
    for (uint16_t v : p->kidx)
        if (v >= K * kBlockLen) return bad();
    factor_kinds(p);
    *out = p;
    return WICK_OK;
}

}  // namespace wick
