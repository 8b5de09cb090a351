// C ABI of the library (declared in include/wick.h): argument validation,
// device copies of plans, per-stream workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <deque>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <sstream>
#include <string>
#include <tuple>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"

namespace wick {

namespace {
thread_local std::string g_last_error;
}

void set_error(const std::string &msg) { g_last_error = msg; }

wick_status fail(wick_status st, const std::string &msg)
{
    set_error(msg);
    return st;
}

namespace {

wick_status hip_fail(hipError_t e, const char *what)
{
    return fail(WICK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

// ------------------------------------------------------------- workspaces
namespace {
struct Workspace {
    void *ptr = nullptr;
    size_t bytes = 0;
};
std::mutex g_ws_mu;
std::map<std::tuple<int, hipStream_t, int>, Workspace> g_ws;  // (device, stream, tag)
wick_status ws_hip_fail(hipError_t e, const char *what)
{
    return fail(WICK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}
}  // namespace

// A device buffer of at least `bytes` private to (device, stream, tag). Growing
// it waits for the stream, so earlier work that used the old buffer is done.
// Tag 0 serves the block and term-sum launches; other tags hold buffers that
// must stay alive across such launches.
wick_status workspace(hipStream_t s, size_t bytes, void **out, int tag)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return ws_hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace &w = g_ws[std::make_tuple(dev, s, tag)];
    if (w.bytes < bytes) {
        if (w.ptr) {
            e = hipStreamSynchronize(s);
            if (e != hipSuccess) return ws_hip_fail(e, "hipStreamSynchronize");
            (void)hipFree(w.ptr);
            w.ptr = nullptr;
            w.bytes = 0;
        }
        size_t want = std::max<size_t>(bytes, 1 << 20);
        e = hipMalloc(&w.ptr, want);
        if (e != hipSuccess) return fail(WICK_ENOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
        w.bytes = want;
    }
    *out = w.ptr;
    return WICK_OK;
}

wick_status workspace(hipStream_t s, size_t bytes, void **out) { return workspace(s, bytes, out, 0); }

namespace {

void release_workspace(hipStream_t s)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(g_ws_mu);
    bool synced = false;
    for (auto it = g_ws.begin(); it != g_ws.end();) {
        if (std::get<0>(it->first) == dev && std::get<1>(it->first) == s) {
            if (!synced) { (void)hipStreamSynchronize(s); synced = true; }
            (void)hipFree(it->second.ptr);
            it = g_ws.erase(it);
        } else {
            ++it;
        }
    }
}

// ---------------------------------------------------------- device tables
struct DevPlan {
    int device = -1;
    int n_tiles = 0, n_passes = 0;
    NucDesc *nuc = nullptr;  // null unless every kind has nucleon form (FP64 packing)
    int nuc_tiles = 0, nuc_passes = 0;
    NucDesc *nuc_split = nullptr;  // the same for the split-precision modes
    int split_tiles = 0, split_passes = 0;
    EGroupDev *groups = nullptr;
    BlocksDesc *desc = nullptr;  // null when the staged kernel does not apply
    uint16_t *kidx = nullptr;  // plain table (null when packed)
    double *coef = nullptr;
    uint64_t *words = nullptr;  // packed or segmented table (null when plain)
    double2 *pal = nullptr;
    int n_pal = 0;
    uint32_t *seg_prefix = nullptr;  // segmented table only
    int64_t *chunk_base = nullptr;
    int32_t *chunk_len = nullptr;
    int32_t *chunk_g = nullptr;  // factored table only
    int n_chunks = 0, seg_len = 0;
    double coef_unit = 0.0;  // segmented table: integer-coefficient words when nonzero
};

TermTable table_of(const DevPlan *d, const wick_plan_s *p)
{
    TermTable t{};
    t.words = d->words;
    t.pal = d->pal;
    t.n_pal = d->n_pal;
    t.coef_real = p->coef_real ? 1 : 0;
    t.kidx = d->kidx;
    t.coef = d->coef;
    t.seg_prefix = d->seg_prefix;
    t.coef_unit = d->coef_unit;
    t.chunk_base = d->chunk_base;
    t.chunk_len = d->chunk_len;
    t.chunk_g = d->chunk_g;
    t.n_chunks = d->n_chunks;
    return t;
}

// Palette index of every term (entry 0 of the palette is zero when `zero`
// is set); false when the table has more distinct coefficients than fit.
bool palette_of(const wick_plan_s *p, bool zero, std::vector<uint8_t> &idx, std::vector<double2> &pal)
{
    const size_t nt = (size_t)p->n_terms;
    idx.assign(nt, 0);
    pal.clear();
    if (zero) pal.push_back(double2{0.0, 0.0});
    int last = -1;
    for (size_t n = 0; n < nt; ++n) {
        const double re = p->coef_re[n], im = p->coef_im[n];
        int c = -1;
        if (last >= 0 && pal[last].x == re && pal[last].y == im) c = last;
        for (int i = 0; c < 0 && i < (int)pal.size(); ++i)
            if (pal[i].x == re && pal[i].y == im) c = i;
        if (c < 0) {
            if ((int)pal.size() == kMaxPalette) return false;
            c = (int)pal.size();
            pal.push_back(double2{re, im});
        }
        last = c;
        idx[n] = (uint8_t)c;
    }
    return true;
}

// Host image of the segmented form of a table (see TermTable).
struct SegTable {
    std::vector<uint64_t> words;
    std::vector<uint32_t> prefix;
    std::vector<int64_t> base;
    std::vector<int32_t> len;  // nodes per lane | (steps with a leaf 1) << 16
    std::vector<int32_t> g;    // factored form: steps of prefix-group words per chunk (else empty)
    std::vector<double2> pal;
    int seg_len = 0;
    double unit = 0.0;  // integer-coefficient words (see TermTable) when nonzero
};

// The common unit of a real table: a number u with every coefficient equal
// to q * u for an integer q, |q| <= the word's limit, to within 2^-50 of the
// coefficient (so the words carry the coefficients to FP64 accuracy), else 0
// (the palette form is used). u is the smallest |coefficient| divided by the
// smallest d <= 64 that makes every ratio an integer, times the gcd of the
// resulting q: the gcd of integer coefficients (4He: 48), or for instance
// 1/24 for an operator whose coefficients are multiples of 1/24.
double coef_unit_of(const wick_plan_s *p)
{
    const size_t nt = (size_t)p->n_terms;
    double s0 = INFINITY;
    for (size_t n = 0; n < nt; ++n) {
        const double re = p->coef_re[n];
        if (p->coef_im[n] != 0.0 || re == 0.0 || !std::isfinite(re)) return 0.0;
        s0 = std::min(s0, std::fabs(re));
    }
    if (!(s0 < INFINITY)) return 0.0;
    auto exact = [](double c, double q, double u) { return std::fabs(c - q * u) <= 0x1p-50 * std::fabs(c); };
    for (int d = 1; d <= 64; ++d) {
        const double u = s0 / d;
        uint64_t g = 0;
        bool ok = true;
        for (size_t n = 0; n < nt && ok; ++n) {
            const double q = std::nearbyint(p->coef_re[n] / u);
            if (std::fabs(q) > 64.0 * kIntCoefMax || !exact(p->coef_re[n], q, u)) {
                ok = false;
                break;
            }
            uint64_t a = (uint64_t)std::fabs(q), b = g;
            while (b) { const uint64_t r = a % b; a = b; b = r; }
            g = a;
        }
        if (!ok) continue;
        const double unit = u * (double)g;
        for (size_t n = 0; n < nt; ++n) {
            const double q = std::nearbyint(p->coef_re[n] / unit);
            if (std::fabs(q) > kIntCoefMax || !exact(p->coef_re[n], q, unit)) return 0.0;
        }
        return unit;
    }
    return 0.0;
}

// LDS bank balance of the gathers of integer-coefficient words. Step j of a
// chunk gathers, for each lane, the node entry, leaf 0 and leaf 1 of the
// lane's j-th word, as three wave-wide 16-byte LDS reads. A 16-byte slot s
// lies in bank group s mod 16, and such a read takes longer the more lanes
// hit the same group (measured on MI355X: 13.5 cycles per wave-wide read for
// random slots; 9.3 when each group is hit at most twice per half-wave or per
// quarter-wave; 6.3 when in addition every quarter-wave uses the same
// lane-to-group pattern). A sum does not depend on the order of its words,
// so each lane's words are reordered greedily: at each step the lanes of a
// half-wave in turn take, among their next kBalanceWindow words (or
// WICK_BALANCE_WINDOW, for measurement), the one
// whose three groups are least used so far in that half-wave at that step
// (balancing per quarter-wave instead measured 2 % slower on the
// 64-configuration batch). A lane's words fall into parts that are reordered
// each among themselves: its prefix-group words (steps [0, lane_g), factored
// form only), then, from the chunk's step G = g[c] (0 unless factored), its
// two-leaf words (lane_two of them) and its one-leaf words (lane_len in all).
// Chunks are independent (host threads).
int slices_per_group(int K, int64_t n_sets);
constexpr int kBalanceWindow = 16;
constexpr uint64_t kIdxMask = (1u << kPackBits) - 1;
void balance_banks(SegTable &out, const std::vector<int32_t> &lane_len, const std::vector<int32_t> &lane_two,
                   const std::vector<int32_t> &lane_g, int ntg)
{
    // LDS bank group of entry e: the term sum interleaves ntg slices, entry e of
    // slice 0 at 16-byte slot e * ntg (slice t adds t to every lane alike)
    auto grp = [ntg](uint64_t e) { return (int)((e * (uint64_t)ntg) & 15); };
    const size_t n_chunks = out.base.size();
    const char *win_env = std::getenv("WICK_BALANCE_WINDOW");  // for measurement
    const int window = win_env ? std::max(1, std::min(256, std::atoi(win_env))) : kBalanceWindow;
    auto work = [&](size_t c_lo, size_t c_hi) {
        for (size_t c = c_lo; c < c_hi; ++c) {
            uint64_t *w = out.words.data() + out.base[c];
            const int len = out.len[c] & 0xffff, G = out.g.empty() ? 0 : out.g[c];
            const int32_t *ll = lane_len.data() + c * 64, *l2 = lane_two.data() + c * 64;
            const int32_t *lg = lane_g.empty() ? nullptr : lane_g.data() + c * 64;
            for (int j = 0; j < len; ++j)
                for (int h = 0; h < 2; ++h) {
                    uint8_t cnt[3][16] = {};
                    for (int l = 32 * h; l < 32 * h + 32; ++l) {
                        int part_end;  // end of the part holding step j (exclusive)
                        if (j < G) {
                            if (j >= lg[l]) continue;
                            part_end = lg[l];
                        } else {
                            const int jm = j - G;
                            if (jm >= ll[l]) continue;
                            part_end = G + (jm < l2[l] ? l2[l] : ll[l]);
                        }
                        const int end = std::min(part_end, j + window);
                        int best = j, best_cost = 1 << 30;
                        for (int k = j; k < end; ++k) {
                            const uint64_t v = w[(size_t)k * 64 + l];
                            int cost = cnt[0][grp((v >> kPackBits) & kIdxMask)] + cnt[1][grp(v & kIdxMask)];
                            if (v >> 53) cost += cnt[2][grp((v >> (2 * kPackBits)) & kIdxMask)];
                            if (cost < best_cost) { best_cost = cost; best = k; }
                        }
                        std::swap(w[(size_t)j * 64 + l], w[(size_t)best * 64 + l]);
                        const uint64_t v = w[(size_t)j * 64 + l];
                        ++cnt[0][grp((v >> kPackBits) & kIdxMask)];
                        ++cnt[1][grp(v & kIdxMask)];
                        if (v >> 53) ++cnt[2][grp((v >> (2 * kPackBits)) & kIdxMask)];
                    }
                }
        }
    };
    const size_t nth = std::max<size_t>(1, std::min<size_t>(16, std::thread::hardware_concurrency()));
    if (n_chunks < 64 || nth == 1) { work(0, n_chunks); return; }
    std::vector<std::thread> th;
    for (size_t i = 0; i < nth; ++i) th.emplace_back(work, n_chunks * i / nth, n_chunks * (i + 1) / nth);
    for (auto &t : th) t.join();
}

bool segment_table(const wick_plan_s *p, SegTable &out)
{
    const int A = p->A;
    const size_t nt = (size_t)p->n_terms;
    if (A < 2 || A > 4 || (int)p->kinds.size() > kMaxLdsKinds || nt == 0 || nt > 0xffffffffULL) return false;
    out = SegTable{};
    std::vector<uint8_t> pidx;
    if (!palette_of(p, true, pidx, out.pal)) return false;
    // integer words for A <= 3 (an A = 4 table with integer coefficients
    // takes the factored form, which sets chunk_g)
    const char *form_env = std::getenv("WICK_TABLE_FORM");
    out.unit = (form_env && std::string(form_env) == "segmented-palette") || A == 4 ? 0.0 : coef_unit_of(p);
    auto qbits = [&](uint32_t t) {  // 11-bit two's complement of coef / unit
        const int64_t q = std::llround(p->coef_re[t] / out.unit);
        return (uint64_t)q & 0x7ff;
    };
    const uint16_t *k = p->kidx.data();
    auto ix = [&](int a, uint32_t t) { return (uint32_t)k[(size_t)a * nt + t]; };
    // terms in lexicographic order of their index tuples (LSD radix sort, 14-bit digits)
    std::vector<uint32_t> ord(nt), tmp(nt);
    for (size_t t = 0; t < nt; ++t) ord[t] = (uint32_t)t;
    std::vector<size_t> cnt((size_t)1 << kPackBits);
    for (int a = A - 1; a >= 0; --a) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (size_t i = 0; i < nt; ++i) ++cnt[ix(a, ord[i])];
        size_t acc = 0;
        for (auto &c : cnt) { const size_t v = c; c = acc; acc += v; }
        for (size_t i = 0; i < nt; ++i) tmp[cnt[ix(a, ord[i])]++] = ord[i];
        ord.swap(tmp);
    }
    tmp.clear();
    tmp.shrink_to_fit();
    auto prefix_of = [&](uint32_t t) {
        uint32_t v = 0;
        for (int a = 0; a < A - 2; ++a) v |= ix(a, t) << (kPackBits * a);
        return v;
    };
    // nodes: runs of terms sharing the first A-1 indices, cut into pieces of
    // kNodeLeaves terms; (start in ord, number of terms <= kNodeLeaves)
    std::vector<std::pair<uint32_t, uint8_t>> nodes;
    for (size_t i = 0; i < nt;) {
        const uint32_t pre = prefix_of(ord[i]), nd = ix(A - 2, ord[i]);
        size_t j = i + 1;
        while (j < nt && j - i < (size_t)kNodeLeaves && ix(A - 2, ord[j]) == nd && prefix_of(ord[j]) == pre) ++j;
        nodes.push_back({(uint32_t)i, (uint8_t)(j - i)});
        i = j;
    }
    // segments: runs of nodes sharing the first A-2 indices, at most seg_nodes
    // nodes: nodes / 8192 within [8, 128], so that a table has about 8192
    // segments (3He: 113; segments of 14, 32, 64 and 128 measured 5.41, 5.11,
    // 5.02 and 4.98 ms for the 64-configuration batch's term sum: each segment
    // and chunk costs a prefix product and a pipeline start); WICK_SEG_WORDS
    // overrides, for measurement
    const char *seg_env = std::getenv("WICK_SEG_WORDS");
    const int seg_nodes = seg_env ? std::max(1, std::min(4096, std::atoi(seg_env)))
                                  : (int)std::min<size_t>(128, std::max<size_t>(8, nodes.size() / 8192));
    out.seg_len = seg_nodes * kNodeLeaves;
    struct Seg {
        uint32_t first, n, two;  // first node, number of nodes, of them with two leaves
    };
    std::vector<Seg> segs;
    for (size_t i = 0; i < nodes.size();) {
        const uint32_t pre = prefix_of(ord[nodes[i].first]);
        size_t j = i + 1;
        while (j < nodes.size() && j - i < (size_t)seg_nodes && prefix_of(ord[nodes[j].first]) == pre) ++j;
        uint32_t two = 0;
        for (size_t q = i; q < j; ++q) two += nodes[q].second > 1;
        segs.push_back({(uint32_t)i, (uint32_t)(j - i), two});
        i = j;
    }
    // longest segments first; among equal lengths, most two-leaf nodes first
    // (so that the lanes of a chunk run out of leaf 1 at about the same step)
    std::stable_sort(segs.begin(), segs.end(),
                     [](const Seg &x, const Seg &y) { return x.n != y.n ? x.n > y.n : x.two > y.two; });
    const size_t n_chunks = (segs.size() + 63) / 64;
    out.prefix.assign(n_chunks * 64, 0);
    out.base.resize(n_chunks);
    out.len.resize(n_chunks);
    size_t total = 0;
    for (size_t c = 0; c < n_chunks; ++c) {
        out.base[c] = (int64_t)total;
        out.len[c] = (int32_t)segs[c * 64].n;  // nodes per lane
        total += (size_t)out.len[c] * 64;  // one word per node
    }
    out.words.assign(total, 0);  // zero word: leaf 0, node 0, palette entry 0 (zero)
    for (size_t c = 0; c < n_chunks; ++c)
        for (int lane = 0; lane < 64; ++lane) {
            const size_t si = c * 64 + lane;
            if (si >= segs.size()) continue;  // an empty lane keeps zero words
            uint64_t *w = out.words.data() + out.base[c] + lane;
            const uint32_t n0 = segs[si].first, nn = segs[si].n;
            out.prefix[si] = prefix_of(ord[nodes[n0].first]);
            // integer words: the two-leaf nodes at steps [0, two), the others after
            uint32_t at2 = 0, at1 = out.unit ? segs[si].two : 0;
            for (uint32_t kk = 0; kk < nn; ++kk) {
                const auto &nd = nodes[n0 + kk];
                const uint32_t t0 = ord[nd.first];
                uint64_t v;
                if (out.unit) {
                    v = (uint64_t)ix(A - 1, t0) | ((uint64_t)ix(A - 2, t0) << kPackBits) | (qbits(t0) << 42);
                    if (nd.second > 1) {
                        const uint32_t t1 = ord[nd.first + 1];
                        v |= ((uint64_t)ix(A - 1, t1) << 28) | (qbits(t1) << 53);
                    }
                } else {
                    v = (uint64_t)ix(A - 1, t0) | ((uint64_t)ix(A - 2, t0) << kPackBits) |
                        ((uint64_t)pidx[t0] << (2 * kPackBits));
                    if (nd.second > 1) {
                        const uint32_t t1 = ord[nd.first + 1];
                        v |= ((uint64_t)ix(A - 1, t1) << 36) | ((uint64_t)pidx[t1] << 50);
                    }
                }
                const uint32_t at = !out.unit ? kk : nd.second > 1 ? at2++ : at1++;
                w[(size_t)at * 64] = v;
            }
        }
    if (out.unit && !std::getenv("WICK_NO_BANK_BALANCE")) {
        // lengths of the lanes' segments, for the reordering below (the
        // variable turns it off, for measurement)
        std::vector<int32_t> lane_len(n_chunks * 64, 0), lane_two(n_chunks * 64, 0);
        for (size_t si = 0; si < segs.size(); ++si) {
            lane_len[si] = (int32_t)segs[si].n;
            lane_two[si] = (int32_t)segs[si].two;
        }
        balance_banks(out, lane_len, lane_two, {}, slices_per_group((int)p->kinds.size(), kMaxTG));
    }
    // steps in which some lane's word has a leaf 1: all of them in the
    // palette form, the lanes' largest number of two-leaf nodes otherwise
    for (size_t c = 0; c < n_chunks; ++c) {
        int32_t two = out.len[c];
        if (out.unit) {
            two = 0;
            for (size_t si = c * 64; si < std::min(segs.size(), c * 64 + 64); ++si)
                two = std::max(two, (int32_t)segs[si].two);
        }
        out.len[c] |= two << 16;
    }
    return true;
}

// Factored form of an A = 4 table with integer coefficients (see TermTable).
// The index positions are reordered so that the pair of positions with the
// fewest distinct index pairs comes first: the prefix (i, j) of a term. The
// terms of one prefix, sorted by their last two indices and divided by g, the
// gcd of their q with the sign of the first, are the prefix's list; prefixes
// with equal lists share it, so that
//   C = unit * sum_m G_m M_m,  M_m = sum over the words of list m of
//   B[node] (q0 B[leaf0] + q1 B[leaf1]),  G_m = sum over the prefixes of
//   list m of g B[i] B[j],
// where each prefix is one G word (node i, leaf j, q = g; the prefixes of a
// list have distinct i and distinct j in every built-in nucleus, so there is
// nothing to pair, and the term sum gathers no leaf 1 for G words). This
// evaluates each list once for all its prefixes (4He: 28751 lists for 364752
// prefixes). Each list's words (two-leaf words first) are cut into pieces of
// at most piece_words (kPieceWords, or WICK_PIECE_WORDS for measurement); a
// piece is one lane's segment and carries all the G words of its list.
// Longer pieces repeat G less often but make fewer, longer chunks. Pieces are
// sorted by length, then by their two-leaf words, and dealt to the 64 lanes of
// a chunk; chunk c holds g[c] steps of G words (fewer in a lane padded with
// zero words), then its list words.
constexpr int kPieceWords = 256;
bool factor_table(const wick_plan_s *p, SegTable &out)
{
    const char *piece_env = std::getenv("WICK_PIECE_WORDS");
    const uint32_t piece_words = piece_env ? (uint32_t)std::max(8, std::min(4096, std::atoi(piece_env))) : kPieceWords;
    const size_t nt = (size_t)p->n_terms;
    if (p->A != 4 || (int)p->kinds.size() > kMaxLdsKinds || nt == 0 || nt > 0xffffffffULL) return false;
    const char *form_env = std::getenv("WICK_TABLE_FORM");
    if (form_env && std::string(form_env) == "segmented-palette") return false;
    out.unit = coef_unit_of(p);
    if (out.unit == 0.0) return false;
    out.pal.assign(1, double2{0.0, 0.0});  // not read by integer words
    const uint16_t *k = p->kidx.data();
    // the leading pair of positions: fewest distinct index pairs (a bitmap of
    // 2^28 pairs per candidate, candidates on host threads)
    int perm[4] = {0, 1, 2, 3};
    {
        const int cand[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
        size_t count[6] = {};
        auto distinct = [&](int i) {
            std::vector<uint64_t> bits((size_t)1 << (2 * kPackBits - 6), 0);
            const uint16_t *ka = k + (size_t)cand[i][0] * nt, *kb = k + (size_t)cand[i][1] * nt;
            for (size_t t = 0; t < nt; ++t) {
                const uint32_t key = ((uint32_t)ka[t] << kPackBits) | kb[t];
                bits[key >> 6] |= (uint64_t)1 << (key & 63);
            }
            size_t n = 0;
            for (uint64_t b : bits) n += (size_t)__builtin_popcountll(b);
            count[i] = n;
        };
        std::vector<std::thread> th;
        for (int i = 0; i < 6; ++i) th.emplace_back(distinct, i);
        for (auto &t : th) t.join();
        int best = 0;
        for (int i = 1; i < 6; ++i)
            if (count[i] < count[best]) best = i;
        perm[0] = cand[best][0];
        perm[1] = cand[best][1];
        for (int a = 0, o = 2; a < 4; ++a)
            if (a != perm[0] && a != perm[1]) perm[o++] = a;
    }
    auto ix = [&](int a, uint32_t t) { return (uint32_t)k[(size_t)perm[a] * nt + t]; };
    auto qv = [&](uint32_t t) { return (int32_t)std::llround(p->coef_re[t] / out.unit); };
    // terms in lexicographic order of their reordered index tuples
    std::vector<uint32_t> ord(nt), tmp(nt);
    for (size_t t = 0; t < nt; ++t) ord[t] = (uint32_t)t;
    {
        std::vector<size_t> cnt((size_t)1 << kPackBits);
        for (int a = 3; a >= 0; --a) {
            std::fill(cnt.begin(), cnt.end(), 0);
            for (size_t i = 0; i < nt; ++i) ++cnt[ix(a, ord[i])];
            size_t acc = 0;
            for (auto &c : cnt) { const size_t v = c; c = acc; acc += v; }
            for (size_t i = 0; i < nt; ++i) tmp[cnt[ix(a, ord[i])]++] = ord[i];
            ord.swap(tmp);
        }
    }
    tmp.clear();
    tmp.shrink_to_fit();
    // prefixes: runs [i0, i1) of ord sharing the first two indices, with g
    struct Prefix {
        uint32_t i0, i1;
        int32_t g;
    };
    std::vector<Prefix> pre;
    for (size_t i = 0; i < nt;) {
        const uint32_t a0 = ix(0, ord[i]), a1 = ix(1, ord[i]);
        size_t j = i + 1;
        while (j < nt && ix(0, ord[j]) == a0 && ix(1, ord[j]) == a1) ++j;
        int32_t g = 0;
        for (size_t n = i; n < j; ++n) {
            int32_t a = std::abs(qv(ord[n])), b = g;
            while (b) { const int32_t r = a % b; a = b; b = r; }
            g = a;
        }
        if (qv(ord[i]) < 0) g = -g;
        pre.push_back({(uint32_t)i, (uint32_t)j, g});
        i = j;
    }
    // distinct lists (hash of (node, leaf, q / g) over the run, equality checked)
    auto list_hash = [&](const Prefix &x) {
        uint64_t h = 0x9e3779b97f4a7c15ULL ^ (uint64_t)(x.i1 - x.i0);
        for (uint32_t n = x.i0; n < x.i1; ++n) {
            const uint32_t t = ord[n];
            const uint64_t v = ((uint64_t)ix(2, t) << 32) | ((uint64_t)ix(3, t) << 11) | (uint64_t)((qv(t) / x.g) & 0x7ff);
            h = (h ^ v) * 0x100000001b3ULL;
            h ^= h >> 29;
        }
        return h;
    };
    auto same_list = [&](const Prefix &x, const Prefix &y) {
        if (x.i1 - x.i0 != y.i1 - y.i0) return false;
        for (uint32_t n = 0; n < x.i1 - x.i0; ++n) {
            const uint32_t t = ord[x.i0 + n], u = ord[y.i0 + n];
            if (ix(2, t) != ix(2, u) || ix(3, t) != ix(3, u) || qv(t) / x.g != qv(u) / y.g) return false;
        }
        return true;
    };
    std::unordered_map<uint64_t, std::vector<uint32_t>> by_hash;  // hash -> lists
    std::vector<uint32_t> rep;                                    // list -> its first prefix
    std::vector<std::vector<uint32_t>> members;                   // list -> its prefixes
    for (uint32_t pi = 0; pi < (uint32_t)pre.size(); ++pi) {
        auto &cands = by_hash[list_hash(pre[pi])];
        uint32_t m = UINT32_MAX;
        for (uint32_t c : cands)
            if (same_list(pre[rep[c]], pre[pi])) { m = c; break; }
        if (m == UINT32_MAX) {
            m = (uint32_t)rep.size();
            rep.push_back(pi);
            members.emplace_back();
            cands.push_back(m);
        }
        members[m].push_back(pi);
    }
    auto word = [](uint32_t node, uint32_t l0, int32_t q0, uint32_t l1, int32_t q1) {
        return (uint64_t)l0 | ((uint64_t)node << kPackBits) | ((uint64_t)l1 << (2 * kPackBits)) |
               ((uint64_t)((uint32_t)q0 & 0x7ff) << 42) | ((uint64_t)((uint32_t)q1 & 0x7ff) << 53);
    };
    // words of each list: list words (two-leaf first) and G words
    const size_t n_lists = rep.size();
    std::vector<size_t> mw_off(n_lists + 1, 0), gw_off(n_lists + 1, 0);
    std::vector<uint32_t> mw_two(n_lists, 0);
    std::vector<uint64_t> mw, gw;
    for (size_t m = 0; m < n_lists; ++m) {
        const Prefix &x = pre[rep[m]];
        std::vector<uint64_t> one;
        for (uint32_t n = x.i0; n < x.i1;) {
            const uint32_t node = ix(2, ord[n]);
            uint32_t e = n + 1;
            while (e < x.i1 && ix(2, ord[e]) == node) ++e;
            for (uint32_t a = n; a < e; a += 2) {
                const uint32_t t0 = ord[a];
                if (a + 1 < e) {
                    const uint32_t t1 = ord[a + 1];
                    mw.push_back(word(node, ix(3, t0), qv(t0) / x.g, ix(3, t1), qv(t1) / x.g));
                    ++mw_two[m];
                } else {
                    one.push_back(word(node, ix(3, t0), qv(t0) / x.g, 0, 0));
                }
            }
            n = e;
        }
        mw.insert(mw.end(), one.begin(), one.end());
        mw_off[m + 1] = mw.size();
        for (uint32_t pi : members[m]) {  // one G word per prefix
            const Prefix &y = pre[pi];
            gw.push_back(word(ix(0, ord[y.i0]), ix(1, ord[y.i0]), y.g, 0, 0));
        }
        gw_off[m + 1] = gw.size();
    }
    // pieces: (list, first list word, words, two-leaf words)
    struct Piece {
        uint32_t m, w0, n, two;
    };
    std::vector<Piece> pieces;
    for (size_t m = 0; m < n_lists; ++m) {
        const uint32_t n = (uint32_t)(mw_off[m + 1] - mw_off[m]);
        for (uint32_t a = 0; a < n; a += piece_words) {
            const uint32_t len = std::min<uint32_t>(piece_words, n - a);
            const uint32_t two = a < mw_two[m] ? std::min<uint32_t>(len, mw_two[m] - a) : 0;
            pieces.push_back({(uint32_t)m, (uint32_t)mw_off[m] + a, len, two});
        }
    }
    std::stable_sort(pieces.begin(), pieces.end(),
                     [](const Piece &x, const Piece &y) { return x.n != y.n ? x.n > y.n : x.two > y.two; });
    const size_t n_chunks = (pieces.size() + 63) / 64;
    out.prefix.assign(n_chunks * 64, 0);
    out.base.resize(n_chunks);
    out.len.resize(n_chunks);
    out.g.resize(n_chunks);
    std::vector<int32_t> lane_len(n_chunks * 64, 0), lane_two(n_chunks * 64, 0), lane_g(n_chunks * 64, 0);
    size_t total = 0;
    for (size_t c = 0; c < n_chunks; ++c) {
        int32_t G = 0, M = 0, two = 0;
        for (size_t si = c * 64; si < std::min(pieces.size(), c * 64 + 64); ++si) {
            const Piece &pc = pieces[si];
            lane_g[si] = (int32_t)(gw_off[pc.m + 1] - gw_off[pc.m]);
            lane_len[si] = (int32_t)pc.n;
            lane_two[si] = (int32_t)pc.two;
            G = std::max(G, lane_g[si]);
            M = std::max(M, lane_len[si]);
            two = std::max(two, lane_two[si]);
        }
        if (G + M > 0xffff) return false;  // (a chunk's steps fit 16 bits)
        out.base[c] = (int64_t)total;
        out.g[c] = G;
        out.len[c] = (G + M) | ((G + two) << 16);
        total += (size_t)(G + M) * 64;
    }
    out.words.assign(total, 0);
    for (size_t si = 0; si < pieces.size(); ++si) {
        const size_t c = si / 64, lane = si % 64;
        uint64_t *w = out.words.data() + out.base[c] + lane;
        const Piece &pc = pieces[si];
        for (int32_t a = 0; a < lane_g[si]; ++a) w[(size_t)a * 64] = gw[gw_off[pc.m] + a];
        for (uint32_t a = 0; a < pc.n; ++a) w[(size_t)(out.g[c] + a) * 64] = mw[pc.w0 + a];
    }
    // terms per lane and chunk, for sizing the term-sum workgroups
    out.seg_len = (int)std::max<size_t>(1, nt / (64 * n_chunks));
    if (!std::getenv("WICK_NO_BANK_BALANCE"))
        balance_banks(out, lane_len, lane_two, lane_g, slices_per_group((int)p->kinds.size(), kMaxTG));
    return true;
}

// The packed form of a table (see TermTable), or false when it does not apply.
bool pack_table(const wick_plan_s *p, std::vector<uint64_t> &words, std::vector<double2> &pal)
{
    const size_t nt = (size_t)p->n_terms;
    if (p->A > 4 || (int)p->kinds.size() > kMaxLdsKinds || nt == 0) return false;
    words.assign(nt, 0);
    pal.clear();
    int last = -1;
    for (size_t n = 0; n < nt; ++n) {
        const double re = p->coef_re[n], im = p->coef_im[n];
        int c = -1;
        if (last >= 0 && pal[last].x == re && pal[last].y == im) c = last;
        for (int i = 0; c < 0 && i < (int)pal.size(); ++i)
            if (pal[i].x == re && pal[i].y == im) c = i;
        if (c < 0) {
            if ((int)pal.size() == kMaxPalette) return false;
            c = (int)pal.size();
            pal.push_back(double2{re, im});
        }
        last = c;
        uint64_t w = (uint64_t)c << 56;
        for (int a = 0; a < p->A; ++a) w |= (uint64_t)p->kidx[(size_t)a * nt + n] << (kPackBits * a);
        words[n] = w;
    }
    return true;
}

std::mutex g_dev_mu;
std::map<const wick_plan_s *, std::deque<DevPlan>> g_dev;  // deque: stable element addresses

// Form of a plan's term table (the values of wick_plan_sum_work's form).
enum TableForm { kFormPlain = 0, kFormPacked = 1, kFormSegPalette = 2, kFormSegInt = 3, kFormFactored = 4 };
bool segment_table(const wick_plan_s *p, SegTable &out);
bool factor_table(const wick_plan_s *p, SegTable &out);
bool pack_table(const wick_plan_s *p, std::vector<uint64_t> &words, std::vector<double2> &pal);

// The table form of a plan: segmented for A >= 3 (sharing the leading indices
// pays: 22 % faster than packed on 4He, 31 % on 3He), factored for A = 4 with
// integer coefficients, packed for A = 2, plain when neither fits;
// WICK_TABLE_FORM=plain|packed|segmented|segmented-palette selects one
// (testing; segmented uses integer-coefficient words when the coefficients
// allow, segmented-palette never). words/pal receive the words and palette of
// the word forms; seg the segmented form's chunk layout.
int choose_table(const wick_plan_s *p, SegTable &seg, std::vector<uint64_t> &words, std::vector<double2> &pal)
{
    const char *form_env = std::getenv("WICK_TABLE_FORM");
    const std::string form = form_env ? form_env : "";
    const bool want_seg = form == "segmented" || form == "segmented-palette" || (form.empty() && p->A >= 3);
    if (want_seg && (factor_table(p, seg) || segment_table(p, seg))) {
        words.swap(seg.words);
        pal = seg.pal;
        return !seg.g.empty() ? kFormFactored : seg.unit != 0.0 ? kFormSegInt : kFormSegPalette;
    }
    if ((form.empty() || form == "packed") && pack_table(p, words, pal)) return kFormPacked;
    return kFormPlain;
}

// Work of a table per time slice: words with two and with one leaf (zero
// padding words not counted) and lanes with a segment; a plain or packed
// table has one word per term.
struct TableWork {
    int32_t form = -1;
    int64_t w2 = 0, w1 = 0, segs = 0;
};
TableWork table_work(int form, const SegTable &seg, const std::vector<uint64_t> &words, int64_t n_terms)
{
    TableWork w;
    w.form = form;
    if (form < kFormSegPalette) {
        w.w1 = n_terms;
        return w;
    }
    for (size_t c = 0; c < seg.base.size(); ++c) {
        const int steps = seg.len[c] & 0xffff;
        for (int l = 0; l < 64; ++l) {
            bool any = false;
            for (int j = 0; j < steps; ++j) {
                const uint64_t v = words[seg.base[c] + (size_t)j * 64 + l];
                if (!v) continue;
                any = true;
                const bool two = form == kFormSegPalette ? ((v >> 50) & 0xff) != 0 : (v >> 53) != 0;
                ++(two ? w.w2 : w.w1);
            }
            w.segs += any;
        }
    }
    return w;
}
std::map<const wick_plan_s *, TableWork> g_work;  // under g_dev_mu

// The table work of a plan: recorded when its table was uploaded, else the
// table is built on the host (no device needed) and the result kept.
TableWork plan_work(const wick_plan_s *p)
{
    {
        std::lock_guard<std::mutex> lk(g_dev_mu);
        auto it = g_work.find(p);
        if (it != g_work.end()) return it->second;
    }
    SegTable seg;
    std::vector<uint64_t> words;
    std::vector<double2> pal;
    const int f = choose_table(p, seg, words, pal);
    const TableWork w = table_work(f, seg, words, p->n_terms);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    g_work.emplace(p, w);
    return w;
}


wick_status check_groups(const wick_plan_s *p)
{
    for (const EGroup &g : p->egroups) {
        if ((int)g.rows.size() > kMaxRows) return fail(WICK_EUNSUPPORTED, "block kinds need more than 8 shared rows");
        for (const ERow &r : g.rows)
            if ((int)r.w.size() > kMaxRowTerms) return fail(WICK_EUNSUPPORTED, "a kind row has more than 16 terms");
        for (auto &a : g.aop)
            if (a[1] == 0 && a[0] != 0) return fail(WICK_EUNSUPPORTED, "a kind uses one row more than twice");
    }
    for (const KindDef &k : p->kinds)
        for (const GInt &w : k.w)
            if (w.im != 0 || w.re > 127 || w.re < -127)
                return fail(WICK_EUNSUPPORTED, "the GPU block kernel takes real weights in [-127, 127]");
    return WICK_OK;
}

wick_status device_plan(wick_plan_s *p, hipStream_t s, DevPlan **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto &vec = g_dev[p];
    for (auto &d : vec)
        if (d.device == dev) {
            *out = &d;
            return WICK_OK;
        }
    wick_status st = check_groups(p);
    if (st != WICK_OK) return st;
    DevPlan d;
    d.device = dev;
    std::vector<EGroupDev> hg(p->egroups.size());
    for (size_t i = 0; i < p->egroups.size(); ++i) {
        const EGroup &g = p->egroups[i];
        EGroupDev &h = hg[i];
        std::memset(&h, 0, sizeof(h));
        h.f = g.f;
        h.g = g.g;
        h.R = (int)g.rows.size();
        h.nk = (int)g.kinds.size();
        h.mt = (12 * h.nk + 15) / 16;
        for (int k = 0; k < h.nk; ++k) h.kind_out[k] = g.kinds[k];
        for (int r = 0; r < h.R; ++r) {
            h.nterm[r] = (int)g.rows[r].w.size();
            for (int t = 0; t < h.nterm[r]; ++t) {
                h.j2[r][t] = g.rows[r].jj[t][0];
                h.j3[r][t] = g.rows[r].jj[t][1];
                h.w[r][t] = g.rows[r].w[t];
            }
            for (int k = 0; k < h.nk; ++k)
                for (int u = 0; u < kMaxAop; ++u) {
                    auto a = g.aop[((size_t)k * h.R + r) * kMaxAop + u];
                    h.aj1[k][r][u] = a[0];
                    h.aa[k][r][u] = a[1];
                }
        }
    }
    // the staged kernel's descriptor: groups packed into passes of at most
    // kPassTiles m-tiles (first fit, largest groups first)
    BlocksDesc bd;
    std::memset(&bd, 0, sizeof(bd));
    for (int pp = 0; pp < kMaxPasses; ++pp)
        for (int t = 0; t < kPassTiles; ++t) bd.tile_group[pp][t] = -1;
    bool staged = (int)hg.size() <= kMaxGroupsStaged;
    int max_tiles = 0;
    if (staged) {
        bd.n_groups = (int)hg.size();
        std::vector<int> order(hg.size());
        for (size_t g = 0; g < hg.size(); ++g) order[g] = (int)g;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return hg[x].mt > hg[y].mt; });
        for (int g : order) {
            bd.groups[g] = hg[g];
            if (hg[g].mt > kPassTiles) { staged = false; break; }
            int pp = 0;
            while (pp < bd.n_passes && bd.pass_tiles[pp] + hg[g].mt > kPassTiles) ++pp;
            if (pp == kMaxPasses) { staged = false; break; }
            if (pp == bd.n_passes) ++bd.n_passes;
            bd.pass_groups[pp][bd.pass_ngroups[pp]++] = g;
            for (int mt = 0; mt < hg[g].mt; ++mt) {
                bd.tile_group[pp][bd.pass_tiles[pp]] = g;
                bd.tile_mt[pp][bd.pass_tiles[pp]] = mt;
                ++bd.pass_tiles[pp];
            }
            max_tiles = std::max(max_tiles, bd.pass_tiles[pp]);
        }
    }
    if (staged) {
        d.n_tiles = max_tiles;
        d.n_passes = bd.n_passes;
        if ((e = hipMalloc(&d.desc, sizeof(BlocksDesc))) != hipSuccess)
            return fail(WICK_ENOMEM, std::string("plan upload hipMalloc: ") + hipGetErrorString(e));
        if ((e = hipMemcpy(d.desc, &bd, sizeof(bd), hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "plan upload hipMemcpy");
    }
    // the nucleon kernel's descriptors: groups packed into passes of at most
    // 4 m-tiles (FP64) or 3 (split modes, which also hold FP32 accumulators)
    if (!p->nucgroups.empty() && p->nucgroups.size() <= (size_t)kMaxGroupsStaged) {
        // twin groups (see NucGroupDev) share one E; WICK_NO_TWINS=1 keeps them apart (testing)
        auto twins = [&](const NucGroup &a, const NucGroup &b) {
            if (b.f != a.g || b.g != a.f || a.pairs.size() != b.pairs.size()) return false;
            for (const auto &x : a.pairs) {
                bool found = false;
                for (const auto &y : b.pairs) found |= y[0] == x[1] && y[1] == x[0] && y[2] == -x[2];
                if (!found) return false;
            }
            return true;
        };
        const bool no_twins = std::getenv("WICK_NO_TWINS") != nullptr;
        struct DevGroup {
            const NucGroup *own;
            std::vector<std::array<int, 4>> kinds;  // kind_out, alpha, flv, tr
        };
        for (int which = 0; which < 2; ++which) {
            const int cap = which == 0 ? 4 : 3;
            const int G0 = (int)p->nucgroups.size();
            std::vector<DevGroup> dgs;
            std::vector<char> used(G0, 0);
            for (int a = 0; a < G0; ++a) {
                if (used[a]) continue;
                used[a] = 1;
                const NucGroup &na = p->nucgroups[a];
                DevGroup dg{&na, {}};
                for (size_t k = 0; k < na.kinds.size(); ++k) dg.kinds.push_back({na.kinds[k], na.alpha[k], 0, 0});
                for (int b = a + 1; b < G0 && !no_twins; ++b) {
                    const NucGroup &nb = p->nucgroups[b];
                    const size_t nk = na.kinds.size() + nb.kinds.size();
                    if (used[b] || nk > (size_t)kMaxKindsPerGroup || (int)(12 * nk + 15) / 16 > cap || !twins(na, nb))
                        continue;
                    used[b] = 1;
                    for (size_t k = 0; k < nb.kinds.size(); ++k) dg.kinds.push_back({nb.kinds[k], nb.alpha[k], 1, 1});
                    break;
                }
                dgs.push_back(dg);
            }
            NucDesc nd;
            std::memset(&nd, 0, sizeof(nd));
            for (int pp = 0; pp < kMaxPasses; ++pp)
                for (int t = 0; t < kPassTiles; ++t) nd.tile_group[pp][t] = -1;
            bool ok = true;
            int maxt = 0;
            const int G = (int)dgs.size();
            std::vector<int> order(G);
            for (int g = 0; g < G; ++g) order[g] = g;
            auto tiles_of = [&](int g) { return (12 * (int)dgs[g].kinds.size() + 15) / 16; };
            std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return tiles_of(x) > tiles_of(y); });
            nd.n_groups = G;
            for (int g : order) {
                const NucGroup &ng = *dgs[g].own;
                NucGroupDev &h = nd.groups[g];
                h.f = ng.f;
                h.g = ng.g;
                h.npair = (int)ng.pairs.size();
                h.nk = (int)dgs[g].kinds.size();
                // diquark entries ordered M = +1, M = -1, other values (the kernel
                // folds a unit M into the sign pattern of its FMA chains)
                std::vector<std::array<int8_t, 3>> pr(ng.pairs.begin(), ng.pairs.end());
                auto cls = [](int m) { return m == 1 ? 0 : (m == -1 ? 1 : 2); };
                std::stable_sort(pr.begin(), pr.end(), [&](const auto &x, const auto &y) { return cls(x[2]) < cls(y[2]); });
                h.npos = h.nneg = 0;
                for (int i = 0; i < h.npair; ++i) {
                    h.s2[i] = pr[i][0];
                    h.s3[i] = pr[i][1];
                    h.m[i] = pr[i][2];
                    h.npos += pr[i][2] == 1;
                    h.nneg += pr[i][2] == -1;
                }
                for (int k = 0; k < h.nk; ++k) {
                    h.kind_out[k] = dgs[g].kinds[k][0];
                    h.alpha[k] = dgs[g].kinds[k][1];
                    h.flv[k] = dgs[g].kinds[k][2];
                    h.tr[k] = dgs[g].kinds[k][3];
                }
                const int mt = tiles_of(g);
                int pp = 0;
                while (pp < nd.n_passes && nd.pass_tiles[pp] + mt > cap) ++pp;
                if (mt > cap || pp == kMaxPasses) { ok = false; break; }
                if (pp == nd.n_passes) ++nd.n_passes;
                nd.pass_groups[pp][nd.pass_ngroups[pp]++] = g;
                for (int t = 0; t < mt; ++t) {
                    nd.tile_group[pp][nd.pass_tiles[pp]] = g;
                    nd.tile_mt[pp][nd.pass_tiles[pp]] = t;
                    ++nd.pass_tiles[pp];
                }
                maxt = std::max(maxt, nd.pass_tiles[pp]);
            }
            if (!ok) continue;
            NucDesc **dst = which == 0 ? &d.nuc : &d.nuc_split;
            if ((e = hipMalloc(dst, sizeof(NucDesc))) != hipSuccess)
                return fail(WICK_ENOMEM, std::string("plan upload hipMalloc: ") + hipGetErrorString(e));
            if ((e = hipMemcpy(*dst, &nd, sizeof(nd), hipMemcpyHostToDevice)) != hipSuccess)
                return hip_fail(e, "plan upload hipMemcpy");
            (which == 0 ? d.nuc_tiles : d.split_tiles) = maxt;
            (which == 0 ? d.nuc_passes : d.split_passes) = nd.n_passes;
        }
    }
    const size_t nt = (size_t)p->n_terms;
    std::vector<uint64_t> words;
    std::vector<double2> pal;
    SegTable seg;
    const int tform = choose_table(p, seg, words, pal);
    const bool segmented = tform >= kFormSegPalette, packed = tform == kFormPacked;
    if (!g_work.count(p)) g_work[p] = table_work(tform, seg, words, p->n_terms);
    const size_t coef_n = p->coef_real ? nt : 2 * nt;
    auto undo = [&] {
        for (void *q : {(void *)d.groups, (void *)d.desc, (void *)d.nuc, (void *)d.nuc_split, (void *)d.kidx,
                        (void *)d.coef, (void *)d.words, (void *)d.pal, (void *)d.seg_prefix, (void *)d.chunk_base,
                        (void *)d.chunk_len, (void *)d.chunk_g})
            if (q) (void)hipFree(q);
    };
    const bool word_form = segmented || packed;
    if ((e = hipMalloc(&d.groups, std::max<size_t>(1, hg.size()) * sizeof(EGroupDev))) != hipSuccess ||
        (word_form && (e = hipMalloc(&d.words, words.size() * sizeof(uint64_t))) != hipSuccess) ||
        (word_form && (e = hipMalloc(&d.pal, pal.size() * sizeof(double2))) != hipSuccess) ||
        (segmented && (e = hipMalloc(&d.seg_prefix, seg.prefix.size() * sizeof(uint32_t))) != hipSuccess) ||
        (segmented && (e = hipMalloc(&d.chunk_base, seg.base.size() * sizeof(int64_t))) != hipSuccess) ||
        (segmented && (e = hipMalloc(&d.chunk_len, seg.len.size() * sizeof(int32_t))) != hipSuccess) ||
        (!seg.g.empty() && (e = hipMalloc(&d.chunk_g, seg.g.size() * sizeof(int32_t))) != hipSuccess) ||
        (!word_form && (e = hipMalloc(&d.kidx, std::max<size_t>(1, nt * p->A) * sizeof(uint16_t))) != hipSuccess) ||
        (!word_form && (e = hipMalloc(&d.coef, std::max<size_t>(1, coef_n) * sizeof(double))) != hipSuccess)) {
        undo();
        return fail(WICK_ENOMEM, std::string("plan upload hipMalloc: ") + hipGetErrorString(e));
    }
    if (segmented) {
        d.n_chunks = (int)seg.base.size();
        d.seg_len = seg.seg_len;
        d.coef_unit = seg.unit;
        if ((e = hipMemcpy(d.seg_prefix, seg.prefix.data(), seg.prefix.size() * sizeof(uint32_t), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(d.chunk_base, seg.base.data(), seg.base.size() * sizeof(int64_t), hipMemcpyHostToDevice)) != hipSuccess ||
            (e = hipMemcpy(d.chunk_len, seg.len.data(), seg.len.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
            (!seg.g.empty() &&
             (e = hipMemcpy(d.chunk_g, seg.g.data(), seg.g.size() * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess)) {
            undo();
            return hip_fail(e, "plan upload hipMemcpy");
        }
    }
    d.n_pal = (int)pal.size();
    std::vector<double> coef(word_form ? 0 : coef_n);
    for (size_t n = 0; n < nt && !word_form; ++n) {
        if (p->coef_real) coef[n] = p->coef_re[n];
        else { coef[2 * n] = p->coef_re[n]; coef[2 * n + 1] = p->coef_im[n]; }
    }
    // synchronous copies: the host staging vectors die at return
    if ((e = hipMemcpy(d.groups, hg.data(), hg.size() * sizeof(EGroupDev), hipMemcpyHostToDevice)) != hipSuccess ||
        (word_form && (e = hipMemcpy(d.words, words.data(), words.size() * sizeof(uint64_t), hipMemcpyHostToDevice)) != hipSuccess) ||
        (word_form && (e = hipMemcpy(d.pal, pal.data(), pal.size() * sizeof(double2), hipMemcpyHostToDevice)) != hipSuccess) ||
        (!word_form && nt && (e = hipMemcpy(d.kidx, p->kidx.data(), nt * p->A * sizeof(uint16_t), hipMemcpyHostToDevice)) != hipSuccess) ||
        (!word_form && nt && (e = hipMemcpy(d.coef, coef.data(), coef_n * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)) {
        undo();
        return hip_fail(e, "plan upload hipMemcpy");
    }
    (void)s;
    vec.push_back(d);
    *out = &vec.back();
    return WICK_OK;
}

// ------------------------------------------------------------- tuning
struct Tune {
    int chunk_sites = 256;      // sites per workgroup of the block kernel
    int batch_chunk_sites = 0;  // the same for batched launches (0: derived from the batch size)
};
std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune;

std::string tune_key(const wick_plan_s *p, const int32_t dims[4], int dtype, int prec)
{
    std::ostringstream o;
    o << "gfx950:" << dims[0] << "x" << dims[1] << "x" << dims[2] << "x" << dims[3] << ":K" << p->kinds.size()
      << ":A" << p->A << ":N" << p->n_terms << ":d" << dtype << ":p" << prec;
    return o.str();
}

Tune tune_for(const wick_plan_s *p, const int32_t dims[4], int dtype, int prec)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(p, dims, dtype, prec));
    return it == g_tune.end() ? Tune{} : it->second;
}

// term-slice length of the sum, keyed by the table and the number of (cfg, t) sets
std::map<std::string, int64_t> g_slice;

std::string slice_key(const wick_plan_s *p, int64_t n_ct)
{
    std::ostringstream o;
    o << "gfx950:A" << p->A << ":K" << p->kinds.size() << ":N" << p->n_terms << ":ct" << n_ct;
    return o.str();
}

int64_t tuned_slice(const wick_plan_s *p, int64_t n_ct)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_slice.find(slice_key(p, n_ct));
    return it == g_slice.end() ? 0 : it->second;
}

// workgroups sharing one table slice in the term sum (ContractLaunch::share),
// under the same key; 1 (group-major order) unless tuned
std::map<std::string, int> g_share;

int tuned_share(const wick_plan_s *p, int64_t n_ct)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_share.find(slice_key(p, n_ct));
    return it == g_share.end() ? 1 : it->second;
}

// batched launches tuned as a whole: (block sites per workgroup, terms per
// term-sum workgroup), keyed by the lattice, storage, precision and the
// multiset of the items' tables (which configuration an item reads does not
// change the launch)
struct BatchTune {
    int chunk = 0;
    int64_t terms = 0;
    int share = 2;
};
std::map<std::string, BatchTune> g_batch_tune;

std::string batch_key(const wick_plan_t *plans, const wick_item *items, int n_items, const int32_t dims[4], int dtype,
                      int prec)
{
    std::map<std::string, int> count;
    for (int i = 0; i < n_items; ++i) {
        const wick_plan_s *p = plans[items[i].plan];
        std::ostringstream o;
        o << "A" << p->A << "K" << p->kinds.size() << "N" << p->n_terms;
        ++count[o.str()];
    }
    std::ostringstream o;
    o << "gfx950:" << dims[0] << "x" << dims[1] << "x" << dims[2] << "x" << dims[3] << ":d" << dtype << ":p" << prec;
    for (auto &kv : count) o << ":" << kv.first << "x" << kv.second;
    return o.str();
}

bool tuned_batch(const std::string &key, BatchTune *out)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_batch_tune.find(key);
    if (it == g_batch_tune.end()) return false;
    *out = it->second;
    return true;
}

// terms per workgroup: about 1024 workgroups over all n_groups (sets of time
// slices), at least 4096 terms each, a multiple of the workgroup size
int64_t default_slice_len(int64_t N, int64_t n_groups)
{
    int64_t len = std::max<int64_t>(4096, (N * n_groups + 1023) / 1024);
    return (len + kCThreads - 1) / kCThreads * kCThreads;
}

// chunks of a segmented table per term-sum workgroup for a target number of
// terms per workgroup: a multiple of the workgroup's 16 waves
int64_t chunks_per_group(int64_t terms, int seg_len)
{
    const int64_t waves = kCThreads / 64;
    const int64_t c = std::max<int64_t>(1, terms / (64 * (int64_t)seg_len));
    return (c + waves - 1) / waves * waves;
}

// time slices per term-sum workgroup (0: the blocks do not fit in LDS)
int slices_per_group(int K, int64_t n_sets)
{
    if (K > kMaxLdsKinds) return 0;
    return (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)kMaxTG, kMaxLdsKinds / K, n_sets}));
}

wick_status check_dims(const int32_t dims[4], int32_t n_cfg, int64_t *V)
{
    if (!dims) return fail(WICK_EINVAL, "dims is null");
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 1) return fail(WICK_EINVAL, "dims must be positive");
    if (n_cfg < 1) return fail(WICK_EINVAL, "n_cfg must be >= 1");
    int64_t v = (int64_t)dims[0] * dims[1] * dims[2];
    if (v > (1LL << 30)) return fail(WICK_ETOOBIG, "spatial volume above 2^30");
    if ((int64_t)n_cfg * dims[3] > (1LL << 24)) return fail(WICK_ETOOBIG, "n_cfg * T above 2^24");
    *V = v;
    return WICK_OK;
}

wick_status do_blocks(wick_plan_s *p, const void *Su, const void *Sd, int dtype, const int32_t dims[4], int n_cfg,
                      int prec, hipStream_t s, double *B, int chunk_override = 0)
{
    int64_t V;
    wick_status st = check_dims(dims, n_cfg, &V);
    if (st != WICK_OK) return st;
    if (!Su || !Sd || !B) return fail(WICK_EINVAL, "wick_blocks: null pointer");
    if (((uintptr_t)Su | (uintptr_t)Sd) & 15) return fail(WICK_EINVAL, "wick_blocks: propagators must be 16-byte aligned");
    if (dtype != WICK_C128 && dtype != WICK_C64) return fail(WICK_EINVAL, "wick_blocks: bad dtype");
    if (prec < WICK_P64 || prec > WICK_PB6) return fail(WICK_EINVAL, "wick_blocks: bad precision");
    DevPlan *dp;
    if ((st = device_plan(p, s, &dp)) != WICK_OK) return st;
    Tune tu = tune_for(p, dims, dtype, prec);
    BlockLaunch L{};
    L.Su = Su;
    L.Sd = Sd;
    L.dtype = dtype;
    L.prec = prec;
    L.groups = dp->groups;
    L.n_groups = (int)p->egroups.size();
    L.desc = dp->desc;
    L.n_tiles = dp->n_tiles;
    L.n_passes = dp->n_passes;
    L.nuc = prec == WICK_P64 ? dp->nuc : dp->nuc_split;
    L.nuc_tiles = prec == WICK_P64 ? dp->nuc_tiles : dp->split_tiles;
    L.nuc_passes = prec == WICK_P64 ? dp->nuc_passes : dp->split_passes;
    // WICK_BLOCKS_KERNEL selects a kernel for testing: "generic" (one wave per
    // tile, global loads) or "rows" (staged, general E rows); default: nucleon
    // form when every kind has it, else rows, else generic.
    if (const char *k = std::getenv("WICK_BLOCKS_KERNEL")) {
        if (std::strcmp(k, "generic") == 0) { L.desc = nullptr; L.nuc = nullptr; }
        if (std::strcmp(k, "rows") == 0) L.nuc = nullptr;
    }
    if (prec != WICK_P64 && !L.nuc)
        return fail(WICK_EUNSUPPORTED, "wick_blocks: split precision needs kinds of nucleon form");
    L.V = V;
    L.T = dims[3];
    L.n_cfg = n_cfg;
    L.K = (int)p->kinds.size();
    L.chunk_sites = std::max(4, (chunk_override > 0 ? chunk_override : tu.chunk_sites) / 4 * 4);
    L.n_chunks = (int)((V + L.chunk_sites - 1) / L.chunk_sites);
    L.B = B;
    size_t bytes = (size_t)n_cfg * dims[3] * L.n_chunks * L.K * 1728 * 16;
    void *ws;
    if ((st = workspace(s, bytes, &ws)) != WICK_OK) return st;
    L.partial = (double *)ws;
    hipError_t e = launch_blocks(L, s);
    if (e != hipSuccess) return hip_fail(e, "wick_blocks launch");
    return WICK_OK;
}

// The device copy of a plan on the current device, without building it:
// WICK_EINVAL when it is not there yet (no allocation of any kind).
wick_status resident_plan(wick_plan_s *p, DevPlan **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_dev.find(p);
    if (it != g_dev.end())
        for (auto &d : it->second)
            if (d.device == dev) {
                *out = &d;
                return WICK_OK;
            }
    return fail(WICK_EINVAL, "the plan's table is not on this device yet: call wick_contract (or wick_blocks) "
                             "with it once on this device first");
}

// The term sum. With `fixed` set, the partial sums go to fixed[0 .. cap)
// (bytes) instead of the stream's workspace, the plan must already be on the
// device, and nothing is allocated; a launch needing more than cap bytes of
// partial sums is WICK_ETOOBIG.
wick_status do_contract(wick_plan_s *p, const double *B, int n_cfg, int T, hipStream_t s, double *C,
                        int64_t slice_override = 0, void *fixed = nullptr, size_t cap = 0, int share_override = 0)
{
    if (!B || !C) return fail(WICK_EINVAL, "wick_contract: null pointer");
    if (n_cfg < 1 || T < 1) return fail(WICK_EINVAL, "wick_contract: n_cfg and T must be >= 1");
    DevPlan *dp;
    wick_status st = fixed ? resident_plan(p, &dp) : device_plan(p, s, &dp);
    if (st != WICK_OK) return st;
    const int64_t n_ct = (int64_t)n_cfg * T;
    if (p->n_terms == 0) {
        hipError_t e = launch_zero(C, n_ct * 2, s);
        return e == hipSuccess ? WICK_OK : hip_fail(e, "wick_contract zero fill");
    }
    ContractLaunch L{};
    L.B = B;
    L.tab = table_of(dp, p);
    L.A = p->A;
    L.K = (int)p->kinds.size();
    L.N = p->n_terms;
    L.n_ct = (int)n_ct;
    L.tg = slices_per_group(L.K, n_ct);
    L.share = share_override > 0 ? share_override : tuned_share(p, n_ct);
    const int64_t n_groups = L.tg ? (n_ct + L.tg - 1) / L.tg : n_ct;
    const int64_t sl = slice_override > 0 ? slice_override : tuned_slice(p, n_ct);
    L.slice_len = sl > 0 ? sl : default_slice_len(L.N, n_groups);
    if (dp->seg_prefix) {
        // terms per workgroup -> chunks per workgroup, a multiple of the 16 waves
        L.slice_len = chunks_per_group(L.slice_len, dp->seg_len);
        L.n_slices = (int)((dp->n_chunks + L.slice_len - 1) / L.slice_len);
    } else {
        L.n_slices = (int)((L.N + L.slice_len - 1) / L.slice_len);
    }
    if ((int64_t)L.n_slices * n_groups > 0x7ffffff0LL) return fail(WICK_ETOOBIG, "wick_contract: grid too large");
    void *ws;
    const size_t bytes = (size_t)n_ct * L.n_slices * 16;
    if (fixed) {
        if (bytes > cap)
            return fail(WICK_ETOOBIG, "wick_contract_noalloc: " + std::to_string(n_ct * L.n_slices) +
                                          " partial sums exceed the static scratch of " + std::to_string(cap / 16));
        ws = fixed;
    } else if ((st = workspace(s, bytes, &ws)) != WICK_OK) {
        return st;
    }
    L.partial = (double *)ws;
    L.C = C;
    hipError_t e = launch_contract(L, s);
    if (e != hipSuccess) return hip_fail(e, "wick_contract launch");
    return WICK_OK;
}

// ------------------------------------------------------------- profiling
std::mutex g_prof_mu;
bool g_prof_on = false;
struct ProfRec {
    std::string name;
    hipEvent_t a, b;
};
std::vector<ProfRec> g_prof_pending;
std::map<std::string, std::pair<int64_t, double>> g_prof_done;

void prof_flush_locked()
{
    for (auto &r : g_prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            auto &d = g_prof_done[r.name];
            d.first += 1;
            d.second += ms;
        }
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_prof_pending.clear();
}


// ---------------------------------------------------------------- batches
// A batch of (plan, configuration) items runs as one launch of each kernel
// (blocks, block reduction, term sum, finalize) over device work lists. The
// lists, workspaces and (optionally) a hipGraph of the launches are cached per
// (plans, items, shapes, pointers, stream).
struct BatchEntry {
    int device = -1;
    std::vector<const wick_plan_s *> plans;
    BatchBlockItem *bitems = nullptr;
    BatchBlockWork *bwork = nullptr;
    int64_t *bout = nullptr;
    BatchContractItem *citems = nullptr;
    BatchContractWork *cwork = nullptr;
    void *partial = nullptr, *B = nullptr, *cpartial = nullptr;
    BatchLaunch L{};
    hipStream_t cap = nullptr, cap1 = nullptr;  // capture streams (phase 0, phase 1)
    hipEvent_t fork = nullptr, join = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;  // for least-recently-used eviction
};
std::mutex g_batch_mu;
std::map<std::string, BatchEntry> g_batch;
uint64_t g_batch_clock = 0;
// cached batches (work lists, workspaces, graph) kept at once; the least
// recently used one is released when a new one would exceed this
constexpr size_t kMaxBatchEntries = 8;
thread_local bool t_capturing = false;
thread_local bool t_no_alloc = false;  // inside wick_contract_noalloc: no profiling events

void free_batch(BatchEntry &b)
{
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(b.device);
    (void)hipDeviceSynchronize();
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.graph) (void)hipGraphDestroy(b.graph);
    if (b.cap) (void)hipStreamDestroy(b.cap);
    if (b.cap1) (void)hipStreamDestroy(b.cap1);
    if (b.fork) (void)hipEventDestroy(b.fork);
    if (b.join) (void)hipEventDestroy(b.join);
    for (void *q : {(void *)b.bitems, (void *)b.bwork, (void *)b.bout, (void *)b.citems, (void *)b.cwork, b.partial,
                    b.B, b.cpartial})
        if (q) (void)hipFree(q);
    (void)hipSetDevice(cur);
}

template <class T> wick_status upload(const std::vector<T> &h, T **d)
{
    hipError_t e = hipMalloc((void **)d, std::max<size_t>(1, h.size()) * sizeof(T));
    if (e != hipSuccess) return fail(WICK_ENOMEM, std::string("batch hipMalloc: ") + hipGetErrorString(e));
    if (!h.empty() && (e = hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "batch hipMemcpy");
    return WICK_OK;
}

wick_status build_batch(const wick_plan_t *plans, const wick_item *items, int n_items, const void *S_u,
                        const void *S_d, int dtype, const int32_t dims[4], int64_t V, int prec, int chunk_hint,
                        double *C, BatchEntry &b, int64_t terms_hint = 0, int share = 2)
{
    share = std::max(1, share);
    const int T = dims[3];
    (void)hipGetDevice(&b.device);
    // two phases of about equal work: the items of each plan dealt alternately
    // (internal order: phase 0's items, then phase 1's); C keeps the caller's order
    std::vector<int> order;
    int n_phase0 = 0;
    {
        std::vector<int> byplan(n_items);
        for (int i = 0; i < n_items; ++i) byplan[i] = i;
        std::stable_sort(byplan.begin(), byplan.end(), [&](int x, int y) { return items[x].plan < items[y].plan; });
        for (int pass = 0; pass < 2; ++pass)
            for (int j = pass; j < n_items; j += 2) order.push_back(byplan[j]);
        n_phase0 = (n_items + 1) / 2;
    }
    std::vector<BatchBlockItem> bi(n_items);
    std::vector<BatchBlockWork> bw;
    std::vector<int64_t> bout(n_items + 1, 0);
    std::vector<BatchContractItem> ci(n_items);
    std::vector<BatchContractWork> cw;
    int nt_max = 0, passes_max = 1;
    std::vector<DevPlan *> dps(n_items);
    for (int i = 0; i < n_items; ++i) {
        wick_plan_s *p = plans[items[order[i]].plan];
        wick_status st = device_plan(p, nullptr, &dps[i]);
        if (st != WICK_OK) return st;
        DevPlan *dp = dps[i];
        const NucDesc *nd = prec == WICK_P64 ? dp->nuc : dp->nuc_split;
        if (!nd) return fail(WICK_EUNSUPPORTED, "batched path needs kinds of nucleon form");
        nt_max = std::max(nt_max, prec == WICK_P64 ? dp->nuc_tiles : dp->split_tiles);
        passes_max = std::max(passes_max, prec == WICK_P64 ? dp->nuc_passes : dp->split_passes);
    }
    // sites per chunk: enough workgroups to fill the chip, at least 64 sites each
    int64_t want_chunks = std::max<int64_t>(1, (2048 + (int64_t)n_items * T * passes_max - 1) /
                                                   ((int64_t)n_items * T * passes_max));
    int chunk_sites = chunk_hint > 0 ? chunk_hint
                                     : (int)std::max<int64_t>(64, (V + want_chunks - 1) / want_chunks);
    chunk_sites = (chunk_sites + 7) / 8 * 8;
    const int n_chunks = (int)((V + chunk_sites - 1) / chunk_sites);
    int64_t part = 0, bo = 0, cpart = 0;
    // term sum: terms per workgroup from the whole batch's work (about 2048 workgroups)
    int64_t total = 0;
    size_t clds = 0;
    for (int i = 0; i < n_items; ++i) {
        const wick_plan_s *p = plans[items[order[i]].plan];
        const int tg = slices_per_group((int)p->kinds.size(), T);
        if (tg == 0) return fail(WICK_EUNSUPPORTED, "batch: a plan with more than 12 kinds");
        total += p->n_terms * ((T + tg - 1) / tg);
        clds = std::max(clds, contract_tg_lds_bytes((int)p->kinds.size(), tg));
    }
    // and at most 2^20 terms per workgroup (measured on the 64-configuration batch:
    // 2^20 is 10 % faster than 2^23 and 20 % faster than the uncapped 2^24.4)
    int64_t S = terms_hint > 0 ? terms_hint
                               : std::max<int64_t>(4096, std::min<int64_t>((total + 2047) / 2048, 1 << 20));
    S = (S + kCThreads - 1) / kCThreads * kCThreads;
    BatchPhase ph[2] = {};
    for (int i = 0; i < n_items; ++i) {
        if (i == 0 || i == n_phase0) {
            BatchPhase &P = ph[i == 0 ? 0 : 1];
            P.bw0 = (int)bw.size();
            P.i0 = i;
            P.bout0 = bo;
            P.cw0 = (int)cw.size();
        }
        wick_plan_s *p = plans[items[order[i]].plan];
        DevPlan *dp = dps[i];
        const int K = (int)p->kinds.size();
        const int passes = prec == WICK_P64 ? dp->nuc_passes : dp->split_passes;
        bi[i].desc = prec == WICK_P64 ? dp->nuc : dp->nuc_split;
        bi[i].s_off = (int64_t)items[order[i]].cfg * T * V * 144;
        bi[i].part_off = part;
        bi[i].b_off = bo;
        bi[i].K = K;
        bi[i].n_chunks = n_chunks;
        part += (int64_t)T * n_chunks * K * 1728;
        bout[i] = bo;
        bo += (int64_t)T * K * 792;
        for (int t = 0; t < T; ++t)
            for (int ch = 0; ch < n_chunks; ++ch)
                for (int ps = 0; ps < passes; ++ps) bw.push_back({i, t, ch, ps});
        BatchContractItem &c = ci[i];
        c.tab = table_of(dp, p);
        c.N = p->n_terms;
        if (dp->seg_prefix) {
            c.slice_len = chunks_per_group(S, dp->seg_len);
            c.n_slices = (int)std::max<int64_t>(1, (dp->n_chunks + c.slice_len - 1) / c.slice_len);
        } else {
            c.slice_len = S;
            c.n_slices = (int)std::max<int64_t>(1, (c.N + S - 1) / S);
        }
        c.b_off = bi[i].b_off;
        c.part_off = cpart;
        c.A = p->A;
        c.K = K;
        c.tg = slices_per_group(K, T);
        c.out_item = order[i];
        cpart += (int64_t)T * c.n_slices;
        // `share` groups of time slices take each table slice together (adjacent
        // workgroups, one XCD: the slice is shared through its L2), then the
        // next `share` groups (see contract_tg_kernel)
        const int n_tgroups = (T + c.tg - 1) / c.tg;
        for (int g0 = 0; g0 < n_tgroups; g0 += share)
            for (int sl = 0; sl < c.n_slices; ++sl)
                for (int gg = g0; gg < std::min(n_tgroups, g0 + share); ++gg) {
                    const int t0 = gg * c.tg;
                    cw.push_back({i, t0, sl, std::min(c.tg, T - t0)});
                }
        if (i + 1 == n_phase0 || i + 1 == n_items) {
            BatchPhase &P = ph[i + 1 == n_phase0 ? 0 : 1];
            P.nbw = (int)bw.size() - P.bw0;
            P.ni = i + 1 - P.i0;
            P.nbout = bo - P.bout0;
            P.ncw = (int)cw.size() - P.cw0;
        }
    }
    bout[n_items] = bo;
    if (bw.size() > 0x7ffffff0ULL || cw.size() > 0x7ffffff0ULL) return fail(WICK_ETOOBIG, "batch too large");
    wick_status st;
    if ((st = upload(bi, &b.bitems)) != WICK_OK || (st = upload(bw, &b.bwork)) != WICK_OK ||
        (st = upload(bout, &b.bout)) != WICK_OK || (st = upload(ci, &b.citems)) != WICK_OK ||
        (st = upload(cw, &b.cwork)) != WICK_OK)
        return st;
    hipError_t e;
    if ((e = hipMalloc(&b.partial, std::max<int64_t>(1, part) * 16)) != hipSuccess ||
        (e = hipMalloc(&b.B, std::max<int64_t>(1, bo) * 16)) != hipSuccess ||
        (e = hipMalloc(&b.cpartial, std::max<int64_t>(1, cpart) * 16)) != hipSuccess)
        return fail(WICK_ENOMEM, std::string("batch workspace hipMalloc: ") + hipGetErrorString(e));
    BatchLaunch &L = b.L;
    L.ph[0] = ph[0];
    L.ph[1] = ph[1];
    L.Su = S_u;
    L.Sd = S_d;
    L.dtype = dtype;
    L.prec = prec;
    L.nt_max = nt_max;
    L.V = V;
    L.T = T;
    L.chunk_sites = chunk_sites;
    L.n_items = n_items;
    L.bitems = b.bitems;
    L.bwork = b.bwork;
    L.n_bwork = (int)bw.size();
    L.bout_off = b.bout;
    L.n_bout = bo;
    L.citems = b.citems;
    L.cwork = b.cwork;
    L.n_cwork = (int)cw.size();
    L.contract_lds = clds;
    L.partial = (double *)b.partial;
    L.B = (double *)b.B;
    L.cpartial = (double *)b.cpartial;
    L.C = C;
    return WICK_OK;
}
// ------------------------------------------------------------- autotuning
// Cache file: a header line, then one line per tuned shape,
//   "blocks <shape key> <chunk_sites> <batch_chunk_sites>" or "contract <table key> <slice_len>".
const char *kTuneHeader = "wick-tune 1";

wick_status load_tune_file(const char *path)
{
    std::ifstream f(path);
    if (!f) return WICK_OK;  // no cache yet
    std::string line;
    if (!std::getline(f, line) || line != kTuneHeader)
        return fail(WICK_ECORRUPT, std::string("tune cache ") + path + ": bad header");
    std::map<std::string, Tune> tb;
    std::map<std::string, int64_t> ts;
    std::map<std::string, BatchTune> tbt;
    std::map<std::string, int> tsh;
    int ln = 1;
    while (std::getline(f, line)) {
        ++ln;
        if (line.empty()) continue;
        std::istringstream is(line);
        std::string what, key, extra;
        bool ok = static_cast<bool>(is >> what >> key);
        if (ok && what == "blocks") {
            Tune t;
            ok = static_cast<bool>(is >> t.chunk_sites >> t.batch_chunk_sites) && t.chunk_sites >= 4 &&
                 t.chunk_sites <= (1 << 24) && t.batch_chunk_sites >= 0 && t.batch_chunk_sites <= (1 << 24);
            if (ok) tb[key] = t;
        } else if (ok && what == "batch") {
            BatchTune bt;
            ok = static_cast<bool>(is >> bt.chunk >> bt.terms >> bt.share) && bt.chunk >= 4 && bt.chunk <= (1 << 24) &&
                 bt.terms >= 1024 && bt.terms <= (1LL << 30) && bt.share >= 1 && bt.share <= 64;
            if (ok) tbt[key] = bt;
        } else if (ok && what == "share") {
            int v = 0;
            ok = static_cast<bool>(is >> v) && v >= 1 && v <= 64;
            if (ok) tsh[key] = v;
        } else if (ok && what == "contract") {
            int64_t v = 0;
            ok = static_cast<bool>(is >> v) && v >= 1 && v <= (1LL << 30);  // terms or chunks per workgroup
            if (ok) ts[key] = v;
        } else {
            ok = false;
        }
        if (!ok || (is >> extra))
            return fail(WICK_ECORRUPT, std::string("tune cache ") + path + ": bad line " + std::to_string(ln));
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &kv : tb) g_tune[kv.first] = kv.second;
    for (auto &kv : ts) g_slice[kv.first] = kv.second;
    for (auto &kv : tbt) g_batch_tune[kv.first] = kv.second;
    for (auto &kv : tsh) g_share[kv.first] = kv.second;
    return WICK_OK;
}

wick_status save_tune_file(const char *path)
{
    const std::string tmp = std::string(path) + ".tmp";
    {
        std::ofstream f(tmp, std::ios::trunc);
        if (!f) return fail(WICK_EINVAL, std::string("cannot write tune cache ") + tmp);
        std::lock_guard<std::mutex> lk(g_tune_mu);
        f << kTuneHeader << "\n";
        for (auto &kv : g_tune) f << "blocks " << kv.first << ' ' << kv.second.chunk_sites << ' '
                                  << kv.second.batch_chunk_sites << "\n";
        for (auto &kv : g_slice) f << "contract " << kv.first << ' ' << kv.second << "\n";
        for (auto &kv : g_share) f << "share " << kv.first << ' ' << kv.second << "\n";
        for (auto &kv : g_batch_tune)
            f << "batch " << kv.first << ' ' << kv.second.chunk << ' ' << kv.second.terms << ' ' << kv.second.share
              << "\n";
        if (!f) return fail(WICK_EINVAL, std::string("cannot write tune cache ") + tmp);
    }
    if (std::rename(tmp.c_str(), path) != 0) return fail(WICK_EINVAL, std::string("cannot replace ") + path);
    return WICK_OK;
}

// Average time of `reps` back-to-back runs of f on s, after one untimed run.
template <class F> wick_status time_runs(hipStream_t s, int reps, F f, float *ms)
{
    wick_status st = f();
    if (st != WICK_OK) return st;
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return hip_fail(e, "autotune hipEventCreate");
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "autotune hipEventCreate");
    }
    (void)hipEventRecord(a, s);
    for (int r = 0; r < reps && st == WICK_OK; ++r) st = f();
    (void)hipEventRecord(b, s);
    e = hipEventSynchronize(b);
    float t = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != WICK_OK) return st;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    *ms = t / reps;
    return WICK_OK;
}

// Device scratch of one autotune call, released on every exit path.
struct TuneScratch {
    void *Su = nullptr, *Sd = nullptr, *B = nullptr, *C = nullptr;
    hipStream_t s = nullptr;
    ~TuneScratch()
    {
        if (s) {
            (void)hipStreamSynchronize(s);
            release_workspace(s);
            (void)hipStreamDestroy(s);
        }
        for (void *q : {Su, Sd, B, C})
            if (q) (void)hipFree(q);
    }
};

wick_status autotune(wick_plan_s *p, const int32_t dims[4], int dtype, int prec, const char *cache_path)
{
    int64_t V;
    wick_status st = check_dims(dims, 1, &V);
    if (st != WICK_OK) return st;
    if (dtype != WICK_C128 && dtype != WICK_C64) return fail(WICK_EINVAL, "wick_autotune: bad dtype");
    if (prec < WICK_P64 || prec > WICK_PB6) return fail(WICK_EINVAL, "wick_autotune: bad precision");
    if (cache_path && (st = load_tune_file(cache_path)) != WICK_OK) return st;
    const int T = dims[3];
    const std::string key = tune_key(p, dims, dtype, prec), skey = slice_key(p, T);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune.count(key) && (p->n_terms == 0 || g_slice.count(skey))) return WICK_OK;
    }
    // one configuration of constant, nonzero propagators (timing does not depend on the values)
    TuneScratch sc;
    const int K = (int)p->kinds.size();
    const size_t esz = dtype == WICK_C128 ? 16 : 8, n_prop = (size_t)V * T * 144 * esz;
    hipError_t e;
    if ((e = hipMalloc(&sc.Su, n_prop)) != hipSuccess || (e = hipMalloc(&sc.Sd, n_prop)) != hipSuccess ||
        (e = hipMalloc(&sc.B, (size_t)T * K * kBlockLen * 16)) != hipSuccess ||
        (e = hipMalloc(&sc.C, (size_t)T * 16)) != hipSuccess)
        return fail(WICK_ENOMEM, std::string("wick_autotune hipMalloc: ") + hipGetErrorString(e));
    const uint32_t pattern = dtype == WICK_C128 ? 0x3fe00000u : 0x3f000000u;  // ~0.5 in every real and imaginary part
    if ((e = hipMemsetD32((hipDeviceptr_t)sc.Su, (int)pattern, n_prop / 4)) != hipSuccess ||
        (e = hipMemsetD32((hipDeviceptr_t)sc.Sd, (int)pattern, n_prop / 4)) != hipSuccess ||
        (e = hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "wick_autotune setup");

    // block kernel: sites per workgroup (bounded by a 4 GiB split-K workspace)
    const int cand[] = {32, 64, 128, 256, 512, 1024, 2048, 4096};
    int best_chunk = 0;
    float best = 0.f;
    for (int c : cand) {
        if (c >= 2 * V && c != cand[0]) break;  // larger chunks than twice the volume change nothing
        const int64_t n_chunks = (V + c - 1) / c;
        if ((double)T * n_chunks * K * 1728 * 16 > 4.0 * (1ull << 30)) continue;
        float ms = 0.f;
        st = time_runs(sc.s, 3, [&] {
            return do_blocks(p, sc.Su, sc.Sd, dtype, dims, 1, prec, sc.s, (double *)sc.B, c);
        }, &ms);
        if (st != WICK_OK) return st;
        if (!best_chunk || ms < best) { best = ms; best_chunk = c; }
    }
    if (!best_chunk) return fail(WICK_ETOOBIG, "wick_autotune: no site chunk fits the workspace bound");

    // term sum: terms per workgroup
    int64_t best_slice = 0;
    int best_share = 1;
    if (p->n_terms > 0) {
        if ((st = do_blocks(p, sc.Su, sc.Sd, dtype, dims, 1, prec, sc.s, (double *)sc.B, best_chunk)) != WICK_OK)
            return st;
        const int64_t scand[] = {4096, 16384, 65536, 262144, 1048576, 4194304};
        best = 0.f;
        for (int64_t sl : scand) {
            if (sl >= 2 * p->n_terms && sl != scand[0]) break;
            float ms = 0.f;
            st = time_runs(sc.s, 3, [&] { return do_contract(p, (const double *)sc.B, 1, T, sc.s, (double *)sc.C, sl); },
                           &ms);
            if (st != WICK_OK) return st;
            if (!best_slice || ms < best) { best = ms; best_slice = sl; }
        }
        // then how many groups of slices read one table slice together
        for (int h : {2, 4}) {
            if (h > (T + 2) / 3) break;  // fewer groups of slices than h
            float ms = 0.f;
            st = time_runs(sc.s, 3, [&] {
                return do_contract(p, (const double *)sc.B, 1, T, sc.s, (double *)sc.C, best_slice, nullptr, 0, h);
            }, &ms);
            if (st != WICK_OK) return st;
            if (ms < best) { best = ms; best_share = h; }
        }
    }

    // batched launch of this plan alone: sites per workgroup (plans without nucleon form have no batched path)
    int best_batch = 0;
    best = 0.f;
    wick_plan_t plist[1] = {p};
    const wick_item item{0, 0};
    for (int c : cand) {
        if (c < 64) continue;
        if (c >= 2 * V) break;
        BatchEntry b;
        st = build_batch(plist, &item, 1, sc.Su, sc.Sd, dtype, dims, V, prec, c, (double *)sc.C, b);
        if (st == WICK_EUNSUPPORTED) { free_batch(b); best_batch = 0; break; }
        if (st != WICK_OK) { free_batch(b); return st; }
        float ms = 0.f;
        st = time_runs(sc.s, 3, [&] {
            hipError_t le = launch_batch(b.L, sc.s);
            return le == hipSuccess ? WICK_OK : hip_fail(le, "wick_autotune batch launch");
        }, &ms);
        free_batch(b);
        if (st != WICK_OK) return st;
        if (!best_batch || ms < best) { best = ms; best_batch = c; }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = Tune{best_chunk, best_batch};
        if (best_slice > 0) g_slice[skey] = best_slice;
        if (best_slice > 0) g_share[skey] = best_share;
    }
    return cache_path ? save_tune_file(cache_path) : WICK_OK;
}

// Arguments of a batched call (wick_correlator, wick_autotune_batch).
wick_status check_batch(const wick_plan_t *plans, int n_plans, const wick_item *items, int n_items, const void *S_u,
                        const void *S_d, int dtype, const int32_t dims[4], int n_cfg, int prec, int64_t *V)
{
    if (!plans || n_plans < 1 || !items || n_items < 1 || !S_u || !S_d)
        return fail(WICK_EINVAL, "batch: bad plans / items / pointers");
    if (((uintptr_t)S_u | (uintptr_t)S_d) & 15) return fail(WICK_EINVAL, "batch: propagators must be 16-byte aligned");
    wick_status st = check_dims(dims, n_cfg, V);
    if (st != WICK_OK) return st;
    if (dtype != WICK_C128 && dtype != WICK_C64) return fail(WICK_EINVAL, "batch: bad dtype");
    if (prec < WICK_P64 || prec > WICK_PB6) return fail(WICK_EINVAL, "batch: bad precision");
    for (int i = 0; i < n_plans; ++i)
        if (!plans[i]) return fail(WICK_EINVAL, "batch: null plan");
    for (int i = 0; i < n_items; ++i)
        if (items[i].plan < 0 || items[i].plan >= n_plans || items[i].cfg < 0 || items[i].cfg >= n_cfg)
            return fail(WICK_EINVAL, "batch: item index out of range");
    return WICK_OK;
}

// A batched launch tuned as a whole on the caller's propagators: the block
// kernel's sites per workgroup (one site chunk per (item, t) down to
// sixteen), then the term sum's terms per workgroup (2^16 .. 2^22), each by
// timing eager launches of the whole batch (blocking, on a stream of its own).
wick_status autotune_batch(const wick_plan_t *plans, int n_plans, const wick_item *items, int n_items,
                           const void *S_u, const void *S_d, int dtype, const int32_t dims[4], int n_cfg, int prec,
                           const char *cache_path)
{
    int64_t V;
    wick_status st = check_batch(plans, n_plans, items, n_items, S_u, S_d, dtype, dims, n_cfg, prec, &V);
    if (st != WICK_OK) return st;
    if (cache_path && (st = load_tune_file(cache_path)) != WICK_OK) return st;
    const std::string key = batch_key(plans, items, n_items, dims, dtype, prec);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_batch_tune.count(key)) return WICK_OK;
    }
    TuneScratch sc;
    hipError_t e;
    if ((e = hipMalloc(&sc.C, (size_t)n_items * dims[3] * 16)) != hipSuccess)
        return fail(WICK_ENOMEM, std::string("wick_autotune_batch hipMalloc: ") + hipGetErrorString(e));
    if ((e = hipStreamCreateWithFlags(&sc.s, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "wick_autotune_batch stream");
    auto run = [&](int chunk, int64_t terms, int share, float *ms) {
        BatchEntry b;
        wick_status r = build_batch(plans, items, n_items, S_u, S_d, dtype, dims, V, prec, chunk, (double *)sc.C, b,
                                    terms, share);
        if (r == WICK_OK)
            r = time_runs(sc.s, 2, [&] {
                hipError_t le = launch_batch(b.L, sc.s);
                return le == hipSuccess ? WICK_OK : hip_fail(le, "wick_autotune_batch launch");
            }, ms);
        free_batch(b);
        return r;
    };
    int best_chunk = 0;
    float best = 0.f;
    for (int div = 1; div <= 16; div *= 2) {
        const int c = (int)((V + div - 1) / div + 7) / 8 * 8;
        if (div > 1 && c < 256) break;
        float ms = 0.f;
        if ((st = run(c, 0, 2, &ms)) != WICK_OK) return st;
        if (!best_chunk || ms < best) { best = ms; best_chunk = c; }
    }
    int64_t best_terms = 0;
    best = 0.f;
    for (int64_t S = 1 << 16; S <= (1 << 22); S *= 2) {
        float ms = 0.f;
        if ((st = run(best_chunk, S, 2, &ms)) != WICK_OK) return st;
        if (!best_terms || ms < best) { best = ms; best_terms = S; }
    }
    // groups of time slices that take a table slice together
    int best_share = 2;
    for (int h : {1, 4, 16}) {
        float ms = 0.f;
        if ((st = run(best_chunk, best_terms, h, &ms)) != WICK_OK) return st;
        if (ms < best) { best = ms; best_share = h; }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_batch_tune[key] = BatchTune{best_chunk, best_terms, best_share};
    }
    return cache_path ? save_tune_file(cache_path) : WICK_OK;
}
}  // namespace

Probe::Probe(const char *n, hipStream_t st) : name(n), s(st)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (!g_prof_on || t_capturing || t_no_alloc) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) { a = b = nullptr; return; }
    (void)hipEventRecord(a, s);
}

void Probe::stop()
{
    if (!a) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_pending.push_back({name, a, b});
    a = b = nullptr;
}

void release_device_tables(wick_plan_s *p)
{
    release_plain_tables(p);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    g_work.erase(p);
    auto it = g_dev.find(p);
    if (it == g_dev.end()) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &d : it->second) {
        (void)hipSetDevice(d.device);
        (void)hipDeviceSynchronize();
        (void)hipFree(d.groups);
        (void)hipFree(d.desc);
        (void)hipFree(d.nuc);
        (void)hipFree(d.nuc_split);
        (void)hipFree(d.kidx);
        (void)hipFree(d.coef);
        (void)hipFree(d.words);
        (void)hipFree(d.pal);
        (void)hipFree(d.seg_prefix);
        (void)hipFree(d.chunk_base);
        (void)hipFree(d.chunk_len);
        (void)hipFree(d.chunk_g);
    }
    (void)hipSetDevice(cur);
    g_dev.erase(it);
    g_work.erase(p);
}

}  // namespace wick

wick_plan_s::~wick_plan_s() {}

using namespace wick;

#define WICK_TRY(expr)                                              \
    try {                                                           \
        expr;                                                       \
    } catch (const std::bad_alloc &) {                              \
        return fail(WICK_ENOMEM, "out of host memory");             \
    } catch (const std::exception &ex) {                            \
        return fail(WICK_EINVAL, std::string("internal: ") + ex.what()); \
    } catch (...) {                                                 \
        return fail(WICK_EINVAL, "internal error");                 \
    }

// ------------------------------------------- allocation-free term sum
// The partial sums of wick_contract_noalloc live in this static device array
// (one copy per GPU, kept until the process ends). Host code never uses its
// name as an address: the device address of each GPU's copy is looked up
// once per device with hipGetSymbolAddress and used from then on.
namespace {
constexpr size_t kScratchPartials = 131072;  // complex FP64 partial sums: 2 MiB
__device__ __align__(256) double2 scratch[kScratchPartials];
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxScratchDevices] = {};

wick_status noalloc_scratch(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxScratchDevices) return fail(WICK_EUNSUPPORTED, "wick_contract_noalloc: device index");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return WICK_OK;
}
}  // namespace

extern "C" {

wick_status wick_plan(const wick_nucleus_desc *desc, wick_plan_t *out) { WICK_TRY(return build_plan(desc, out)); }

wick_status wick_plan_std(const char *nucleus, int32_t J, wick_plan_t *out) { WICK_TRY(return std_plan(nucleus, J, out)); }

wick_status wick_plan_std_pair(const char *sink, int32_t J_sink, const char *source, int32_t J_source, wick_plan_t *out)
{
    WICK_TRY(return std_pair_plan(sink, J_sink, source, J_source, out));
}

wick_status wick_plan_info(wick_plan_t p, int32_t *A, int32_t *n_kinds, int64_t *n_terms)
{
    if (!p) return fail(WICK_EINVAL, "wick_plan_info: null plan");
    if (A) *A = p->A;
    if (n_kinds) *n_kinds = (int32_t)p->kinds.size();
    if (n_terms) *n_terms = p->n_terms;
    return WICK_OK;
}

wick_status wick_plan_stats(wick_plan_t p, int64_t *n_enum, int64_t *n_groups, int64_t *n_terms, double *bound)
{
    if (!p) return fail(WICK_EINVAL, "wick_plan_stats: null plan");
    if (n_enum) *n_enum = p->n_enumerated;
    if (n_groups) *n_groups = p->n_groups;
    if (n_terms) *n_terms = p->n_terms;
    if (bound) *bound = p->bound;
    return WICK_OK;
}

wick_status wick_plan_sum_work(wick_plan_t p, int32_t *form, int64_t *words2, int64_t *words1, int64_t *segments)
{
    if (!p) return fail(WICK_EINVAL, "wick_plan_sum_work: null plan");
    TableWork w;
    WICK_TRY(w = wick::plan_work(p));
    if (form) *form = w.form;
    if (words2) *words2 = w.w2;
    if (words1) *words1 = w.w1;
    if (segments) *segments = w.segs;
    return WICK_OK;
}

wick_status wick_plan_table(wick_plan_t p, uint16_t *kidx, double *coef)
{
    if (!p) return fail(WICK_EINVAL, "wick_plan_table: null plan");
    if (kidx) std::memcpy(kidx, p->kidx.data(), p->kidx.size() * sizeof(uint16_t));
    if (coef)
        for (int64_t n = 0; n < p->n_terms; ++n) {
            coef[2 * n] = p->coef_re[n];
            coef[2 * n + 1] = p->coef_im[n];
        }
    return WICK_OK;
}

wick_status wick_plan_kind(wick_plan_t p, int32_t k, int32_t flavor[3], int32_t *n_w, int8_t *j, int64_t *w_re,
                           int64_t *w_im)
{
    if (!p || k < 0 || k >= (int32_t)p->kinds.size()) return fail(WICK_EINVAL, "wick_plan_kind: bad plan or kind");
    const KindDef &kd = p->kinds[k];
    if (flavor)
        for (int s = 0; s < 3; ++s) flavor[s] = kd.flav[s];
    if (n_w) *n_w = (int32_t)kd.w.size();
    for (size_t e = 0; e < kd.w.size(); ++e) {
        if (j)
            for (int s = 0; s < 3; ++s) j[3 * e + s] = kd.j[e][s];
        if (w_re) w_re[e] = kd.w[e].re;
        if (w_im) w_im[e] = kd.w[e].im;
    }
    return WICK_OK;
}

wick_status wick_plan_save(wick_plan_t p, const char *path) { WICK_TRY(return save_plan(p, path)); }

wick_status wick_plan_load(const char *path, wick_plan_t *out) { WICK_TRY(return load_plan(path, out)); }

wick_status wick_plan_truncate(wick_plan_t p, const double *B_cal, int32_t n_slices, double keep_fraction,
                               wick_plan_t *out, double *dropped)
{
    WICK_TRY(return truncate_plan(p, B_cal, n_slices, keep_fraction, out, dropped));
}

void wick_plan_destroy(wick_plan_t p)
{
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_batch_mu);
        for (auto it = g_batch.begin(); it != g_batch.end();) {
            if (std::find(it->second.plans.begin(), it->second.plans.end(), p) != it->second.plans.end()) {
                free_batch(it->second);
                it = g_batch.erase(it);
            } else {
                ++it;
            }
        }
    }
    release_device_tables(p);
    delete p;
}

wick_status wick_blocks(wick_plan_t p, const void *S_u, const void *S_d, wick_dtype dtype, const int32_t dims[4],
                        int32_t n_cfg, wick_precision prec, wick_stream_t stream, double *B)
{
    if (!p) return fail(WICK_EINVAL, "wick_blocks: null plan");
    WICK_TRY(return do_blocks(p, S_u, S_d, (int)dtype, dims, n_cfg, (int)prec, (hipStream_t)stream, B));
}

wick_status wick_contract(wick_plan_t p, const double *B, int32_t n_cfg, int32_t T, wick_stream_t stream, double *C)
{
    if (!p) return fail(WICK_EINVAL, "wick_contract: null plan");
    WICK_TRY(return do_contract(p, B, n_cfg, T, (hipStream_t)stream, C));
}

wick_status wick_contract_noalloc(wick_plan_t p, const double *B, int32_t n_cfg, int32_t T, wick_stream_t stream,
                                  double *C)
{
    if (!p) return fail(WICK_EINVAL, "wick_contract_noalloc: null plan");
    void *ptr = nullptr;
    wick_status st = noalloc_scratch(&ptr);
    if (st != WICK_OK) return st;
    t_no_alloc = true;
    try {
        st = do_contract(p, B, n_cfg, T, (hipStream_t)stream, C, 0, ptr, kScratchPartials * sizeof(double2));
    } catch (...) {
        st = fail(WICK_EINVAL, "wick_contract_noalloc: internal error");
    }
    t_no_alloc = false;
    return st;
}

wick_status wick_correlator(const wick_plan_t *plans, int32_t n_plans, const wick_item *items, int32_t n_items,
                            const void *S_u, const void *S_d, wick_dtype dtype, const int32_t dims[4], int32_t n_cfg,
                            wick_precision prec, int32_t use_graph, wick_stream_t stream, double *C)
{
    if (!C) return fail(WICK_EINVAL, "wick_correlator: null output");
    int64_t V;
    wick_status st = check_batch(plans, n_plans, items, n_items, S_u, S_d, (int)dtype, dims, n_cfg, (int)prec, &V);
    if (st != WICK_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::ostringstream key;
    key << dev << ':' << (const void *)s << ':' << S_u << ':' << S_d << ':' << (const void *)C << ':' << dims[0] << 'x'
        << dims[1] << 'x' << dims[2] << 'x' << dims[3] << ':' << n_cfg << ':' << (int)dtype << ':' << (int)prec << ':'
        << (use_graph ? 1 : 0);
    for (int i = 0; i < n_plans; ++i) key << ':' << (const void *)plans[i];
    for (int i = 0; i < n_items; ++i) key << ';' << items[i].plan << ',' << items[i].cfg;
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto it = g_batch.find(key.str());
    if (it == g_batch.end()) {
        while (g_batch.size() >= kMaxBatchEntries) {
            auto lru = g_batch.begin();
            for (auto jt = g_batch.begin(); jt != g_batch.end(); ++jt)
                if (jt->second.last_use < lru->second.last_use) lru = jt;
            free_batch(lru->second);  // waits for the device first
            g_batch.erase(lru);
        }
        BatchEntry b;
        // launch shape: tuned for this batch (wick_autotune_batch), else the
        // first plan's batched block shape and the default term split
        BatchTune bt;
        bt.chunk = tune_for(plans[0], dims, (int)dtype, (int)prec).batch_chunk_sites;
        (void)tuned_batch(batch_key(plans, items, n_items, dims, (int)dtype, (int)prec), &bt);
        WICK_TRY(st = build_batch(plans, items, n_items, S_u, S_d, (int)dtype, dims, V, (int)prec, bt.chunk, C, b,
                                  bt.terms, bt.share));
        if (st != WICK_OK) {
            free_batch(b);
            return st;
        }
        for (int i = 0; i < n_plans; ++i) b.plans.push_back(plans[i]);
        if (use_graph) {
            hipError_t e;
            // the two phases as two branches: phase 1's blocks run beside
            // phase 0's term sum (default-priority streams only)
            if ((e = hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking)) != hipSuccess ||
                (e = hipStreamCreateWithFlags(&b.cap1, hipStreamNonBlocking)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&b.fork, hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&b.join, hipEventDisableTiming)) != hipSuccess ||
                (e = hipStreamBeginCapture(b.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
                free_batch(b);
                return hip_fail(e, "wick_correlator: graph capture");
            }
            t_capturing = true;
            hipError_t le = launch_batch_forked(b.L, b.cap, b.cap1, b.fork, b.join);
            t_capturing = false;
            e = hipStreamEndCapture(b.cap, &b.graph);
            if (le != hipSuccess || e != hipSuccess ||
                (e = hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0)) != hipSuccess) {
                free_batch(b);
                return hip_fail(le != hipSuccess ? le : e, "wick_correlator: graph capture");
            }
        }
        it = g_batch.emplace(key.str(), b).first;
    }
    it->second.last_use = ++g_batch_clock;
    Probe pr("correlator", s);
    hipError_t e = it->second.exec ? hipGraphLaunch(it->second.exec, s) : launch_batch(it->second.L, s);
    pr.stop();
    if (e != hipSuccess) return hip_fail(e, "wick_correlator launch");
    return WICK_OK;
}

wick_status wick_autotune(wick_plan_t p, const int32_t dims[4], wick_dtype dtype, wick_precision prec,
                          const char *cache_path)
{
    if (!p) return fail(WICK_EINVAL, "wick_autotune: null plan");
    WICK_TRY(return autotune(p, dims, (int)dtype, (int)prec, cache_path));
}

wick_status wick_autotune_batch(const wick_plan_t *plans, int32_t n_plans, const wick_item *items, int32_t n_items,
                                const void *S_u, const void *S_d, wick_dtype dtype, const int32_t dims[4],
                                int32_t n_cfg, wick_precision prec, const char *cache_path)
{
    WICK_TRY(return autotune_batch(plans, n_plans, items, n_items, S_u, S_d, (int)dtype, dims, n_cfg, (int)prec,
                                   cache_path));
}

wick_status wick_shutdown(void)
{
    {
        std::lock_guard<std::mutex> lb(g_batch_mu);
        for (auto &kv : g_batch) free_batch(kv.second);
        g_batch.clear();
    }
    std::lock_guard<std::mutex> lk(g_ws_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &kv : g_ws) {
        (void)hipSetDevice(std::get<0>(kv.first));
        (void)hipStreamSynchronize(std::get<1>(kv.first));
        (void)hipFree(kv.second.ptr);
    }
    (void)hipSetDevice(cur);
    g_ws.clear();
    return WICK_OK;
}

wick_status wick_profile(int32_t enable)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    if (enable) {
        prof_flush_locked();
        g_prof_done.clear();
    }
    g_prof_on = enable != 0;
    return WICK_OK;
}

wick_status wick_profile_read(const char *kernel, int64_t *launches, double *total_ms)
{
    if (!kernel) return fail(WICK_EINVAL, "wick_profile_read: null name");
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof_flush_locked();
    auto it = g_prof_done.find(kernel);
    if (launches) *launches = it == g_prof_done.end() ? 0 : it->second.first;
    if (total_ms) *total_ms = it == g_prof_done.end() ? 0.0 : it->second.second;
    return WICK_OK;
}

const char *wick_last_error(void) { return g_last_error.c_str(); }

const char *wick_version(void) { return "wick-mi355x 0.1 (gfx950)"; }

}  // extern "C"
