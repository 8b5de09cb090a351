// Point-sink correlators by determinants (Sec. 3.1 Eq. 2.9, App. A Eq. A1):
// device tables, kernels and the wick_point_correlator entry point.
//
// Per site-slice (configuration, t, x) the minimal set is every
// det S_f[R; K] for a sink row set R and a source column set K of flavor f.
// Instead of one factorisation per determinant, all minors of the rows R are
// built by Laplace expansion along the last row, level by level over the
// column subsets: the k x k minors of rows R[0..k) are
//   M_k(c) = sum_j (-1)^(k-1+j) S[R[k-1]][c_j] M_{k-1}(c \ c_j)
// for every k-subset c of the 12 columns (colex-ranked). Level n holds
// det S[R; K] for every column set K at once; building all levels costs
// sum_k binom(12,k) k complex multiply-adds per row set (6744 for n = 5),
// a few per determinant, and is division-free.
//
// Row sets are sorted, so a workgroup's consecutive row sets often share
// their first n-1 rows: levels 1..n-1 are then kept, and level n is formed
// only for the column sets the source uses.
//
// Kernels (one site-slice per "slot"):
//   pt_minors_kernel: the d determinants of every sink row set at the source
//     column sets, to a workspace [slot][row set][column set].
//   pt_pairs_kernel: the u determinants of a chunk of sink row sets in LDS, then
//     for every sink group g of those row sets the sum over source groups h
//     of W'_h det_u[U_g; U'_h] det_d[D_g; D'_h], times W_g (the Theta-weighted
//     double sum of Eq. A1), into one partial per (slot, chunk).
//   pt_reduce_kernel: C[cfg][t] = scale * the sum of the partials of its slots
//     in a fixed order (deterministic).
// The host walks the site-slices in chunks that bound the d workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace wick {

wick_status workspace(hipStream_t s, size_t bytes, void **out);
wick_status workspace(hipStream_t s, size_t bytes, void **out, int tag);

namespace {

constexpr int kPtThreads = 256;
constexpr int kPtSubsets = 2509;    // sum_{k=1..6} binom(12, k)
constexpr int kPtRowsPerWG = 8;     // sink row sets per workgroup

__host__ __device__ constexpr int binom12c(int k)
{
    int r = 1;
    for (int i = 0; i < k; ++i) r = r * (12 - i) / (i + 1);
    return r;
}
__host__ __device__ constexpr int level_off(int k)
{
    int o = 0;
    for (int i = 1; i < k; ++i) o += binom12c(i);
    return o;
}

// One subset of level k (1..6), entry level_off(k) + colex rank: its elements
// (4 bits each) and, for each element j, the colex rank of the subset without
// it (a (k-1)-subset). 16 bytes, read with one vector load.
struct alignas(16) PtSubset {
    uint32_t elems;
    uint16_t sub[6];
};

struct PtDev {
    int device = -1;
    PtSubset *sub = nullptr;
    int8_t *rows_u = nullptr, *rows_d = nullptr;   // [n][8]
    int32_t *u_beg = nullptr, *g_d = nullptr;
    double2 *g_w = nullptr;
    uint16_t *h_ru = nullptr;                      // source groups sorted by d column: compact u column
    double2 *h_w = nullptr;                        // and weight
    int32_t *cd_beg = nullptr;                     // [n_cd + 1] source groups of each d column
    uint16_t *d_cols = nullptr, *u_cols = nullptr; // compact column index -> colex rank
    int n_cd = 0, n_cu = 0;
};

struct PtArgs {
    const PtSubset *sub;
    const int8_t *rows_u, *rows_d;
    const int32_t *u_beg, *g_d;
    const double2 *g_w;
    const uint16_t *h_ru, *d_cols, *u_cols;  // h_ru: compact u column of each source group
    const int32_t *cd_beg;
    const double2 *h_w;
    int n_u, n_d, n_rows_u, n_rows_d, n_h, n_cd, n_cu;
    int n_uchunks, n_dchunks;
    int64_t slot0;       // first site-slice of this launch
    int n_slots;         // site-slices in this launch
    double2 *dd;         // [n_slots][n_rows_d][n_cd]
    double2 *partial;    // [total slots][n_uchunks]
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ int xcd_id(int nb)
{
    const int b = blockIdx.x;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

template <typename TIn>
__device__ __forceinline__ void stage_site(const TIn *__restrict__ S, int64_t slot, double2 *sS)
{
    const TIn *p = S + slot * 144;
    for (int e = threadIdx.x; e < 144; e += kPtThreads) sS[e] = make_double2((double)p[e].x, (double)p[e].y);
}

// Levels 1..M of the minors of rows R[0..M) of the staged 12x12 matrix, in
// ping-pong LDS buffers of binom(12, M) entries; returns the buffer holding
// level M (entry = colex rank of the column subset).
template <int M>
__device__ const double2 *levels(const PtSubset *__restrict__ T, const double2 *sS, const int8_t *R, double2 *buf0,
                                 double2 *buf1)
{
    if (threadIdx.x == 0) buf0[0] = make_double2(1.0, 0.0);
    __syncthreads();
    double2 *prev = buf0, *cur = buf1;
#pragma unroll
    for (int k = 1; k <= M; ++k) {
        const double2 *srow = sS + 12 * R[k - 1];
        const PtSubset *lev = T + level_off(k);
        for (int r = threadIdx.x; r < binom12c(k); r += kPtThreads) {
            const PtSubset e = lev[r];
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int j = 0; j < k; ++j) {
                const double2 t = cmul(srow[(e.elems >> (4 * j)) & 15], prev[e.sub[j]]);
                if ((k - 1 + j) & 1) { s.x -= t.x; s.y -= t.y; }
                else { s.x += t.x; s.y += t.y; }
            }
            cur[r] = s;
        }
        __syncthreads();
        double2 *t = prev;
        prev = cur;
        cur = t;
    }
    return prev;
}

// One minor of the last level N: the column subset of colex rank `rank`,
// expanded along row `row` over the level N-1 minors in Lp.
template <int N>
__device__ __forceinline__ double2 last_minor(const PtSubset *__restrict__ T, const double2 *srow, const double2 *Lp,
                                              int rank)
{
    if (N == 0) return make_double2(1.0, 0.0);
    const PtSubset e = T[level_off(N) + rank];
    double2 s = make_double2(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double2 t = cmul(srow[(e.elems >> (4 * j)) & 15], Lp[e.sub[j]]);
        if ((N - 1 + j) & 1) { s.x -= t.x; s.y -= t.y; }
        else { s.x += t.x; s.y += t.y; }
    }
    return s;
}

// Whether row set r shares its first N-1 rows with row set r-1 (rows sorted
// lexicographically, so such row sets are adjacent): then the levels below N
// are the same and are kept.
template <int N>
__device__ __forceinline__ bool same_prefix(const int8_t *rows, int r, int r0)
{
    if (r == r0) return false;
    bool same = true;
#pragma unroll
    for (int q = 0; q + 1 < N; ++q) same = same && rows[8 * r + q] == rows[8 * (r - 1) + q];
    return same;
}

template <typename TIn, int ND>
__global__ __launch_bounds__(kPtThreads) void pt_minors_kernel(const TIn *__restrict__ Sd, PtArgs a)
{
    constexpr int LB = binom12c(ND > 0 ? ND - 1 : 0);
    __shared__ double2 sS[144];
    __shared__ double2 buf[2][LB];
    const int total = a.n_slots * a.n_dchunks;
    const int id = xcd_id(gridDim.x);
    if (id >= total) return;
    const int slot = id / a.n_dchunks, chunk = id % a.n_dchunks;
    stage_site(Sd, a.slot0 + slot, sS);
    __syncthreads();
    const int r0 = chunk * kPtRowsPerWG, r1 = min(a.n_rows_d, r0 + kPtRowsPerWG);
    const double2 *Lp = buf[0];
    for (int r = r0; r < r1; ++r) {
        const int8_t *R = a.rows_d + 8 * r;
        if (!same_prefix<ND>(a.rows_d, r, r0)) Lp = levels<(ND > 0 ? ND - 1 : 0)>(a.sub, sS, R, buf[0], buf[1]);
        const double2 *srow = sS + 12 * (ND > 0 ? R[ND - 1] : 0);
        double2 *out = a.dd + ((int64_t)slot * a.n_rows_d + r) * a.n_cd;
        for (int c = threadIdx.x; c < a.n_cd; c += kPtThreads) out[c] = last_minor<ND>(a.sub, srow, Lp, a.d_cols[c]);
        __syncthreads();  // Lp is read until here; the next row set may rebuild it
    }
}

// The double sum over (sink group g, source group h) is regrouped by the
// source d column set c: for a sink u row set U,
//   A_U[c] = sum over source groups h with D'_h = c of W'_h det_u[U; U'_h]
// (source groups are sorted by c, so each c owns a contiguous range), and
// every sink group g of U adds W_g sum_c A_U[c] det_d[D_g; c]. The u
// determinants of U are formed for the source u column sets only (compact
// index), from level N-1 kept across row sets with equal leading rows.
// Thread t owns the d columns c = t + 256 i (i < CS): it builds their A_U[c],
// then reads the d determinants of each sink group at its own columns
// (contiguous across the wave).
template <typename TIn, int NU, int CS>
__global__ __launch_bounds__(kPtThreads) void pt_pairs_kernel(const TIn *__restrict__ Su, PtArgs a)
{
    constexpr int LB = binom12c(NU > 0 ? NU - 1 : 0);
    __shared__ double2 sS[144];
    __shared__ double2 buf[2][LB];
    __shared__ double2 red[kPtThreads / 64];
    extern __shared__ double2 du[];  // [n_cu] u determinants of the current row set
    const int total = a.n_slots * a.n_uchunks;
    const int id = xcd_id(gridDim.x);
    if (id >= total) return;
    const int slot = id / a.n_uchunks, chunk = id % a.n_uchunks;
    stage_site(Su, a.slot0 + slot, sS);
    int hb[CS], he[CS];  // source-group range of each owned column (empty past n_cd)
#pragma unroll
    for (int i = 0; i < CS; ++i) {
        const int c = threadIdx.x + kPtThreads * i;
        hb[i] = c < a.n_cd ? a.cd_beg[c] : 0;
        he[i] = c < a.n_cd ? a.cd_beg[c + 1] : 0;
    }
    __syncthreads();
    double2 tot = make_double2(0.0, 0.0);
    const int r0 = chunk * kPtRowsPerWG, r1 = min(a.n_rows_u, r0 + kPtRowsPerWG);
    const double2 *ddslot = a.dd + (int64_t)slot * a.n_rows_d * a.n_cd;
    const double2 *Lp = buf[0];
    for (int r = r0; r < r1; ++r) {
        const int8_t *R = a.rows_u + 8 * r;
        if (!same_prefix<NU>(a.rows_u, r, r0)) Lp = levels<(NU > 0 ? NU - 1 : 0)>(a.sub, sS, R, buf[0], buf[1]);
        const double2 *srow = sS + 12 * (NU > 0 ? R[NU - 1] : 0);
        for (int c = threadIdx.x; c < a.n_cu; c += kPtThreads) du[c] = last_minor<NU>(a.sub, srow, Lp, a.u_cols[c]);
        __syncthreads();
        double2 av[CS];
#pragma unroll
        for (int i = 0; i < CS; ++i) {
            double2 acc = make_double2(0.0, 0.0);
            for (int h = hb[i]; h < he[i]; ++h) {
                const double2 t = cmul(a.h_w[h], du[a.h_ru[h]]);
                acc.x += t.x;
                acc.y += t.y;
            }
            av[i] = acc;
        }
        for (int g = a.u_beg[r]; g < a.u_beg[r + 1]; ++g) {
            const double2 *drow = ddslot + (int64_t)a.g_d[g] * a.n_cd;
            double2 s = make_double2(0.0, 0.0);
#pragma unroll
            for (int i = 0; i < CS; ++i) {
                const int c = threadIdx.x + kPtThreads * i;
                if (c < a.n_cd) {
                    const double2 d = drow[c];
                    s.x += av[i].x * d.x - av[i].y * d.y;
                    s.y += av[i].x * d.y + av[i].y * d.x;
                }
            }
            const double2 t = cmul(a.g_w[g], s);
            tot.x += t.x;
            tot.y += t.y;
        }
        __syncthreads();
    }
    // workgroup sum: wave shuffle tree, then the waves in order
    for (int o = 32; o > 0; o >>= 1) {
        tot.x += __shfl_down(tot.x, o, 64);
        tot.y += __shfl_down(tot.y, o, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = tot;
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 s = red[0];
        for (int w = 1; w < kPtThreads / 64; ++w) { s.x += red[w].x; s.y += red[w].y; }
        a.partial[(a.slot0 + slot) * a.n_uchunks + chunk] = s;
    }
}

__global__ __launch_bounds__(kPtThreads) void pt_reduce_kernel(const double2 *__restrict__ partial, int64_t per_ct,
                                                              double scale, double2 *__restrict__ C)
{
    __shared__ double2 red[kPtThreads];
    const int64_t ct = blockIdx.x;
    const double2 *p = partial + ct * per_ct;
    double2 s = make_double2(0.0, 0.0);
    for (int64_t i = threadIdx.x; i < per_ct; i += kPtThreads) { s.x += p[i].x; s.y += p[i].y; }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = kPtThreads / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) { red[threadIdx.x].x += red[threadIdx.x + o].x; red[threadIdx.x].y += red[threadIdx.x + o].y; }
        __syncthreads();
    }
    if (threadIdx.x == 0) C[ct] = make_double2(scale * red[0].x, scale * red[0].y);
}

// ---------------------------------------------- point sinks from site blocks
// The point-sink correlator in the block form (Eq. 3.1): at every site the
// blocks of that site alone, contracted with the plan's signed term table,
// summed over sites. pt_site_blocks_kernel writes the compact blocks of every
// kind for a chunk of site-slices (one workgroup per site-slice: the
// antisymmetrised sum over the kind's weights); the term sum over each
// site-slice is then the plane-wave term-sum kernel with site-slices in place
// of time slices, and pt_reduce_kernel sums the sites of each (configuration, t).
constexpr int kPbThreads = 256;

struct PbKind {
    int32_t f, g, n_w, off;  // slot flavors (f, g, f), weights [off, off + n_w)
};

template <typename TIn>
__global__ __launch_bounds__(kPbThreads) void pt_site_blocks_kernel(const TIn *__restrict__ Su,
                                                                   const TIn *__restrict__ Sd, const PbKind *kinds,
                                                                   const double2 *__restrict__ ww,
                                                                   const int8_t *__restrict__ wj, int K, int64_t slot0,
                                                                   double2 *__restrict__ Bout)
{
    __shared__ double2 sS[288];
    const int64_t slot = slot0 + blockIdx.x;
    for (int e = threadIdx.x; e < 288; e += kPbThreads) {
        const TIn *src = (e < 144 ? Su : Sd) + slot * 144 + e % 144;
        sS[e] = make_double2((double)src->x, (double)src->y);
    }
    __syncthreads();
    double2 *out = Bout + (int64_t)blockIdx.x * K * 792;
    for (int e = threadIdx.x; e < K * 792; e += kPbThreads) {
        const int k = e / 792, c = e % 792;
        const int pair = c / 12, i2 = c % 12;
        int i3 = 1;
        while ((i3 + 1) * i3 / 2 <= pair) ++i3;
        const int i1 = pair - i3 * (i3 - 1) / 2;
        const PbKind kd = kinds[k];
        const double2 *F = sS + kd.f * 144, *G = sS + kd.g * 144;
        double2 acc = make_double2(0.0, 0.0);
        for (int w = kd.off; w < kd.off + kd.n_w; ++w) {
            const int j1 = wj[3 * w], j2 = wj[3 * w + 1], j3 = wj[3 * w + 2];
            const double2 x = cmul(F[j1 * 12 + i1], F[j3 * 12 + i3]);
            const double2 y = cmul(F[j1 * 12 + i3], F[j3 * 12 + i1]);
            const double2 t = cmul(ww[w], cmul(G[j2 * 12 + i2], make_double2(x.x - y.x, x.y - y.y)));
            acc.x += t.x;
            acc.y += t.y;
        }
        out[e] = acc;
    }
}

// ------------------------------------------------------------ host side
wick_status pt_hip_fail(hipError_t e, const char *what)
{
    return fail(WICK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void build_subsets(std::vector<PtSubset> &T)
{
    T.assign(kPtSubsets, PtSubset{0, {0, 0, 0, 0, 0, 0}});
    for (int k = 1; k <= 6; ++k) {
        // colex order of k-subsets = increasing bitmask
        std::vector<int> rank_of(4096, -1), rank_prev(4096, -1);
        int r = 0, q = 0;
        for (int m = 0; m < 4096; ++m) {
            if (__builtin_popcount(m) == k) rank_of[m] = r++;
            if (__builtin_popcount(m) == k - 1) rank_prev[m] = q++;
        }
        for (int m = 0; m < 4096; ++m) {
            if (__builtin_popcount(m) != k) continue;
            PtSubset &e = T[level_off(k) + rank_of[m]];
            int j = 0;
            for (int c = 0; c < 12; ++c)
                if (m >> c & 1) {
                    e.elems |= (uint32_t)c << (4 * j);
                    e.sub[j] = (uint16_t)rank_prev[m & ~(1 << c)];
                    ++j;
                }
        }
    }
}

template <class T>
wick_status upload(const std::vector<T> &v, T **out)
{
    const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
    hipError_t e = hipMalloc((void **)out, bytes);
    if (e != hipSuccess) return fail(WICK_ENOMEM, std::string("wick_point: hipMalloc: ") + hipGetErrorString(e));
    if (!v.empty()) {
        e = hipMemcpy(*out, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return pt_hip_fail(e, "wick_point: hipMemcpy");
    }
    return WICK_OK;
}

void free_dev(PtDev *d)
{
    (void)hipFree(d->sub);
    (void)hipFree(d->rows_u);
    (void)hipFree(d->rows_d);
    (void)hipFree(d->u_beg);
    (void)hipFree(d->g_d);
    (void)hipFree(d->g_w);
    (void)hipFree(d->h_ru);
    (void)hipFree(d->cd_beg);
    (void)hipFree(d->h_w);
    (void)hipFree(d->d_cols);
    (void)hipFree(d->u_cols);
    delete d;
}

wick_status device_tables(wick_point_s *p, PtDev **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pt_hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(p->dev_mu);
    for (void *v : p->dev)
        if (((PtDev *)v)->device == dev) { *out = (PtDev *)v; return WICK_OK; }
    auto d = new PtDev();
    d->device = dev;
    std::vector<PtSubset> tv;
    build_subsets(tv);
    std::vector<int8_t> ru, rd;
    for (auto &r : p->rows_u) ru.insert(ru.end(), r.begin(), r.end());
    for (auto &r : p->rows_d) rd.insert(rd.end(), r.begin(), r.end());
    std::vector<double2> gw(p->g_u.size());
    for (size_t i = 0; i < gw.size(); ++i) gw[i] = make_double2(p->g_w[2 * i], p->g_w[2 * i + 1]);
    // compact d columns: the source column sets that occur, in rank order
    std::map<int, int> cols;
    for (uint16_t r : p->h_rd) cols.emplace(r, 0);
    std::vector<uint16_t> dcols;
    for (auto &c : cols) { c.second = (int)dcols.size(); dcols.push_back((uint16_t)c.first); }
    d->n_cd = (int)dcols.size();
    std::map<int, int> ucols;
    for (uint16_t r : p->h_ru) ucols.emplace(r, 0);
    std::vector<uint16_t> ucl;
    for (auto &c : ucols) { c.second = (int)ucl.size(); ucl.push_back((uint16_t)c.first); }
    d->n_cu = (int)ucl.size();
    // source groups ordered by (d column, u column), with the range of each d column
    const size_t H = p->h_ru.size();
    std::vector<size_t> ord(H);
    for (size_t i = 0; i < H; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](size_t x, size_t y) {
        return p->h_rd[x] != p->h_rd[y] ? p->h_rd[x] < p->h_rd[y] : p->h_ru[x] < p->h_ru[y];
    });
    std::vector<uint16_t> hru(H);
    std::vector<double2> hw(H);
    std::vector<int32_t> cdb(d->n_cd + 1, 0);
    for (size_t i = 0; i < H; ++i) {
        const size_t h = ord[i];
        hru[i] = (uint16_t)ucols[p->h_ru[h]];
        hw[i] = make_double2(p->h_w[2 * h], p->h_w[2 * h + 1]);
        cdb[cols[p->h_rd[h]] + 1]++;
    }
    for (int c = 0; c < d->n_cd; ++c) cdb[c + 1] += cdb[c];
    wick_status st;
    if ((st = upload(tv, &d->sub)) != WICK_OK || (st = upload(ru, &d->rows_u)) != WICK_OK ||
        (st = upload(rd, &d->rows_d)) != WICK_OK || (st = upload(p->u_beg, &d->u_beg)) != WICK_OK ||
        (st = upload(p->g_d, &d->g_d)) != WICK_OK || (st = upload(gw, &d->g_w)) != WICK_OK ||
        (st = upload(hru, &d->h_ru)) != WICK_OK || (st = upload(cdb, &d->cd_beg)) != WICK_OK ||
        (st = upload(hw, &d->h_w)) != WICK_OK || (st = upload(dcols, &d->d_cols)) != WICK_OK ||
        (st = upload(ucl, &d->u_cols)) != WICK_OK) {
        free_dev(d);
        return st;
    }
    p->dev.push_back(d);
    *out = d;
    return WICK_OK;
}

int64_t check_point_dims(const int32_t dims[4], int32_t n_cfg)
{
    if (!dims || n_cfg < 1) return -1;
    for (int i = 0; i < 4; ++i)
        if (dims[i] < 1) return -1;
    const int64_t V = (int64_t)dims[0] * dims[1] * dims[2];
    if (V > (1LL << 30) || (int64_t)n_cfg * dims[3] > (1LL << 24)) return -2;
    return V;
}

template <typename TIn>
wick_status launch_point(wick_point_s *p, PtDev *d, const TIn *Su, const TIn *Sd, int64_t V, int64_t n_ct,
                         hipStream_t s, double2 *C)
{
    const int64_t slots = V * n_ct;
    if (p->g_u.empty() || p->h_ru.empty()) {
        // no sink or no source groups: C is zero (a fill kernel, also inside graph capture)
        hipError_t e = launch_zero((double *)C, 2 * n_ct, s);
        return e == hipSuccess ? WICK_OK : pt_hip_fail(e, "zero_kernel");
    }
    PtArgs a{};
    a.sub = d->sub;
    a.rows_u = d->rows_u;
    a.rows_d = d->rows_d;
    a.u_beg = d->u_beg;
    a.g_d = d->g_d;
    a.g_w = d->g_w;
    a.h_ru = d->h_ru;
    a.cd_beg = d->cd_beg;
    a.d_cols = d->d_cols;
    a.u_cols = d->u_cols;
    a.h_w = d->h_w;
    a.n_u = p->n_u;
    a.n_d = p->n_d;
    a.n_rows_u = (int)p->rows_u.size();
    a.n_rows_d = (int)p->rows_d.size();
    a.n_h = (int)p->h_ru.size();
    a.n_cd = d->n_cd;
    a.n_cu = d->n_cu;
    a.n_uchunks = (a.n_rows_u + kPtRowsPerWG - 1) / kPtRowsPerWG;
    a.n_dchunks = (a.n_rows_d + kPtRowsPerWG - 1) / kPtRowsPerWG;
    const size_t per_slot_dd = (size_t)a.n_rows_d * a.n_cd * sizeof(double2);
    const size_t partial_bytes = (size_t)slots * a.n_uchunks * sizeof(double2);
    int64_t chunk = std::max<int64_t>(8, (int64_t)((512ull << 20) / std::max<size_t>(per_slot_dd, 1)) / 8 * 8);
    chunk = std::min<int64_t>(chunk, slots);
    const int64_t max_wg = (1LL << 31) - 64;
    chunk = std::min<int64_t>(chunk, max_wg / std::max(a.n_uchunks, a.n_dchunks));
    void *ws = nullptr;
    const size_t part_off = ((size_t)chunk * per_slot_dd + 255) / 256 * 256;
    wick_status st = workspace(s, part_off + partial_bytes, &ws);
    if (st != WICK_OK) return st;
    a.dd = (double2 *)ws;
    a.partial = (double2 *)((char *)ws + part_off);
    for (int64_t s0 = 0; s0 < slots; s0 += chunk) {
        a.slot0 = s0;
        a.n_slots = (int)std::min<int64_t>(chunk, slots - s0);
        const int64_t nd = (int64_t)a.n_slots * a.n_dchunks, nu = (int64_t)a.n_slots * a.n_uchunks;
        const dim3 gd((unsigned)((nd + 7) / 8 * 8)), gu((unsigned)((nu + 7) / 8 * 8)), blk(kPtThreads);
        Probe pa("point_minors", s);
        switch (a.n_d) {
#define PT_MINORS(n) case n: pt_minors_kernel<TIn, n><<<gd, blk, 0, s>>>(Sd, a); break;
            PT_MINORS(0) PT_MINORS(1) PT_MINORS(2) PT_MINORS(3) PT_MINORS(4) PT_MINORS(5) PT_MINORS(6)
#undef PT_MINORS
        }
        pa.stop();
        Probe pb("point_pairs", s);
        const int cs = (a.n_cd + kPtThreads - 1) / kPtThreads;  // 1..4 (n_cd <= 924)
        const size_t shu = (size_t)std::max(1, a.n_cu) * sizeof(double2);  // <= 924 entries: 14.8 KB
        switch (a.n_u * 4 + cs - 1) {
#define PT_PAIRS(n)                                                                \
    case 4 * n + 0: pt_pairs_kernel<TIn, n, 1><<<gu, blk, shu, s>>>(Su, a); break;  \
    case 4 * n + 1: pt_pairs_kernel<TIn, n, 2><<<gu, blk, shu, s>>>(Su, a); break;  \
    case 4 * n + 2: pt_pairs_kernel<TIn, n, 3><<<gu, blk, shu, s>>>(Su, a); break;  \
    case 4 * n + 3: pt_pairs_kernel<TIn, n, 4><<<gu, blk, shu, s>>>(Su, a); break;
            PT_PAIRS(0) PT_PAIRS(1) PT_PAIRS(2) PT_PAIRS(3) PT_PAIRS(4) PT_PAIRS(5) PT_PAIRS(6)
#undef PT_PAIRS
        }
        pb.stop();
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return pt_hip_fail(e, "point kernels");
    }
    Probe pc("point_reduce", s);
    pt_reduce_kernel<<<dim3((unsigned)n_ct), dim3(kPtThreads), 0, s>>>(a.partial, V * a.n_uchunks, p->scale, C);
    pc.stop();
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? WICK_OK : pt_hip_fail(e, "pt_reduce_kernel");
}

// The plan's kind weights on the current device (cached in the plan, released
// with it): the kinds, then the weights (16-byte aligned), then their indices.
wick_status kind_tables(wick_plan_s *p, DeviceTable *out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pt_hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(p->dev_mu);
    for (auto &d : p->dev)
        if (d.device == dev) { *out = d; return WICK_OK; }
    DeviceTable d;
    d.device = dev;
    const int K = (int)p->kinds.size();
    std::vector<PbKind> kinds(K);
    std::vector<int8_t> wj;
    std::vector<double2> ww;
    for (int k = 0; k < K; ++k) {
        const KindDef &kd = p->kinds[k];
        kinds[k] = PbKind{kd.flav[0], kd.flav[1], (int32_t)kd.w.size(), (int32_t)ww.size()};
        for (size_t n = 0; n < kd.w.size(); ++n) {
            for (int q = 0; q < 3; ++q) wj.push_back(kd.j[n][q]);
            ww.push_back(make_double2((double)kd.w[n].re, (double)kd.w[n].im));
        }
    }
    const size_t kb = ((K * sizeof(PbKind)) + 15) / 16 * 16, wb = ww.size() * sizeof(double2);
    std::vector<char> blob(kb + wb + wj.size() + 16, 0);
    std::memcpy(blob.data(), kinds.data(), K * sizeof(PbKind));
    std::memcpy(blob.data() + kb, ww.data(), wb);
    std::memcpy(blob.data() + kb + wb, wj.data(), wj.size());
    if ((e = hipMalloc(&d.kinds, blob.size())) != hipSuccess)
        return fail(WICK_ENOMEM, std::string("wick_point_blocks_correlator: hipMalloc: ") + hipGetErrorString(e));
    if ((e = hipMemcpy(d.kinds, blob.data(), blob.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(d.kinds);
        return pt_hip_fail(e, "wick_point_blocks_correlator: hipMemcpy");
    }
    p->dev.push_back(d);
    *out = d;
    return WICK_OK;
}

template <typename TIn>
wick_status launch_point_blocks(wick_plan_s *p, const DeviceTable *d, const TIn *Su, const TIn *Sd, int64_t V,
                                int64_t n_ct, hipStream_t s, double2 *C)
{
    const int64_t slots = V * n_ct;
    if (p->n_terms == 0) {
        hipError_t e = launch_zero((double *)C, 2 * n_ct, s);
        return e == hipSuccess ? WICK_OK : pt_hip_fail(e, "zero_kernel");
    }
    const int K = (int)p->kinds.size();
    const size_t per_slot = (size_t)K * 792 * sizeof(double2);
    // site-slices per chunk: at most 512 MB of blocks and at most 2^20 sets per term-sum call
    const int64_t chunk = std::max<int64_t>(1, std::min<int64_t>({slots, (int64_t)((512ull << 20) / per_slot), 1 << 20}));
    void *ws = nullptr;
    const size_t c_off = ((size_t)chunk * per_slot + 255) / 256 * 256;
    wick_status st = workspace(s, c_off + (size_t)slots * sizeof(double2), &ws, 1);
    if (st != WICK_OK) return st;
    double2 *Bw = (double2 *)ws, *Cs = (double2 *)((char *)ws + c_off);
    size_t nw = 0;
    for (auto &kd : p->kinds) nw += kd.w.size();
    const size_t kb = ((K * sizeof(PbKind)) + 15) / 16 * 16;
    const PbKind *kinds = (const PbKind *)d->kinds;
    const double2 *ww = (const double2 *)((const char *)d->kinds + kb);
    const int8_t *wj = (const int8_t *)((const char *)d->kinds + kb + nw * sizeof(double2));
    for (int64_t s0 = 0; s0 < slots; s0 += chunk) {
        const int64_t n = std::min<int64_t>(chunk, slots - s0);
        Probe pb("point_site_blocks", s);
        pt_site_blocks_kernel<TIn><<<dim3((unsigned)n), dim3(kPbThreads), 0, s>>>(Su, Sd, kinds, ww, wj, K, s0, Bw);
        pb.stop();
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return pt_hip_fail(e, "pt_site_blocks_kernel");
        // the plane-wave term sum, one set per site-slice
        if ((st = wick_contract(p, (const double *)Bw, 1, (int32_t)n, (wick_stream_t)s, (double *)(Cs + s0))) != WICK_OK)
            return st;
    }
    Probe pc("point_reduce", s);
    pt_reduce_kernel<<<dim3((unsigned)n_ct), dim3(kPtThreads), 0, s>>>(Cs, V, 1.0, C);
    pc.stop();
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? WICK_OK : pt_hip_fail(e, "pt_reduce_kernel");
}

}  // namespace

void release_point_tables(wick_point_s *p)
{
    std::lock_guard<std::mutex> lk(p->dev_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (void *v : p->dev) {
        PtDev *d = (PtDev *)v;
        (void)hipSetDevice(d->device);
        free_dev(d);
    }
    p->dev.clear();
    (void)hipSetDevice(cur);
}

void release_plain_tables(wick_plan_s *p)
{
    std::lock_guard<std::mutex> lk(p->dev_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &d : p->dev) {
        (void)hipSetDevice(d.device);
        (void)hipDeviceSynchronize();
        (void)hipFree(d.kinds);
    }
    p->dev.clear();
    (void)hipSetDevice(cur);
}

}  // namespace wick

using namespace wick;

extern "C" wick_status wick_point_blocks_correlator(wick_plan_t p, const void *S_u, const void *S_d, wick_dtype dtype,
                                                    const int32_t dims[4], int32_t n_cfg, wick_stream_t stream,
                                                    double *C)
{
    try {
        if (!p || !S_u || !S_d || !C) return fail(WICK_EINVAL, "wick_point_blocks_correlator: null pointer");
        if (((uintptr_t)S_u | (uintptr_t)S_d | (uintptr_t)C) & 15)
            return fail(WICK_EINVAL, "wick_point_blocks_correlator: propagators and C must be 16-byte aligned");
        if (dtype != WICK_C128 && dtype != WICK_C64) return fail(WICK_EINVAL, "wick_point_blocks_correlator: bad dtype");
        const int64_t V = check_point_dims(dims, n_cfg);
        if (V == -1) return fail(WICK_EINVAL, "wick_point_blocks_correlator: bad dims or n_cfg");
        if (V < 0) return fail(WICK_ETOOBIG, "wick_point_blocks_correlator: lattice too large");
        const int64_t n_ct = (int64_t)n_cfg * dims[3];
        DeviceTable d;
        wick_status st = kind_tables(p, &d);
        if (st != WICK_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        if (dtype == WICK_C128)
            return launch_point_blocks(p, &d, (const double2 *)S_u, (const double2 *)S_d, V, n_ct, s, (double2 *)C);
        return launch_point_blocks(p, &d, (const float2 *)S_u, (const float2 *)S_d, V, n_ct, s, (double2 *)C);
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_point_blocks_correlator: out of host memory");
    } catch (...) {
        return fail(WICK_EINVAL, "wick_point_blocks_correlator: internal error");
    }
}

extern "C" wick_status wick_point_correlator(wick_point_t p, const void *S_u, const void *S_d, wick_dtype dtype,
                                             const int32_t dims[4], int32_t n_cfg, wick_stream_t stream, double *C)
{
    try {
        if (!p || !S_u || !S_d || !C) return fail(WICK_EINVAL, "wick_point_correlator: null pointer");
        if (((uintptr_t)S_u | (uintptr_t)S_d | (uintptr_t)C) & 15)
            return fail(WICK_EINVAL, "wick_point_correlator: propagators and C must be 16-byte aligned");
        if (dtype != WICK_C128 && dtype != WICK_C64) return fail(WICK_EINVAL, "wick_point_correlator: bad dtype");
        const int64_t V = check_point_dims(dims, n_cfg);
        if (V == -1) return fail(WICK_EINVAL, "wick_point_correlator: bad dims or n_cfg");
        if (V < 0) return fail(WICK_ETOOBIG, "wick_point_correlator: lattice too large");
        const int64_t n_ct = (int64_t)n_cfg * dims[3];
        if ((int64_t)(p->rows_u.size() + kPtRowsPerWG) / kPtRowsPerWG * V * n_ct > (1LL << 40))
            return fail(WICK_ETOOBIG, "wick_point_correlator: too many partial sums");
        PtDev *d = nullptr;
        wick_status st = device_tables(p, &d);
        if (st != WICK_OK) return st;
        hipStream_t s = (hipStream_t)stream;
        if (dtype == WICK_C128)
            return launch_point(p, d, (const double2 *)S_u, (const double2 *)S_d, V, n_ct, s, (double2 *)C);
        return launch_point(p, d, (const float2 *)S_u, (const float2 *)S_d, V, n_ct, s, (double2 *)C);
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_point_correlator: out of host memory");
    } catch (...) {
        return fail(WICK_EINVAL, "wick_point_correlator: internal error");
    }
}
