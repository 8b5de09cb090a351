// HIP kernels for gfx950 (MI355X): baryon blocks on MFMA and the FP64 Wick-term sum.
//
// Block build (Eq. 2.4, App. D). For a group of kinds sharing their diquark
// rows (same flavors (f, g, f) and the same eps * (C g5 P) structure),
//   Braw_k[i1, (i2,i3)] = sum_x sum_r Aop_k(x, r)[i1] * E_r(x)[(i2,i3)],
//   E_r(x)[i2,i3]      = sum_t w_t S_g(x)[j2_t, i2] S_f(x)[j3_t, i3]   (VALU),
//   Aop_k(x, r)[i1]    = sum_e a_e S_f(x)[j1_e, i1]                     (a row of S_f),
// i.e. a complex GEMM with M = 144 (i2, i3), N = 12 per kind (i1), and
// K = R per site summed over all sites. It runs on v_mfma_f64_16x16x4f64:
// the A operand is E (lane l: column n = 16*tile + l%16, site l/16), the B
// operand is Aop (lane l: site l/16, row m = 16*mtile + l%16 -> (kind, i1)),
// so each MFMA contracts four sites at once. In this generic kernel a
// complex product takes four real MFMAs (re*re - im*im, re*im + im*re); the
// nucleon-form kernel below takes three in FP64 (Gauss's form).
//
// Sites are split into chunks (split-K); each wave writes its chunk's partial
// block and a second kernel sums the chunks in a fixed order and
// antisymmetrises the two same-flavor slots (Eq. 2.4), so results are
// bitwise repeatable.
//
// Term sum (Eq. 2.6, App. D): one workgroup per (configuration, time slice,
// slice of the term table); the blocks of its (cfg, t) sit in LDS, each lane
// gathers A entries per term, multiplies in FP64 and accumulates; a fixed
// shuffle/LDS tree reduces the workgroup and a second kernel sums the slices
// in order.
#include <hip/hip_runtime.h>
#include <type_traits>

#include "kernels.hpp"

namespace wick {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct cplx {
    double x, y;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

template <typename TIn>
__device__ __forceinline__ cplx ld(const TIn *p)
{
    return {(double)p->x, (double)p->y};
}

// Block id remapped so that consecutive logical ids run on one XCD
// (hardware places block b on XCD b % 8). Requires gridDim.x % 8 == 0.
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, b = blockIdx.x;
    return (b & 7) * (nb >> 3) + (b >> 3);
}

constexpr int kMT = 4;  // maximum MFMA m-tiles per group (5 kinds x 12 rows <= 64)

template <typename TIn>
__global__ __launch_bounds__(256) void blocks_f64_kernel(
    const TIn *__restrict__ Su, const TIn *__restrict__ Sd, const EGroupDev *__restrict__ groups,
    int n_units, int64_t V, int chunk_sites, int n_chunks, int K, int64_t n_waves_total,
    double2 *__restrict__ partial)
{
    const int64_t wave =
        __builtin_amdgcn_readfirstlane((int64_t)xcd_block() * (blockDim.x >> 6) + (threadIdx.x >> 6));
    if (wave >= n_waves_total) return;
    const int unit = (int)(wave % n_units);
    const int64_t rest = wave / n_units;
    const int chunk = (int)(rest % n_chunks);
    const int64_t ct = rest / n_chunks;
    const int gi = unit / kNTiles, nt = unit % kNTiles;
    const EGroupDev &G = groups[gi];
    const int R = G.R, nk = G.nk, MT = G.mt;

    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int n = nt * 16 + c, i2 = n / 12, i3 = n % 12;
    const TIn *Sf = (G.f == 0 ? Su : Sd) + ct * V * 144;
    const TIn *Sg = (G.g == 0 ? Su : Sd) + ct * V * 144;

    int kk_m[kMT], i1_m[kMT];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) {
        const int m = mt * 16 + c;
        kk_m[mt] = m / 12;
        i1_m[mt] = m % 12;
    }

    d4 acc[kMT][2];
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) acc[mt][0] = acc[mt][1] = d4{0, 0, 0, 0};

    const int64_t x0 = (int64_t)chunk * chunk_sites;
    const int64_t x1 = x0 + chunk_sites < V ? x0 + chunk_sites : V;
    for (int64_t xs = x0; xs < x1; xs += 4) {
        const int64_t x = xs + q;
        const bool ok = x < x1;
        const TIn *sf = Sf + (ok ? x : x0) * 144;
        const TIn *sg = Sg + (ok ? x : x0) * 144;
        for (int r = 0; r < R; ++r) {
            cplx E = {0.0, 0.0};
            const int nterm = G.nterm[r];
            for (int t = 0; t < nterm; ++t) {
                const cplx a = ld(sg + G.j2[r][t] * 12 + i2);
                const cplx b = ld(sf + G.j3[r][t] * 12 + i3);
                const cplx p = cmul(a, b);
                const double w = (double)G.w[r][t];
                E.x += w * p.x;
                E.y += w * p.y;
            }
            if (!ok) E = {0.0, 0.0};
#pragma unroll
            for (int mt = 0; mt < kMT; ++mt) {
                if (mt >= MT) break;
                cplx Ao = {0.0, 0.0};
                const int kk = kk_m[mt];
                if (kk < nk) {
#pragma unroll
                    for (int e = 0; e < kMaxAop; ++e) {
                        const int a = G.aa[kk][r][e];
                        if (a) {
                            const cplx s = ld(sf + G.aj1[kk][r][e] * 12 + i1_m[mt]);
                            Ao.x += a * s.x;
                            Ao.y += a * s.y;
                        }
                    }
                }
                acc[mt][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(E.x, Ao.x, acc[mt][0], 0, 0, 0);
                acc[mt][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(E.y, -Ao.y, acc[mt][0], 0, 0, 0);
                acc[mt][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(E.x, Ao.y, acc[mt][1], 0, 0, 0);
                acc[mt][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(E.y, Ao.x, acc[mt][1], 0, 0, 0);
            }
        }
    }
    // D layout of the 16x16x4 f64 MFMA (measured on gfx950): lane l, item v ->
    // row 4*v + l/16, column l%16. (The f32 variant uses row 4*(l/16) + v.)
    double2 *P = partial + (ct * n_chunks + chunk) * (int64_t)K * 1728;
#pragma unroll
    for (int mt = 0; mt < kMT; ++mt) {
        if (mt >= MT) break;
        const int kk = kk_m[mt];
        if (kk >= nk) continue;
        const int kind = G.kind_out[kk];
        double2 *row = P + ((int64_t)kind * 12 + i1_m[mt]) * 144 + nt * 16 + q;
#pragma unroll
        for (int v = 0; v < 4; ++v) row[4 * v] = double2{acc[mt][0][v], acc[mt][1][v]};
    }
}

// Staged variant: one workgroup of 9 waves per (cfg*T + t, site chunk); wave
// w owns column tile w (16 of the 144 (i2, i3) columns) for every group, so
// all waves share the sites' propagators, which are brought from HBM once
// per workgroup with coalesced 16-byte loads into double-buffered LDS
// (kSB sites per buffer; the next batch is loaded while this one is used).
constexpr int kSB = 8;
constexpr int kStagedThreads = 64 * kNTiles;

template <typename TIn, int NT>
__global__ __launch_bounds__(kStagedThreads) void blocks_f64_staged_kernel(
    const TIn *__restrict__ Su, const TIn *__restrict__ Sd, const BlocksDesc *__restrict__ desc, int64_t V,
    int chunk_sites, int n_chunks, int K, int n_work, double2 *__restrict__ partial)
{
    __shared__ double2 sbuf[2][kSB][2][144];
    // E-row terms of the pass's groups: (j2*12) | (j3*12) << 8 | (w & 0xff) << 16
    __shared__ int32_t s_et[kPassTiles][kMaxRows][kMaxRowTerms];
    // per tile, row and column lane: two (offset j1*12 + i1, coefficient) entries of Aop
    __shared__ int2 s_ao[NT][kMaxRows][16];
    const int lb = xcd_block();
    if (lb >= n_work) return;
    const int pass = lb % desc->n_passes;
    const int chunk = (lb / desc->n_passes) % n_chunks;
    const int64_t ct = lb / desc->n_passes / n_chunks;
    const int nt = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int n = nt * 16 + c, i2 = n / 12, i3 = n % 12;
    const int npg = desc->pass_ngroups[pass];
    const int32_t *tgroup = desc->tile_group[pass];

    // descriptors -> LDS (once per workgroup)
    for (int e = threadIdx.x; e < kPassTiles * kMaxRows * kMaxRowTerms; e += kStagedThreads) {
        const int gl = e / (kMaxRows * kMaxRowTerms), r = (e / kMaxRowTerms) % kMaxRows, t = e % kMaxRowTerms;
        int32_t v = 0;
        if (gl < npg) {
            const EGroupDev &G = desc->groups[desc->pass_groups[pass][gl]];
            if (r < G.R && t < G.nterm[r])
                v = (G.j2[r][t] * 12) | ((G.j3[r][t] * 12) << 8) | (((int)G.w[r][t] & 0xff) << 16);
        }
        (&s_et[0][0][0])[e] = v;
    }
    for (int e = threadIdx.x; e < NT * kMaxRows * 16; e += kStagedThreads) {
        const int t = e / (kMaxRows * 16), r = (e / 16) % kMaxRows, cc = e % 16;
        int2 v = int2{0, 0};
        const int g = tgroup[t];
        if (g >= 0) {
            const EGroupDev &G = desc->groups[g];
            const int m = desc->tile_mt[pass][t] * 16 + cc, kk = m / 12, i1 = m % 12;
            if (kk < G.nk && r < G.R) {
                v.x = (G.aj1[kk][r][0] * 12 + i1) | ((int)G.aa[kk][r][0] << 16);
                v.y = (G.aj1[kk][r][1] * 12 + i1) | ((int)G.aa[kk][r][1] << 16);
            }
        }
        (&s_ao[0][0][0])[e] = v;
    }

    d4 acc[NT][2];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t][0] = acc[t][1] = d4{0, 0, 0, 0};

    const int64_t x0 = (int64_t)chunk * chunk_sites;
    const int64_t x1 = x0 + chunk_sites < V ? x0 + chunk_sites : V;
    const int nb = (int)((x1 - x0 + kSB - 1) / kSB);
    const TIn *base[2] = {Su + ct * V * 144, Sd + ct * V * 144};
    // each thread moves kPer of the kSB*2*144 entries of a batch
    constexpr int kPer = kSB * 2 * 144 / kStagedThreads;
    double2 stage[kPer];
    auto load = [&](int b) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) {
            const int e = threadIdx.x + u * kStagedThreads;     // [site][flavor][144]
            const int s = e / 288, fl = (e / 144) & 1, j = e % 144;
            const int64_t x = x0 + (int64_t)b * kSB + s;
            if (x < x1) {
                const TIn v = base[fl][x * 144 + j];
                stage[u] = double2{(double)v.x, (double)v.y};
            } else {
                stage[u] = double2{0.0, 0.0};
            }
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < kPer; ++u) (&sbuf[buf][0][0][0])[threadIdx.x + u * kStagedThreads] = stage[u];
    };
    load(0);
    store(0);
    __syncthreads();
    for (int b = 0; b < nb; ++b) {
        const int cur = b & 1;
        if (b + 1 < nb) load(b + 1);
        for (int st = 0; st < kSB / 4; ++st) {
            const int s = st * 4 + q;
            // sites past the end were stored as zeros: their E and Aop vanish
            for (int gl = 0; gl < npg; ++gl) {
                const int g = desc->pass_groups[pass][gl];
                const EGroupDev &G = desc->groups[g];
                const double2 *sf = sbuf[cur][s][G.f];
                const double2 *sg = sbuf[cur][s][G.g];
                const double2 *sgi = sg + i2, *sfi = sf + i3;
                for (int r = 0; r < G.R; ++r) {
                    double ex = 0.0, ey = 0.0;
                    const int nterm = G.nterm[r];
                    const int32_t *et = s_et[gl][r];
#pragma unroll 4
                    for (int t = 0; t < nterm; ++t) {
                        const int32_t pk = et[t];
                        const double2 a = sgi[pk & 0xff];
                        const double2 bb = sfi[(pk >> 8) & 0xff];
                        const double w = (double)(int8_t)(pk >> 16);
                        ex += w * (a.x * bb.x - a.y * bb.y);
                        ey += w * (a.x * bb.y + a.y * bb.x);
                    }
#pragma unroll
                    for (int t = 0; t < NT; ++t) {
                        if (tgroup[t] != g) continue;
                        const int2 ao = s_ao[t][r][c];
                        const double2 v0 = sf[ao.x & 0xffff], v1 = sf[ao.y & 0xffff];
                        const double a0 = (double)(ao.x >> 16), a1 = (double)(ao.y >> 16);
                        const double ax = a0 * v0.x + a1 * v1.x, ay = a0 * v0.y + a1 * v1.y;
                        acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ex, ax, acc[t][0], 0, 0, 0);
                        acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ex, ay, acc[t][1], 0, 0, 0);
                        acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(ey, -ay, acc[t][0], 0, 0, 0);
                        acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ey, ax, acc[t][1], 0, 0, 0);
                    }
                }
            }
        }
        if (b + 1 < nb) store(cur ^ 1);
        __syncthreads();
    }
    double2 *P = partial + (ct * n_chunks + chunk) * (int64_t)K * 1728;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (tgroup[t] < 0) continue;
        const EGroupDev &G = desc->groups[tgroup[t]];
        const int m = desc->tile_mt[pass][t] * 16 + c, kk = m / 12, i1 = m % 12;
        if (kk >= G.nk) continue;
        const int kind = G.kind_out[kk];
        double2 *row = P + ((int64_t)kind * 12 + i1) * 144 + nt * 16 + q;
#pragma unroll
        for (int v = 0; v < 4; ++v) row[4 * v] = double2{acc[t][0][v], acc[t][1][v]};
    }
}

// Nucleon-form kernel: the staged layout (9 waves, one column tile each,
// double-buffered LDS propagators in FP64) with the E rows computed in FP64
// as colour cross products per nonzero diquark-matrix entry (6 LDS loads for
// all three rows) and Aop read with a per-lane base offset fixed at kernel
// start. The GEMM runs, by MODE, on
//   P64: v_mfma_f64_16x16x4f64, three real MFMAs per complex product
//        (Gauss): with E = a + ib and Aop = c + id, K1 += (a + b) c,
//        K2 += a (d - c), K3 += b (c + d), then Re = K1 - K3, Im = K1 + K2,
//        formed once per workgroup after the site loop;
//   P32: v_mfma_f32_16x16x4f32, four real MFMAs per complex product with E
//        and Aop rounded to FP32 (complex64 entries are used as stored; the
//        three-product form measured no faster here and doubled the error);
//   PB3: v_mfma_f32_16x16x32_bf16, E and Aop split into two BF16 limbs
//        (hi + lo), the three products hi*hi + hi*lo + lo*hi packed along K:
//        one MFMA per real/imaginary output;
//   PB6: three limbs (hi + mid + lo) and the six products of limb order <= 2:
//        two MFMAs per output.
// In the split modes E is scaled by an exact power of two per wave and group
// (see the kernel) and Aop is not scaled; the MFMAs accumulate in FP32 over
// a few batches and are folded into FP64 accumulators with the exact inverse
// factor. Operand layout of the BF16 MFMA (measured): A[i][k] at lane
// i + 16*(k/8), element k%8; B[k][j] at lane j + 16*(k/8); D as for the f32
// 16x16x4 MFMA, row 4*(lane/16) + item, column lane%16. Lane group q
// (= k/8 for BF16, = k for the 16x16x4 MFMAs) is site q of the step.
typedef float f4 __attribute__((ext_vector_type(4)));
extern "C" __device__ int __ockl_wfred_max_i32(int);  // wave-wide maximum (device library)
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// One wave-wide 16-byte-per-lane load from global memory straight into LDS:
// lane i's 16 bytes land at lds_dst + 16 i (lds_dst wave-uniform). Written as
// inline assembly so that the compiler's wait-count insertion, which cannot
// tell the two staging buffers apart, does not make every LDS read of the
// batch in use wait for the loads of the next one; the kernel waits for them
// itself (vmcnt) before the barrier that publishes the buffer.
__device__ __forceinline__ void lds_dma16(const void *src, void *lds_dst)
{
    const uint32_t l = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) void *)lds_dst;
    // the LDS address goes in through the M0 constraint: the compiler writes
    // M0 itself and so keeps no value of its own there across this statement
    asm volatile("global_load_lds_dwordx4 %0, off" : : "v"(src), "{m0}"(l) : "memory");
}

typedef const __attribute__((address_space(4))) NucDesc CNucDesc;
typedef const __attribute__((address_space(4))) NucGroupDev CNucGroup;

constexpr int kNucWaves = 12;                   // 3 column tiles x 4 site phases
constexpr int kNucThreads = 64 * kNucWaves;
constexpr int kNucSites = 16;                   // sites per staged batch: one quad per phase
constexpr int kNucColGroups = kNTiles / 3;      // workgroups per work unit (column tiles 3j .. 3j+2)

__device__ __forceinline__ void split2(double x, __bf16 &h, __bf16 &l)
{
    h = (__bf16)(float)x;
    l = (__bf16)(float)(x - (double)(float)h);
}
__device__ __forceinline__ void split3(double x, __bf16 &h, __bf16 &m, __bf16 &l)
{
    h = (__bf16)(float)x;
    const double r = x - (double)(float)h;
    m = (__bf16)(float)r;
    l = (__bf16)(float)(r - (double)(float)m);
}

template <typename TIn, int NT, int MODE>
__global__ __launch_bounds__(kNucThreads) void blocks_nucleon_kernel(
    const TIn *__restrict__ Su, const TIn *__restrict__ Sd, const NucDesc *__restrict__ desc_one, int64_t V,
    int chunk_sites, int n_chunks_one, int K_one, int n_work, double2 *__restrict__ partial,
    const BatchBlockItem *__restrict__ bitems, const BatchBlockWork *__restrict__ bwork, int T)
{
    constexpr bool kSplit = MODE != WICK_P64;
    // two staging buffers [flavor][site][144] as distinct LDS variables, so the
    // compiler can tell the reads of one from the loads into the other
    __shared__ __attribute__((aligned(16))) TIn sbuf0[2][kNucSites][144];
    __shared__ __attribute__((aligned(16))) TIn sbuf1[2][kNucSites][144];
    // FP64 from complex64: a third buffer (three 36.9 KB buffers fit where two
    // complex128 ones do) for the staggered single-group loop below (in the
    // split modes its extra live rows spill, so they keep the two-buffer loop)
    constexpr bool kTriple = sizeof(TIn) == 8 && MODE == WICK_P64;
    __shared__ __attribute__((aligned(16))) TIn sbuf2[kTriple ? 2 : 1][kTriple ? kNucSites : 1][144];
    const int lbw = xcd_block();
    if (lbw >= n_work * kNucColGroups) return;
    // the kNucColGroups workgroups of one work unit are adjacent (one XCD, shared L2)
    const int lb = lbw / kNucColGroups, jg = lbw % kNucColGroups;
    // one plan: the workgroup's (cfg*T + t, chunk, pass) follow from its id;
    // a batch: from its work entry and its item's descriptor
    const NucDesc *desc_ptr;
    int pass, chunk, n_chunks, K;
    int64_t s_off, p_off;
    if (bwork) {
        const BatchBlockWork w = bwork[lb];
        const BatchBlockItem &it = bitems[w.item];
        desc_ptr = it.desc;
        pass = w.pass;
        chunk = w.chunk;
        n_chunks = it.n_chunks;
        K = it.K;
        s_off = it.s_off + (int64_t)w.t * V * 144;
        p_off = it.part_off + ((int64_t)w.t * n_chunks + chunk) * K * 1728;
    } else {
        desc_ptr = desc_one;
        n_chunks = n_chunks_one;
        K = K_one;
        pass = lb % desc_one->n_passes;
        chunk = (lb / desc_one->n_passes) % n_chunks;
        const int64_t ct = lb / desc_one->n_passes / n_chunks;
        s_off = ct * V * 144;
        p_off = (ct * n_chunks + chunk) * (int64_t)K * 1728;
    }
    // the descriptor is read through the constant address space: uniform scalar
    // loads (counted apart from the propagator loads in flight)
    const CNucDesc *desc = (const CNucDesc *)desc_ptr;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int ph = wv / 3, nt = 3 * jg + wv % 3;  // site phase, column tile
    const int lane = threadIdx.x & 63, q = lane >> 4, c = lane & 15;
    const int n = nt * 16 + c, i2 = n / 12, i3 = n % 12;
    const int npg = desc->pass_ngroups[pass];
    const __attribute__((address_space(4))) int32_t *tgroup = desc->tile_group[pass];

    // per tile: offset of this lane's Aop column inside a site's S_f (row 3*alpha, column i1);
    // padded columns (kind index past the group) read a valid entry and are never stored
    int bo[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int g = tgroup[t];
        bo[t] = 0;
        if (g >= 0) {
            const CNucGroup &G = desc->groups[g];
            const int m = desc->tile_mt[pass][t] * 16 + c;
            const int kk = m / 12 < G.nk ? m / 12 : G.nk - 1;
            // a twin kind reads its row from S_g: the other flavor's staging area
            bo[t] = (G.flv[kk] ? (G.g - G.f) * kNucSites * 144 : 0) + 36 * G.alpha[kk] + m % 12;
        }
    }
    // P64: acc[t] = (K1, K2) and acc3[t] = K3 of the three-product form;
    // the split modes: (Re, Im) in FP64
    d4 acc[NT][2], acc3[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t][0] = acc[t][1] = acc3[t] = d4{0, 0, 0, 0};

    const int64_t x0 = (int64_t)chunk * chunk_sites;
    const int64_t x1 = x0 + chunk_sites < V ? x0 + chunk_sites : V;
    const int nb = (int)((x1 - x0 + kNucSites - 1) / kNucSites);
    const TIn *const bu = Su + s_off, *const bd = Sd + s_off;
    // Staging of batch b into buffer buf, layout [flavor][site][144]. A full
    // batch goes from global memory straight to LDS (16 bytes per lane, no
    // registers): each wave-wide load covers 64 lanes x 16 bytes inside one
    // flavor, contiguous in global memory and in LDS. The ragged last batch
    // of a chunk goes through registers with zeros past the end (E = 0 there).
    constexpr int kFlavorEnt = kNucSites * 144;
    constexpr int kEntries = 2 * kFlavorEnt;
    constexpr int kLaneEnt = 16 / (int)sizeof(TIn);                // entries per lane and load
    constexpr int kWaveEnt = 64 * kLaneEnt;
    constexpr int kLoads = kEntries / (kNucThreads * kLaneEnt);    // loads per lane and batch
    static_assert(kEntries % (kNucThreads * kLaneEnt) == 0 && kFlavorEnt % kWaveEnt == 0,
                  "wave loads must tile the batch without crossing a flavor");
    auto issue = [&](int b, TIn *dst0) {
        const int64_t xb = x0 + (int64_t)b * kNucSites;
        if (xb + kNucSites <= x1) {
#pragma unroll
            for (int u = 0; u < kLoads; ++u) {
                const int e0 = (u * kNucWaves + wv) * kWaveEnt;  // wave-uniform first entry
                const int fl = e0 / kFlavorEnt;
                const TIn *src = (fl ? bd : bu) + xb * 144 + (e0 - fl * kFlavorEnt) + lane * kLaneEnt;
                lds_dma16(src, dst0 + e0);
            }
        } else {
            for (int e = threadIdx.x; e < kEntries; e += kNucThreads) {
                const int fl = e / kFlavorEnt, st = (e % kFlavorEnt) / 144, j = e % 144;
                TIn v{};
                if (xb + st < x1) v = (fl ? bd : bu)[(xb + st) * 144 + j];
                dst0[e] = v;
            }
        }
    };
    auto wait_staged = [] { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); };
    auto rd = [](const TIn *p) {
        const TIn v = *p;
        return double2{(double)v.x, (double)v.y};
    };
    issue(0, &sbuf0[0][0][0]);
    wait_staged();
    __syncthreads();
    // Split modes: the MFMAs of a group accumulate FP32 sums of E' * Aop with
    // E' = E * 2^-sc and Aop unscaled (a propagator entry is an FP32 number or
    // close to one). sc, the group's current scale, is the exponent of the
    // largest |E| of the wave (wave-uniform, so every MFMA sum has one scale);
    // it changes only when a batch's largest |E| moves more than kScaleSlack
    // binades away, and the FP32 sums are folded into the FP64 accumulators
    // with the exact factor 2^sc then, every kFoldBatches batches and at the
    // end. |E'| stays within 2^+-kScaleSlack of the wave's largest entry, so no
    // product leaves the FP32 range for any propagator magnitude.
    constexpr int kNoScale = -100000, kScaleSlack = 24, kFoldBatches = 4, kExpBias = 2048;
    f4 acc32[NT][2];  // FP32 sums of (Re, Im)
    int sc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        acc32[t][0] = acc32[t][1] = f4{0, 0, 0, 0};
        sc[t] = kNoScale;
    }
    int nfold = 0;
    // split modes: acc (FP64, (Re, Im)) += 2^sc * this tile's FP32 sums
    auto fold = [&](int t) {
        if constexpr (kSplit) {
            const double u = ldexp(1.0, sc[t]);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                acc[t][0][v] = fma((double)acc32[t][0][v], u, acc[t][0][v]);
                acc[t][1][v] = fma((double)acc32[t][1][v], u, acc[t][1][v]);
            }
            acc32[t][0] = acc32[t][1] = f4{0, 0, 0, 0};
        }
    };
    // one staged batch: this wave's site quad against every group of the pass
    // The diquark rows of group g (pass-group index gl) of this wave's site quad
    // in buffer buf, scaled for the split modes (the scale of the group is
    // settled here, folding its earlier sums when it changes).
    struct ERows {
        double e0x, e0y, e1x, e1y, e2x, e2y;
    };
    const int s = 4 * ph + q;  // this wave's site quad; sites past the end are zeros in LDS: E = 0
    auto group_e = [&](const TIn (*buf)[kNucSites][144], int gl) {
        const int g = desc->pass_groups[pass][gl];
        const CNucGroup &G = desc->groups[g];
        const TIn *sfb = buf[G.f][s];
        const TIn *sgb = buf[G.g][s];
        double e0x = 0, e0y = 0, e1x = 0, e1y = 0, e2x = 0, e2y = 0;
        // E_r += M * sum eps[r][c3][c2] a_c2 b_c3 with a = S_g(3 s2 + ., i2),
        // b = S_f(3 s3 + ., i3): E_0 += a2 b1 - a1 b2, E_1 += a0 b2 - a2 b0,
        // E_2 += a1 b0 - a0 b1, accumulated as FMA chains; M = -1 swaps the
        // roles of the two products, other values scale them
        auto cross = [&](int p, double sgn, double scale) {
            const TIn *pa = sgb + 36 * G.s2[p] + i2;
            const TIn *pb = sfb + 36 * G.s3[p] + i3;
            double2 a0 = rd(pa), a1 = rd(pa + 12), a2 = rd(pa + 24);
            const double2 b0 = rd(pb), b1 = rd(pb + 12), b2 = rd(pb + 24);
            if (scale != 1.0) {
                a0 = double2{a0.x * scale, a0.y * scale};
                a1 = double2{a1.x * scale, a1.y * scale};
                a2 = double2{a2.x * scale, a2.y * scale};
            }
            auto acc2 = [&](double &ex, double &ey, double2 u, double2 v, double s) {
                // (ex, ey) += s * u * v
                ex = fma(s * u.x, v.x, ex);
                ex = fma(-s * u.y, v.y, ex);
                ey = fma(s * u.x, v.y, ey);
                ey = fma(s * u.y, v.x, ey);
            };
            acc2(e0x, e0y, a2, b1, sgn);
            acc2(e0x, e0y, a1, b2, -sgn);
            acc2(e1x, e1y, a0, b2, sgn);
            acc2(e1x, e1y, a2, b0, -sgn);
            acc2(e2x, e2y, a1, b0, sgn);
            acc2(e2x, e2y, a0, b1, -sgn);
        };
        {
            int p = 0;
            for (; p < G.npos; ++p) cross(p, 1.0, 1.0);
            for (; p < G.npos + G.nneg; ++p) cross(p, -1.0, 1.0);
            for (; p < G.npair; ++p) cross(p, 1.0, (double)G.m[p]);
        }
        double fE = 1.0;  // split modes: E' = E * 2^-sc of this group
        if constexpr (kSplit) {
            const double m = fmax(fmax(fmax(fabs(e0x), fabs(e0y)), fmax(fabs(e1x), fabs(e1y))),
                                  fmax(fabs(e2x), fabs(e2y)));
            const int bw = __ockl_wfred_max_i32(m > 0.0 ? ilogb(m) + kExpBias : 0);
            int cur = kNoScale;
#pragma unroll
            for (int t = 0; t < NT; ++t)
                if (tgroup[t] == g) cur = sc[t];
            int want = cur;
            if (bw != 0) {
                const int x = min(max(bw - kExpBias, -1000), 1000);
                if (cur == kNoScale || x > cur + kScaleSlack || x < cur - kScaleSlack) want = x;
            } else if (cur == kNoScale) {
                want = 0;  // every E of the group is zero so far: any scale
            }
            if (want != cur) {
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    if (tgroup[t] == g) {
                        if (cur != kNoScale) fold(t);
                        sc[t] = want;
                    }
            }
            fE = ldexp(1.0, -want);
        }
        return ERows{e0x * fE, e0y * fE, e1x * fE, e1y * fE, e2x * fE, e2y * fE};
    };
    // the MFMAs of group g (pass-group index gl) with its diquark rows E and the
    // S_f rows of buffer buf
    auto group_mfma = [&](const ERows &E, const TIn (*buf)[kNucSites][144], int gl) {
        const int g = desc->pass_groups[pass][gl];
        const CNucGroup &G = desc->groups[g];
        const TIn *sfb = buf[G.f][s];
        const double fE = 1.0;  // E arrives scaled
        const double e0x = E.e0x, e0y = E.e0y, e1x = E.e1x, e1y = E.e1y, e2x = E.e2x, e2y = E.e2y;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const double ex = r == 0 ? e0x : (r == 1 ? e1x : e2x);
            const double ey = r == 0 ? e0y : (r == 1 ? e1y : e2y);
            if constexpr (MODE == WICK_P64) {
                const double exy = ex + ey;
                // every tile's entry first (a tile of another group reads
                // offset 0, inside the buffer), then the MFMAs
                double2 v[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) v[t] = rd(sfb + (tgroup[t] == g ? bo[t] : 0) + 12 * r);
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (tgroup[t] != g) continue;
                    acc[t][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(exy, v[t].x, acc[t][0], 0, 0, 0);
                    acc[t][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(ex, v[t].y - v[t].x, acc[t][1], 0, 0, 0);
                    acc3[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ey, v[t].x + v[t].y, acc3[t], 0, 0, 0);
                }
            } else if constexpr (MODE == WICK_P32) {
                // four real products in FP32 (Re += a c - b d, Im += a d + b c with
                // E' = a + ib and the S_f entry c + id); complex64 entries are
                // used as stored
                const float fa = (float)(ex * fE), fb = (float)(ey * fE);
                float vc[NT], vd[NT];
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const TIn e = sfb[(tgroup[t] == g ? bo[t] : 0) + 12 * r];
                    vc[t] = (float)e.x;
                    vd[t] = (float)e.y;
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (tgroup[t] != g) continue;
                    acc32[t][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, vc[t], acc32[t][0], 0, 0, 0);
                    acc32[t][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa, vd[t], acc32[t][1], 0, 0, 0);
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (tgroup[t] != g) continue;
                    acc32[t][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(-fb, vd[t], acc32[t][0], 0, 0, 0);
                    acc32[t][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(fb, vc[t], acc32[t][1], 0, 0, 0);
                }
            } else if constexpr (MODE == WICK_PB3) {
                __bf16 xh, xl, yh, yl;
                split2(ex * fE, xh, xl);
                split2(ey * fE, yh, yl);
                const __bf16 z = (__bf16)0.0f;
                const bf8 Aop = bf8{xh, xh, xl, yh, yh, yl, z, z};
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (tgroup[t] != g) continue;
                    const double2 d = rd(sfb + bo[t] + 12 * r);
                    __bf16 axh, axl, ayh, ayl;
                    split2(d.x, axh, axl);
                    split2(d.y, ayh, ayl);
                    const bf8 Bre = bf8{axh, axl, axh, -ayh, -ayl, -ayh, z, z};
                    const bf8 Bim = bf8{ayh, ayl, ayh, axh, axl, axh, z, z};
                    acc32[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, Bre, acc32[t][0], 0, 0, 0);
                    acc32[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Aop, Bim, acc32[t][1], 0, 0, 0);
                }
            } else {
                __bf16 xh, xm, xl, yh, ym, yl;
                split3(ex * fE, xh, xm, xl);
                split3(ey * fE, yh, ym, yl);
                const __bf16 z = (__bf16)0.0f;
                const bf8 Ax = bf8{xh, xh, xm, xh, xm, xl, z, z};
                const bf8 Ay = bf8{yh, yh, ym, yh, ym, yl, z, z};
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    if (tgroup[t] != g) continue;
                    const double2 d = rd(sfb + bo[t] + 12 * r);
                    __bf16 ah, am, al, bh, bm, bl;
                    split3(d.x, ah, am, al);
                    split3(d.y, bh, bm, bl);
                    const bf8 Bx = bf8{ah, am, ah, al, am, ah, z, z};
                    const bf8 By = bf8{bh, bm, bh, bl, bm, bh, z, z};
                    const bf8 nBy = bf8{-bh, -bm, -bh, -bl, -bm, -bh, z, z};
                    acc32[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ax, Bx, acc32[t][0], 0, 0, 0);
                    acc32[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ax, By, acc32[t][1], 0, 0, 0);
                    acc32[t][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ay, nBy, acc32[t][0], 0, 0, 0);
                    acc32[t][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ay, Bx, acc32[t][1], 0, 0, 0);
                }
            }
        }
    };
    auto count_fold = [&] {
        if constexpr (kSplit) {
            if (++nfold == kFoldBatches) {
                nfold = 0;
#pragma unroll
                for (int t = 0; t < NT; ++t)
                    if (sc[t] != kNoScale) fold(t);
            }
        }
    };
    // one staged batch: this wave's site quad against every group of the pass
    auto batch = [&](const TIn (*buf)[kNucSites][144]) {
#pragma unroll 1
        for (int gl = 0; gl < npg; ++gl) {
            const ERows E = group_e(buf, gl);
            group_mfma(E, buf, gl);
        }
        count_fold();
    };
    bool triple = false;
    if constexpr (kTriple) triple = npg == 1;
    if (!triple) {
        for (int b = 0; b < nb; b += 2) {
            if (b + 1 < nb) issue(b + 1, &sbuf1[0][0][0]);
            batch(sbuf0);
            wait_staged();
            __syncthreads();
            if (b + 1 >= nb) break;
            if (b + 2 < nb) issue(b + 2, &sbuf0[0][0][0]);
            batch(sbuf1);
            wait_staged();
            __syncthreads();
        }
    } else if constexpr (kTriple) {
        // Single-group pass, complex64: three buffers, batches b and b + 1
        // resident while b + 2 loads. The odd site phases run one step ahead on
        // the diquark rows: in step b they issue the MFMAs of batch b with rows
        // computed in step b - 1, then compute the rows of batch b + 1, so in
        // every step half the waves of a SIMD start with vector work and half
        // with MFMAs (64-configuration batch: FP64 blocks 37.8 -> 36.8 ms).
        const bool ahead = (ph & 1) != 0;
        if (nb > 1) issue(1, &sbuf1[0][0][0]);
        wait_staged();
        __syncthreads();
        ERows En = {};
        if (ahead) En = group_e(sbuf0, 0);
        // step b with its buffer, batch b + 1's buffer and the one batch b + 2
        // loads into, each a distinct LDS variable at every call site
        auto step = [&](int b, const TIn (*cur)[kNucSites][144], const TIn (*nxt)[kNucSites][144], TIn *load) {
            if (b + 2 < nb) issue(b + 2, load);
            if (!ahead) En = group_e(cur, 0);
            group_mfma(En, cur, 0);
            if (ahead && b + 1 < nb) En = group_e(nxt, 0);
            count_fold();
            wait_staged();
            __syncthreads();
        };
        for (int b = 0; b < nb; b += 3) {
            step(b, sbuf0, sbuf1, &sbuf2[0][0][0]);
            if (b + 1 >= nb) break;
            step(b + 1, sbuf1, sbuf2, &sbuf0[0][0][0]);
            if (b + 2 >= nb) break;
            step(b + 2, sbuf2, sbuf0, &sbuf1[0][0][0]);
        }
    }
    if constexpr (kSplit) {
#pragma unroll
        for (int t = 0; t < NT; ++t)
            if (sc[t] != kNoScale) fold(t);
    }
    if constexpr (MODE == WICK_P64) {
        // (K1, K2, K3) -> (Re, Im) = (K1 - K3, K1 + K2)
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double k1 = acc[t][0][v];
                acc[t][0][v] = k1 - acc3[t][v];
                acc[t][1][v] = k1 + acc[t][1][v];
            }
    }
    // sum the four site phases in a fixed order through LDS (the staging
    // buffers are free now): ((phase 3 + phase 2) + phase 1) + phase 0
    constexpr int kSlot = NT * 4 * 64;  // double2 per wave; slots 0, 1 in buffer 0, slot 2 in buffer 1
    static_assert(2 * kSlot * sizeof(double2) <= sizeof(sbuf0) && kSlot * sizeof(double2) <= sizeof(sbuf1),
                  "reduction slots must fit the staging buffers");
    const int a3 = wv % 3;
    double2 *slot = (a3 < 2 ? reinterpret_cast<double2 *>(&sbuf0[0][0][0]) + a3 * kSlot
                            : reinterpret_cast<double2 *>(&sbuf1[0][0][0])) + lane;
    for (int src = 3; src >= 1; --src) {
        if (ph == src) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) slot[(t * 4 + v) * 64] = double2{acc[t][0][v], acc[t][1][v]};
        }
        __syncthreads();
        if (ph == src - 1) {
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const double2 o = slot[(t * 4 + v) * 64];
                    acc[t][0][v] += o.x;
                    acc[t][1][v] += o.y;
                }
        }
        __syncthreads();
    }
    if (ph != 0) return;
    double2 *P = partial + p_off;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (tgroup[t] < 0) continue;
        const CNucGroup &G = desc->groups[tgroup[t]];
        const int m = desc->tile_mt[pass][t] * 16 + c, kk = m / 12, i1 = m % 12;
        if (kk >= G.nk) continue;
        double2 *row = P + ((int64_t)G.kind_out[kk] * 12 + i1) * 144;
        const bool tr = G.tr[kk] != 0;
        // f64 MFMA result: column 4*v + q of the tile; f32 / bf16 MFMA result: 4*q + v.
        // A twin kind's column (i2, i3) is (i3, i2) of its own block.
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = nt * 16 + (kSplit ? 4 * q + v : 4 * v + q);
            row[tr ? (col % 12) * 12 + col / 12 : col] = double2{acc[t][0][v], acc[t][1][v]};
        }
    }
}

// Sum the chunks in order and antisymmetrise: B[c] = sum_ch P[i1][i2,i3] - P[i3][i2,i1].
__global__ __launch_bounds__(256) void blocks_reduce_kernel(const double2 *__restrict__ partial, int n_chunks,
                                                            int K, int64_t n_out, double2 *__restrict__ B)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n_out) return;
    const int per = K * 792;
    const int64_t ct = idx / per;
    const int e = (int)(idx % per);
    const int kind = e / 792, cc = e % 792, pr = cc / 12, i2 = cc % 12;
    int i3 = 1;
    while ((i3 + 1) * i3 / 2 <= pr) ++i3;
    const int i1 = pr - i3 * (i3 - 1) / 2;
    const double2 *P = partial + ct * n_chunks * (int64_t)K * 1728 + (int64_t)kind * 1728;
    const int oa = i1 * 144 + i2 * 12 + i3, ob = i3 * 144 + i2 * 12 + i1;
    double sx = 0.0, sy = 0.0;
    for (int ch = 0; ch < n_chunks; ++ch) {
        const double2 a = P[(int64_t)ch * K * 1728 + oa];
        const double2 b = P[(int64_t)ch * K * 1728 + ob];
        sx += a.x - b.x;
        sy += a.y - b.y;
    }
    B[idx] = double2{sx, sy};
}

template <int A, bool REAL>
__global__ __launch_bounds__(256) void contract_kernel(const double2 *__restrict__ B, const uint16_t *__restrict__ kidx,
                                                       const double *__restrict__ coef, int64_t N, int K, int n_ct,
                                                       int n_slices, int64_t slice_len, double2 *__restrict__ partial)
{
    __shared__ double red[2][4];
    const int lb = xcd_block();
    if (lb >= n_ct * n_slices) return;
    const int ct = lb / n_slices, slice = lb % n_slices;
    const double2 *Bc = B + (int64_t)ct * K * 792;
    const double2 *src = Bc;
    const int64_t n0 = (int64_t)slice * slice_len;
    const int64_t n1 = n0 + slice_len < N ? n0 + slice_len : N;
    double ar = 0.0, ai = 0.0;
    for (int64_t n = n0 + threadIdx.x; n < n1; n += blockDim.x) {
        double2 p = src[kidx[n]];
#pragma unroll
        for (int a = 1; a < A; ++a) {
            const double2 b = src[kidx[(int64_t)a * N + n]];
            p = double2{p.x * b.x - p.y * b.y, p.x * b.y + p.y * b.x};
        }
        if (REAL) {
            const double c = coef[n];
            ar += c * p.x;
            ai += c * p.y;
        } else {
            const double cr = coef[2 * n], ci = coef[2 * n + 1];
            ar += cr * p.x - ci * p.y;
            ai += cr * p.y + ci * p.x;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ar += __shfl_xor(ar, off);
        ai += __shfl_xor(ai, off);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = ar;
        red[1][w] = ai;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sr = 0.0, si = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
            sr += red[0][i];
            si += red[1][i];
        }
        partial[(int64_t)ct * n_slices + slice] = double2{sr, si};
    }
}

// Term sum with the blocks of ntg <= kMaxTG consecutive time slices in LDS:
// each term's word (or plain indices and coefficient) is read once and
// evaluated for every staged slice.
template <int A, bool PACKED, bool REAL = false>
__device__ __forceinline__ void term_sum(const double2 *__restrict__ sB, int KB, int ntg,
                                         const double2 *__restrict__ spal, const TermTable &tab, int64_t N,
                                         int64_t n0, int64_t n1, double (&ar)[kMaxTG], double (&ai)[kMaxTG])
{
    auto eval = [&](const int (&idx)[A], double cx, double cy) {
#pragma unroll
        for (int tg = 0; tg < kMaxTG; ++tg) {
            if (tg < ntg) {
                const double2 *Bt = sB + tg * KB;
                double2 p = Bt[idx[0]];
#pragma unroll
                for (int a = 1; a < A; ++a) {
                    const double2 b = Bt[idx[a]];
                    p = double2{p.x * b.x - p.y * b.y, p.x * b.y + p.y * b.x};
                }
                if constexpr (REAL) {
                    ar[tg] += cx * p.x;
                    ai[tg] += cx * p.y;
                } else {
                    ar[tg] += cx * p.x - cy * p.y;
                    ai[tg] += cx * p.y + cy * p.x;
                }
            }
        }
    };
    if constexpr (PACKED) {
        // this thread's terms n0 + tid + k * kCThreads; the words of the next
        // kPrefetch terms are loaded while the current ones are evaluated
        const int64_t first = n0 + threadIdx.x;
        const int64_t cnt = first < n1 ? (n1 - first + kCThreads - 1) / kCThreads : 0;
        uint64_t cur[kPrefetch], nxt[kPrefetch] = {};
        auto fetch = [&](int64_t k0, uint64_t (&w)[kPrefetch]) {
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) w[u] = k0 + u < cnt ? tab.words[first + (k0 + u) * kCThreads] : 0;
        };
        fetch(0, cur);
        for (int64_t k0 = 0; k0 < cnt; k0 += kPrefetch) {
            if (k0 + kPrefetch < cnt) fetch(k0 + kPrefetch, nxt);
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                if (k0 + u < cnt) {
                    const uint64_t w = cur[u];
                    int idx[A];
#pragma unroll
                    for (int a = 0; a < A; ++a) idx[a] = (int)(w >> (kPackBits * a)) & ((1 << kPackBits) - 1);
                    const double2 c = spal[(int)(w >> 56)];
                    eval(idx, c.x, c.y);
                }
            }
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) cur[u] = nxt[u];
        }
    } else {
        for (int64_t n = n0 + threadIdx.x; n < n1; n += kCThreads) {
            int idx[A];
#pragma unroll
            for (int a = 0; a < A; ++a) idx[a] = tab.kidx[(int64_t)a * N + n];
            if (tab.coef_real) eval(idx, tab.coef[n], 0.0);
            else eval(idx, tab.coef[2 * n], tab.coef[2 * n + 1]);
        }
    }
}

// Term sum over the chunks [c0, c1) of a segmented table: wave w of the
// workgroup takes chunks c0 + w, c0 + w + 16, ...; each lane evaluates its
// segment of the chunk for every staged slice (see TermTable). The words of
// the next kPrefetch / kNodeLeaves nodes are loaded while the current ones
// are evaluated.
template <int A, bool REAL>
__device__ __forceinline__ void term_sum_seg(const double2 *__restrict__ sB, int KB, int ntg,
                                             const double2 *__restrict__ spal, const TermTable &tab, int c0, int c1,
                                             double (&ar)[kMaxTG], double (&ai)[kMaxTG])
{
    constexpr uint32_t kMask = (1u << kPackBits) - 1;
    static_assert(kNodeLeaves == 2, "one 64-bit word per node holds two leaves");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = c0 + wave; c < c1; c += kCThreads / 64) {
        const uint32_t pre = tab.seg_prefix[(int64_t)c * 64 + lane];
        double px[kMaxTG], py[kMaxTG], sx[kMaxTG], sy[kMaxTG];
#pragma unroll
        for (int tg = 0; tg < kMaxTG; ++tg) {
            px[tg] = 1.0;
            py[tg] = 0.0;
            sx[tg] = sy[tg] = 0.0;
            if (tg < ntg) {
#pragma unroll
                for (int a = 0; a < A - 2; ++a) {
                    const double2 b = sB[tg * KB + ((pre >> (kPackBits * a)) & kMask)];
                    const double x = px[tg] * b.x - py[tg] * b.y;
                    py[tg] = px[tg] * b.y + py[tg] * b.x;
                    px[tg] = x;
                }
            }
        }
        const uint64_t *wp = tab.words + tab.chunk_base[c] + lane;
        const int nodes = tab.chunk_len[c] & 0xffff;  // uniform over the wave
        uint64_t cur[kPrefetch], nxt[kPrefetch] = {};
        auto fetch = [&](int k0, uint64_t (&w)[kPrefetch]) {
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) w[u] = k0 + u < nodes ? wp[(int64_t)(k0 + u) * 64] : 0;
        };
        fetch(0, cur);
        for (int k0 = 0; k0 < nodes; k0 += kPrefetch) {
            if (k0 + kPrefetch < nodes) fetch(k0 + kPrefetch, nxt);
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) {
                if (k0 + u < nodes) {
                    const uint64_t w = cur[u];
                    const int in = (int)((w >> kPackBits) & kMask);
                    const int l0 = (int)(w & kMask), l1 = (int)((w >> 36) & kMask);
                    const double2 c0v = spal[(int)(w >> 28) & 0xff], c1v = spal[(int)(w >> 50) & 0xff];
#pragma unroll
                    for (int tg = 0; tg < kMaxTG; ++tg) {
                        if (tg < ntg) {
                            const double2 *Bt = sB + tg * KB;
                            const double2 b0 = Bt[l0], b1 = Bt[l1], bn = Bt[in];
                            double s3x, s3y;
                            if constexpr (REAL) {
                                s3x = fma(c1v.x, b1.x, c0v.x * b0.x);
                                s3y = fma(c1v.x, b1.y, c0v.x * b0.y);
                            } else {
                                s3x = c0v.x * b0.x - c0v.y * b0.y + c1v.x * b1.x - c1v.y * b1.y;
                                s3y = c0v.x * b0.y + c0v.y * b0.x + c1v.x * b1.y + c1v.y * b1.x;
                            }
                            sx[tg] += bn.x * s3x - bn.y * s3y;
                            sy[tg] += bn.x * s3y + bn.y * s3x;
                        }
                    }
                }
            }
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) cur[u] = nxt[u];
        }
#pragma unroll
        for (int tg = 0; tg < kMaxTG; ++tg) {
            if (tg < ntg) {
                ar[tg] += px[tg] * sx[tg] - py[tg] * sy[tg];
                ai[tg] += px[tg] * sy[tg] + py[tg] * sx[tg];
            }
        }
    }
}

// Term sum over the chunks [c0, c1) of a segmented table with
// integer-coefficient words, for NTG staged slices (a compile-time count, so
// that the gathers of every slice are issued together and one wait covers
// them). The slices' blocks are interleaved in LDS, entry e of slice s at
// sB[e * NTG + s] (stage_blocks_interleaved), so the NTG gathers of one entry
// share one address and differ by an immediate offset. The first `two` steps
// of a chunk gather both leaves of each lane's word (a missing leaf 1, q = 0,
// reads entry 0 and weighs it by zero; lanes reading one address share the
// read); in the later steps no lane's word has a leaf 1 and its gather is
// skipped, a branch taken by the whole wave. A padding word reads entry 0 with
// weight zero. The coefficients are the integers q; the table's unit
// multiplies each segment's sum once. Chunk index, length and base are the
// same for the whole wave and held in scalar registers, so the loop control
// and the word addresses cost no vector instructions.
// A = 4 tables are factored (chunk_g): the first ng = chunk_g[c] steps of a
// chunk sum the lane's prefix group G (one-leaf words), the later ones its
// list M, and the lane adds unit * G * M; there is no prefix product.
template <int A, int NTG>
__device__ __forceinline__ void term_sum_segi(const double2 *__restrict__ sB, const TermTable &tab, int c0, int c1,
                                              double (&ar)[kMaxTG], double (&ai)[kMaxTG])
{
    constexpr uint32_t kMask = (1u << kPackBits) - 1;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    c0 = __builtin_amdgcn_readfirstlane(c0);
    c1 = __builtin_amdgcn_readfirstlane(c1);
    constexpr bool kFactored = A == 4;
    const double unit = (double)tab.coef_unit;
    for (int c = c0 + wave; c < c1; c += kCThreads / 64) {
        double sx[NTG], sy[NTG], gx[NTG], gy[NTG];
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg) sx[tg] = sy[tg] = gx[tg] = gy[tg] = 0.0;
        const int cl = __builtin_amdgcn_readfirstlane(tab.chunk_len[c]);
        const int nodes = cl & 0xffff, two = cl >> 16;
        const int ng = kFactored ? __builtin_amdgcn_readfirstlane(tab.chunk_g[c]) : 0;
        // factored: the sum so far is the prefix group's; the list's starts
        auto take_g = [&] {
#pragma unroll
            for (int tg = 0; tg < NTG; ++tg) {
                gx[tg] = sx[tg];
                gy[tg] = sy[tg];
                sx[tg] = sy[tg] = 0.0;
            }
        };
        const uint64_t *wp = tab.words + tab.chunk_base[c] + lane;
        auto eval = [&](uint64_t w, auto leaf1) {
            constexpr bool kLeaf1 = decltype(leaf1)::value;
            const double2 *pn = sB + (int)((w >> kPackBits) & kMask) * NTG;
            const double2 *p0 = sB + (int)(w & kMask) * NTG;
            // q of leaf 0 is bits [42, 53) and q of leaf 1 bits [53, 64) of the
            // word: bits [10, 21) and [21, 32) of its high half (32-bit
            // arithmetic shifts sign-extend them)
            const uint32_t hi = (uint32_t)(w >> 32);
            const double cf0 = (double)((int)(hi << 11) >> 21);
            double2 b0[NTG], b1[NTG], bn[NTG];
#pragma unroll
            for (int tg = 0; tg < NTG; ++tg) {
                bn[tg] = pn[tg];
                b0[tg] = p0[tg];
            }
            if constexpr (kLeaf1) {
                const double2 *p1 = sB + (int)((w >> (2 * kPackBits)) & kMask) * NTG;
#pragma unroll
                for (int tg = 0; tg < NTG; ++tg) b1[tg] = p1[tg];
            }
#pragma unroll
            for (int tg = 0; tg < NTG; ++tg) {
                double s3x, s3y;
                if constexpr (kLeaf1) {
                    const double cf1 = (double)((int)hi >> 21);
                    s3x = fma(cf1, b1[tg].x, cf0 * b0[tg].x);
                    s3y = fma(cf1, b1[tg].y, cf0 * b0[tg].y);
                } else {
                    s3x = cf0 * b0[tg].x;
                    s3y = cf0 * b0[tg].y;
                }
                sx[tg] = fma(bn[tg].x, s3x, sx[tg]);
                sx[tg] = fma(-bn[tg].y, s3y, sx[tg]);
                sy[tg] = fma(bn[tg].x, s3y, sy[tg]);
                sy[tg] = fma(bn[tg].y, s3x, sy[tg]);
            }
        };
        constexpr std::true_type kBoth{};
        constexpr std::false_type kLeaf0{};
        // the words of the next kPrefetch nodes are loaded while the current
        // ones are evaluated (indices clamped into the chunk: always valid)
        uint64_t cur[kPrefetch], nxt[kPrefetch];
        auto fetch = [&](int k0, uint64_t (&w)[kPrefetch]) {
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) w[u] = wp[(int64_t)(k0 + u < nodes ? k0 + u : nodes - 1) * 64];
        };
        if (nodes > 0) fetch(0, cur);
        for (int k0 = 0; k0 < nodes; k0 += kPrefetch) {
            if (k0 + kPrefetch < nodes) fetch(k0 + kPrefetch, nxt);
            // steps [0, ng): prefix-group words (factored; one leaf), [ng, two):
            // list words with two leaves in some lane, [two, nodes): one leaf
            if (kFactored && k0 == ng) take_g();
            const int hi = k0 + kPrefetch;
            if (hi <= ng || (k0 >= two && hi <= nodes)) {
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u) eval(cur[u], kLeaf0);
            } else if (k0 >= ng && hi <= two) {
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u) eval(cur[u], kBoth);
            } else {  // the steps where G or leaf 1 ends, or the chunk's last steps
#pragma unroll
                for (int u = 0; u < kPrefetch; ++u) {
                    const int j = k0 + u;
                    if (kFactored && u > 0 && j == ng) take_g();
                    if (j < ng) eval(cur[u], kLeaf0);
                    else if (j < two) eval(cur[u], kBoth);
                    else if (j < nodes) eval(cur[u], kLeaf0);
                }
            }
#pragma unroll
            for (int u = 0; u < kPrefetch; ++u) cur[u] = nxt[u];
        }
        if constexpr (kFactored) {
            if (ng >= nodes) take_g();  // no list steps (not built; kept for safety)
#pragma unroll
            for (int tg = 0; tg < NTG; ++tg) {
                const double px = unit * gx[tg], py = unit * gy[tg];
                ar[tg] += px * sx[tg] - py * sy[tg];
                ai[tg] += px * sy[tg] + py * sx[tg];
            }
        } else {
            const uint32_t pre = tab.seg_prefix[(int64_t)c * 64 + lane];
#pragma unroll
            for (int tg = 0; tg < NTG; ++tg) {
                double px = unit, py = 0.0;
#pragma unroll
                for (int a = 0; a < A - 2; ++a) {
                    const double2 b = sB[(int)((pre >> (kPackBits * a)) & kMask) * NTG + tg];
                    const double x = px * b.x - py * b.y;
                    py = px * b.y + py * b.x;
                    px = x;
                }
                ar[tg] += px * sx[tg] - py * sy[tg];
                ai[tg] += px * sy[tg] + py * sx[tg];
            }
        }
    }
}

template <int A>
__device__ __forceinline__ void term_sum_segi_n(const double2 *__restrict__ sB, int ntg, const TermTable &tab, int c0,
                                                int c1, double (&ar)[kMaxTG], double (&ai)[kMaxTG])
{
    static_assert(kMaxTG == 3, "one instance per slice count");
    if (ntg == 3) term_sum_segi<A, 3>(sB, tab, c0, c1, ar, ai);
    else if (ntg == 2) term_sum_segi<A, 2>(sB, tab, c0, c1, ar, ai);
    else term_sum_segi<A, 1>(sB, tab, c0, c1, ar, ai);
}

// Stage ntg slices of KB block entries each (contiguous in B), interleaved:
// entry e of slice t at sB[e * ntg + t] (integer-coefficient segmented tables).
__device__ __forceinline__ void stage_blocks_interleaved(const double2 *__restrict__ Bsrc, int KB, int ntg,
                                                         double2 *__restrict__ sB)
{
    for (int i = threadIdx.x; i < ntg * KB; i += kCThreads) {
        const int t = i / KB, e = i - t * KB;
        sB[e * ntg + t] = Bsrc[i];
    }
    __syncthreads();
}

// Stage ntg slices of K blocks (contiguous in B) and the palette.
__device__ __forceinline__ void stage_blocks(const double2 *__restrict__ Bsrc, int n, const TermTable &tab,
                                             double2 *__restrict__ sB, double2 *__restrict__ spal)
{
    for (int i = threadIdx.x; i < n; i += kCThreads) sB[i] = Bsrc[i];
    if (tab.words)
        for (int i = threadIdx.x; i < tab.n_pal; i += kCThreads) spal[i] = tab.pal[i];
    __syncthreads();
}

// Workgroup sum of each slice's accumulators in a fixed order; out[tg * stride].
__device__ __forceinline__ void reduce_tg(double (&ar)[kMaxTG], double (&ai)[kMaxTG], int ntg,
                                          double (*red)[2][kCThreads / 64], double2 *__restrict__ out,
                                          int64_t stride)
{
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int tg = 0; tg < kMaxTG; ++tg) {
        if (tg < ntg) {
            double x = ar[tg], y = ai[tg];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                x += __shfl_xor(x, off);
                y += __shfl_xor(y, off);
            }
            if ((threadIdx.x & 63) == 0) {
                red[tg][0][w] = x;
                red[tg][1][w] = y;
            }
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < ntg) {
        const int tg = threadIdx.x;
        double sr = 0.0, si = 0.0;
        for (int i = 0; i < kCThreads / 64; ++i) {
            sr += red[tg][0][i];
            si += red[tg][1][i];
        }
        out[tg * stride] = double2{sr, si};
    }
}

// One plan: workgroup (group of tg consecutive (cfg, t) sets, table slice);
// a slice is slice_len terms (plain, packed) or slice_len chunks (segmented).
// FORM: 0 plain, 1 packed, 2 segmented, 3 packed with a real palette,
// 4 segmented with a real palette, 5 segmented with integer coefficients.
template <int A, int FORM>
__global__ __launch_bounds__(kCThreads) void contract_tg_kernel(const double2 *__restrict__ B, TermTable tab,
                                                                int64_t N, int K, int n_ct, int tg, int n_slices,
                                                                int64_t slice_len, double2 *__restrict__ partial,
                                                                int share)
{
    extern __shared__ double2 lds[];
    __shared__ double red[kMaxTG][2][kCThreads / 64];
    const int n_groups = (n_ct + tg - 1) / tg;
    const int lb = xcd_block();
    if (lb >= n_groups * n_slices) return;
    // share = 1: group-major (adjacent workgroups share their staged blocks);
    // share = h > 1: h adjacent workgroups (one XCD) take h groups of slices
    // at one table slice, so the slice is read from HBM about once per h
    // groups and shared through that XCD's L2
    int g, slice;
    {
        const int h = share < 1 ? 1 : (share > n_groups ? n_groups : share);
        const int full = n_groups / h, rem = n_groups % h;
        if (lb < full * h * n_slices) {
            const int rest = lb / h;
            slice = rest % n_slices;
            g = (rest / n_slices) * h + lb % h;
        } else {
            const int l2 = lb - full * h * n_slices;
            slice = l2 / rem;
            g = full * h + l2 % rem;
        }
    }
    const int ct0 = g * tg, ntg = n_ct - ct0 < tg ? n_ct - ct0 : tg;
    const int KB = K * 792;
    double2 *spal = lds, *sB = lds + kMaxPalette;
    if constexpr (FORM == 5) stage_blocks_interleaved(B + (int64_t)ct0 * KB, KB, ntg, sB);
    else stage_blocks(B + (int64_t)ct0 * KB, ntg * KB, tab, sB, spal);
    double ar[kMaxTG] = {}, ai[kMaxTG] = {};
    if constexpr (FORM == 2 || FORM == 4 || FORM == 5) {
        const int c0 = (int)(slice * slice_len);
        const int c1 = c0 + slice_len < tab.n_chunks ? (int)(c0 + slice_len) : tab.n_chunks;
        if constexpr (FORM == 5) term_sum_segi_n<A>(sB, ntg, tab, c0, c1, ar, ai);
        else term_sum_seg<A, FORM == 4>(sB, KB, ntg, spal, tab, c0, c1, ar, ai);
    } else {
        const int64_t n0 = (int64_t)slice * slice_len;
        const int64_t n1 = n0 + slice_len < N ? n0 + slice_len : N;
        term_sum<A, FORM == 1 || FORM == 3, FORM == 3>(sB, KB, ntg, spal, tab, N, n0, n1, ar, ai);
    }
    reduce_tg(ar, ai, ntg, red, partial + (int64_t)ct0 * n_slices + slice, n_slices);
}

__global__ void zero_kernel(double *__restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ void contract_finalize_kernel(const double2 *__restrict__ partial, int n_ct, int n_slices,
                                         double2 *__restrict__ C)
{
    const int ct = blockIdx.x * blockDim.x + threadIdx.x;
    if (ct >= n_ct) return;
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < n_slices; ++s) {
        const double2 v = partial[(int64_t)ct * n_slices + s];
        sr += v.x;
        si += v.y;
    }
    C[ct] = double2{sr, si};
}


// ------------------------------------------------------------------ batches
// Reduction of a batch's partial blocks: one thread per output entry of all
// items; the item of an entry is found by binary search in the prefix table.
__global__ __launch_bounds__(256) void batch_reduce_kernel(const double2 *__restrict__ partial,
                                                           const BatchBlockItem *__restrict__ items,
                                                           const int64_t *__restrict__ out_off, int n_items,
                                                           int T, int64_t idx0, int64_t n_out, double2 *__restrict__ B)
{
    const int64_t idx = idx0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // outputs [idx0, idx0 + n_out)
    if (idx >= idx0 + n_out) return;
    int lo = 0, hi = n_items - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (out_off[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    const BatchBlockItem &it = items[lo];
    const int64_t r = idx - out_off[lo];
    const int per = it.K * 792;
    const int t = (int)(r / per);
    const int e = (int)(r % per);
    const int kind = e / 792, cc = e % 792, pr = cc / 12, i2 = cc % 12;
    int i3 = 1;
    while ((i3 + 1) * i3 / 2 <= pr) ++i3;
    const int i1 = pr - i3 * (i3 - 1) / 2;
    const double2 *P = partial + it.part_off + (int64_t)t * it.n_chunks * it.K * 1728 + (int64_t)kind * 1728;
    const int oa = i1 * 144 + i2 * 12 + i3, ob = i3 * 144 + i2 * 12 + i1;
    double sx = 0.0, sy = 0.0;
    for (int ch = 0; ch < it.n_chunks; ++ch) {
        const double2 a = P[(int64_t)ch * it.K * 1728 + oa];
        const double2 b = P[(int64_t)ch * it.K * 1728 + ob];
        sx += a.x - b.x;
        sy += a.y - b.y;
    }
    B[idx] = double2{sx, sy};
}

// Term sum of a batch: one workgroup per (item, first time slice, table
// slice) work entry; A, the number of kinds, the slices per workgroup and
// the table form are read from the item.
__global__ __launch_bounds__(kCThreads) void contract_batch_kernel(const double2 *__restrict__ B,
                                                                   const BatchContractItem *__restrict__ items,
                                                                   const BatchContractWork *__restrict__ work,
                                                                   int n_work, double2 *__restrict__ partial)
{
    extern __shared__ double2 lds[];
    __shared__ double red[kMaxTG][2][kCThreads / 64];
    const int lb = xcd_block();
    if (lb >= n_work) return;
    const BatchContractWork w = work[lb];
    const BatchContractItem &it = items[w.item];
    const int KB = it.K * 792, ntg = w.ntg;
    double2 *spal = lds, *sB = lds + kMaxPalette;
    if (it.tab.seg_prefix && it.tab.coef_unit) stage_blocks_interleaved(B + it.b_off + (int64_t)w.t0 * KB, KB, ntg, sB);
    else stage_blocks(B + it.b_off + (int64_t)w.t0 * KB, ntg * KB, it.tab, sB, spal);
    double ar[kMaxTG] = {}, ai[kMaxTG] = {};
    if (it.tab.seg_prefix) {
        const int c0 = (int)(w.slice * it.slice_len);
        const int c1 = c0 + it.slice_len < it.tab.n_chunks ? (int)(c0 + it.slice_len) : it.tab.n_chunks;
        switch (it.tab.coef_unit ? 10 + it.A : it.A * 2 + (it.tab.coef_real ? 1 : 0)) {
        case 12: term_sum_segi_n<2>(sB, ntg, it.tab, c0, c1, ar, ai); break;
        case 13: term_sum_segi_n<3>(sB, ntg, it.tab, c0, c1, ar, ai); break;
        case 14: term_sum_segi_n<4>(sB, ntg, it.tab, c0, c1, ar, ai); break;
        case 4: term_sum_seg<2, false>(sB, KB, ntg, spal, it.tab, c0, c1, ar, ai); break;
        case 5: term_sum_seg<2, true>(sB, KB, ntg, spal, it.tab, c0, c1, ar, ai); break;
        case 6: term_sum_seg<3, false>(sB, KB, ntg, spal, it.tab, c0, c1, ar, ai); break;
        case 7: term_sum_seg<3, true>(sB, KB, ntg, spal, it.tab, c0, c1, ar, ai); break;
        case 8: term_sum_seg<4, false>(sB, KB, ntg, spal, it.tab, c0, c1, ar, ai); break;
        case 9: term_sum_seg<4, true>(sB, KB, ntg, spal, it.tab, c0, c1, ar, ai); break;
        default: break;
        }
        reduce_tg(ar, ai, ntg, red, partial + it.part_off + (int64_t)w.t0 * it.n_slices + w.slice, it.n_slices);
        return;
    }
    const int64_t n0 = (int64_t)w.slice * it.slice_len;
    const int64_t n1 = n0 + it.slice_len < it.N ? n0 + it.slice_len : it.N;
    const int form = it.tab.words ? (it.tab.coef_real ? 3 : 1) : 0;
    switch (it.A * 4 + form) {
    case 4: term_sum<1, false>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 5: term_sum<1, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 7: term_sum<1, true, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 8: term_sum<2, false>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 9: term_sum<2, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 11: term_sum<2, true, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 12: term_sum<3, false>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 13: term_sum<3, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 15: term_sum<3, true, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 16: term_sum<4, false>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 17: term_sum<4, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 19: term_sum<4, true, true>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    case 20: term_sum<5, false>(sB, KB, ntg, spal, it.tab, it.N, n0, n1, ar, ai); break;
    default: break;
    }
    reduce_tg(ar, ai, ntg, red, partial + it.part_off + (int64_t)w.t0 * it.n_slices + w.slice, it.n_slices);
}

__global__ void batch_finalize_kernel(const double2 *__restrict__ partial,
                                      const BatchContractItem *__restrict__ items, int i0, int n_items, int T,
                                      double2 *__restrict__ C)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;  // items [i0, i0 + n_items)
    if (idx >= n_items * T) return;
    const int i = i0 + idx / T, t = idx % T;
    const BatchContractItem &it = items[i];
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < it.n_slices; ++s) {
        const double2 v = partial[it.part_off + (int64_t)t * it.n_slices + s];
        sr += v.x;
        si += v.y;
    }
    C[(int64_t)it.out_item * T + t] = double2{sr, si};
}

int round8(int64_t n) { return (int)((n + 7) / 8 * 8); }

}  // namespace

hipError_t launch_blocks(const BlockLaunch &L, hipStream_t s)
{
    const int n_units = L.n_groups * kNTiles;
    const int64_t n_ct = (int64_t)L.n_cfg * L.T;
    Probe pr("blocks", s);
    if (L.nuc) {
        const int64_t work = n_ct * L.n_chunks * L.nuc_passes;
        if (work * kNucColGroups > 0x7ffffff0LL) return hipErrorInvalidValue;
        const unsigned blocks = (unsigned)round8(work * kNucColGroups);
        bool done = false;
#define WICK_NUC(NTV, MODE)                                                                                       \
    if (L.nuc_tiles == NTV && L.prec == MODE) {                                                                   \
        if (L.dtype == 0)                                                                                         \
            hipLaunchKernelGGL((blocks_nucleon_kernel<double2, NTV, MODE>), dim3(blocks), dim3(kNucThreads), 0,    \
                               s, (const double2 *)L.Su, (const double2 *)L.Sd, L.nuc, L.V, L.chunk_sites,         \
                               L.n_chunks, L.K, (int)work, (double2 *)L.partial, nullptr, nullptr, L.T);         \
        else                                                                                                      \
            hipLaunchKernelGGL((blocks_nucleon_kernel<float2, NTV, MODE>), dim3(blocks), dim3(kNucThreads), 0,     \
                               s, (const float2 *)L.Su, (const float2 *)L.Sd, L.nuc, L.V, L.chunk_sites,           \
                               L.n_chunks, L.K, (int)work, (double2 *)L.partial, nullptr, nullptr, L.T);         \
        done = true;                                                                                              \
    }
        WICK_NUC(1, WICK_P64) WICK_NUC(2, WICK_P64) WICK_NUC(3, WICK_P64) WICK_NUC(4, WICK_P64)
        WICK_NUC(1, WICK_P32) WICK_NUC(2, WICK_P32) WICK_NUC(3, WICK_P32)
        WICK_NUC(1, WICK_PB3) WICK_NUC(2, WICK_PB3) WICK_NUC(3, WICK_PB3)
        WICK_NUC(1, WICK_PB6) WICK_NUC(2, WICK_PB6) WICK_NUC(3, WICK_PB6)
#undef WICK_NUC
        if (!done) return hipErrorInvalidValue;
    } else if (L.desc) {
        const int64_t work = n_ct * L.n_chunks * L.n_passes;
        if (work > 0x7ffffff0LL) return hipErrorInvalidValue;
        const unsigned blocks = (unsigned)round8(work);
        switch (L.n_tiles) {
#define WICK_STAGED(NTV)                                                                                          \
    case NTV:                                                                                                     \
        if (L.dtype == 0)                                                                                         \
            hipLaunchKernelGGL((blocks_f64_staged_kernel<double2, NTV>), dim3(blocks), dim3(kStagedThreads), 0, s, \
                               (const double2 *)L.Su, (const double2 *)L.Sd, L.desc, L.V, L.chunk_sites,         \
                               L.n_chunks, L.K, (int)work, (double2 *)L.partial);                                \
        else                                                                                                      \
            hipLaunchKernelGGL((blocks_f64_staged_kernel<float2, NTV>), dim3(blocks), dim3(kStagedThreads), 0, s,  \
                               (const float2 *)L.Su, (const float2 *)L.Sd, L.desc, L.V, L.chunk_sites,           \
                               L.n_chunks, L.K, (int)work, (double2 *)L.partial);                                \
        break;
            WICK_STAGED(1) WICK_STAGED(2) WICK_STAGED(3) WICK_STAGED(4)
#undef WICK_STAGED
        default: return hipErrorInvalidValue;
        }
    } else {
        const int64_t waves = (int64_t)n_units * L.n_chunks * n_ct;
        const int wpb = 4;
        const int64_t blocks = round8((waves + wpb - 1) / wpb);
        if (blocks > 0x7fffffff) return hipErrorInvalidValue;
        if (L.dtype == 0)
            hipLaunchKernelGGL(blocks_f64_kernel<double2>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s,
                               (const double2 *)L.Su, (const double2 *)L.Sd, L.groups, n_units, L.V, L.chunk_sites,
                               L.n_chunks, L.K, waves, (double2 *)L.partial);
        else
            hipLaunchKernelGGL(blocks_f64_kernel<float2>, dim3((unsigned)blocks), dim3(64 * wpb), 0, s,
                               (const float2 *)L.Su, (const float2 *)L.Sd, L.groups, n_units, L.V, L.chunk_sites,
                               L.n_chunks, L.K, waves, (double2 *)L.partial);
    }
    pr.stop();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n_out = n_ct * L.K * 792;
    Probe pr2("blocks_reduce", s);
    hipLaunchKernelGGL(blocks_reduce_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, s,
                       (const double2 *)L.partial, L.n_chunks, L.K, n_out, (double2 *)L.B);
    pr2.stop();
    return hipGetLastError();
}

size_t contract_tg_lds_bytes(int K, int tg) { return (size_t)(kMaxPalette + (size_t)tg * K * 792) * sizeof(double2); }

namespace {
// Dynamic LDS above the 64 KiB default needs an explicit opt-in per kernel;
// the largest term-sum request (palette + 12 blocks) plus the kernels'
// static LDS stays within the 160 KiB of a CU.
constexpr size_t kMaxContractLds = (kMaxPalette + kMaxLdsKinds * 792) * sizeof(double2);
template <typename F> hipError_t allow_lds(F *kernel)
{
    return hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kMaxContractLds);
}

template <int A, int FORM> hipError_t launch_tg(const ContractLaunch &L, hipStream_t s, unsigned blocks)
{
    static const hipError_t attr = allow_lds(contract_tg_kernel<A, FORM>);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL((contract_tg_kernel<A, FORM>), dim3(blocks), dim3(kCThreads),
                       contract_tg_lds_bytes(L.K, L.tg), s, (const double2 *)L.B, L.tab, L.N, L.K, L.n_ct, L.tg,
                       L.n_slices, L.slice_len, (double2 *)L.partial, L.share);
    return hipSuccess;
}

template <int A> void launch_global(const ContractLaunch &L, hipStream_t s, unsigned blocks)
{
    if (L.tab.coef_real)
        hipLaunchKernelGGL((contract_kernel<A, true>), dim3(blocks), dim3(256), 0, s, (const double2 *)L.B,
                           L.tab.kidx, L.tab.coef, L.N, L.K, L.n_ct, L.n_slices, L.slice_len, (double2 *)L.partial);
    else
        hipLaunchKernelGGL((contract_kernel<A, false>), dim3(blocks), dim3(256), 0, s, (const double2 *)L.B,
                           L.tab.kidx, L.tab.coef, L.N, L.K, L.n_ct, L.n_slices, L.slice_len, (double2 *)L.partial);
}
}  // namespace

hipError_t launch_contract(const ContractLaunch &L, hipStream_t s)
{
    Probe pr("contract", s);
    if (L.tg > 0) {
        if (L.tg > kMaxTG || L.tg * L.K > kMaxLdsKinds) return hipErrorInvalidValue;
        const int64_t n_groups = (L.n_ct + L.tg - 1) / L.tg;
        const unsigned blocks = (unsigned)round8(n_groups * L.n_slices);
        const int form = L.tab.seg_prefix ? (L.tab.coef_unit ? 5 : (L.tab.coef_real ? 4 : 2))
                                           : (L.tab.words ? (L.tab.coef_real ? 3 : 1) : 0);
        hipError_t e = hipErrorInvalidValue;
        switch (L.A * 8 + form) {
        case 8: e = launch_tg<1, 0>(L, s, blocks); break;
        case 9: e = launch_tg<1, 1>(L, s, blocks); break;
        case 11: e = launch_tg<1, 3>(L, s, blocks); break;
        case 16: e = launch_tg<2, 0>(L, s, blocks); break;
        case 17: e = launch_tg<2, 1>(L, s, blocks); break;
        case 18: e = launch_tg<2, 2>(L, s, blocks); break;
        case 19: e = launch_tg<2, 3>(L, s, blocks); break;
        case 20: e = launch_tg<2, 4>(L, s, blocks); break;
        case 21: e = launch_tg<2, 5>(L, s, blocks); break;
        case 24: e = launch_tg<3, 0>(L, s, blocks); break;
        case 25: e = launch_tg<3, 1>(L, s, blocks); break;
        case 26: e = launch_tg<3, 2>(L, s, blocks); break;
        case 27: e = launch_tg<3, 3>(L, s, blocks); break;
        case 28: e = launch_tg<3, 4>(L, s, blocks); break;
        case 29: e = launch_tg<3, 5>(L, s, blocks); break;
        case 32: e = launch_tg<4, 0>(L, s, blocks); break;
        case 33: e = launch_tg<4, 1>(L, s, blocks); break;
        case 34: e = launch_tg<4, 2>(L, s, blocks); break;
        case 35: e = launch_tg<4, 3>(L, s, blocks); break;
        case 36: e = launch_tg<4, 4>(L, s, blocks); break;
        case 37: e = launch_tg<4, 5>(L, s, blocks); break;
        case 40: e = launch_tg<5, 0>(L, s, blocks); break;
        default: break;
        }
        if (e != hipSuccess) return e;
    } else {
        if (L.tab.words) return hipErrorInvalidValue;  // the global-memory kernel reads the plain table
        const unsigned blocks = (unsigned)round8((int64_t)L.n_ct * L.n_slices);
        switch (L.A) {
        case 1: launch_global<1>(L, s, blocks); break;
        case 2: launch_global<2>(L, s, blocks); break;
        case 3: launch_global<3>(L, s, blocks); break;
        case 4: launch_global<4>(L, s, blocks); break;
        case 5: launch_global<5>(L, s, blocks); break;
        default: return hipErrorInvalidValue;
        }
    }
    pr.stop();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    Probe pr2("contract_finalize", s);
    hipLaunchKernelGGL(contract_finalize_kernel, dim3((L.n_ct + 255) / 256), dim3(256), 0, s,
                       (const double2 *)L.partial, L.n_ct, L.n_slices, (double2 *)L.C);
    pr2.stop();
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}


namespace {
// The four launches of a batch phase, one kernel at a time; kernel k in
// {0: blocks, 1: block reduction, 2: term sum, 3: finalize}.
hipError_t batch_kernel(const BatchLaunch &L, const BatchPhase &P, int k, hipStream_t s)
{
    if (k == 0 && P.nbw > 0) {
        const unsigned blocks = (unsigned)round8((int64_t)P.nbw * kNucColGroups);
        const BatchBlockWork *bw = L.bwork + P.bw0;
        bool done = false;
#define WICK_BNUC(NTV, MODE)                                                                                      \
    if (L.nt_max == NTV && L.prec == MODE) {                                                                      \
        if (L.dtype == 0)                                                                                         \
            hipLaunchKernelGGL((blocks_nucleon_kernel<double2, NTV, MODE>), dim3(blocks), dim3(kNucThreads), 0,    \
                               s, (const double2 *)L.Su, (const double2 *)L.Sd, nullptr, L.V, L.chunk_sites, 0, 0, \
                               P.nbw, (double2 *)L.partial, L.bitems, bw, L.T);                                   \
        else                                                                                                      \
            hipLaunchKernelGGL((blocks_nucleon_kernel<float2, NTV, MODE>), dim3(blocks), dim3(kNucThreads), 0,     \
                               s, (const float2 *)L.Su, (const float2 *)L.Sd, nullptr, L.V, L.chunk_sites, 0, 0,   \
                               P.nbw, (double2 *)L.partial, L.bitems, bw, L.T);                                   \
        done = true;                                                                                              \
    }
        WICK_BNUC(1, WICK_P64) WICK_BNUC(2, WICK_P64) WICK_BNUC(3, WICK_P64) WICK_BNUC(4, WICK_P64)
        WICK_BNUC(1, WICK_P32) WICK_BNUC(2, WICK_P32) WICK_BNUC(3, WICK_P32)
        WICK_BNUC(1, WICK_PB3) WICK_BNUC(2, WICK_PB3) WICK_BNUC(3, WICK_PB3)
        WICK_BNUC(1, WICK_PB6) WICK_BNUC(2, WICK_PB6) WICK_BNUC(3, WICK_PB6)
#undef WICK_BNUC
        if (!done) return hipErrorInvalidValue;
    } else if (k == 1 && P.nbout > 0) {
        hipLaunchKernelGGL(batch_reduce_kernel, dim3((unsigned)((P.nbout + 255) / 256)), dim3(256), 0, s,
                           (const double2 *)L.partial, L.bitems, L.bout_off, L.n_items, L.T, P.bout0, P.nbout,
                           (double2 *)L.B);
    } else if (k == 2 && P.ncw > 0) {
        if (L.contract_lds > kMaxContractLds) return hipErrorInvalidValue;
        static const hipError_t attr = allow_lds(contract_batch_kernel);
        if (attr != hipSuccess) return attr;
        hipLaunchKernelGGL(contract_batch_kernel, dim3((unsigned)round8(P.ncw)), dim3(kCThreads), L.contract_lds, s,
                           (const double2 *)L.B, L.citems, L.cwork + P.cw0, P.ncw, (double2 *)L.cpartial);
    } else if (k == 3 && P.ni > 0) {
        hipLaunchKernelGGL(batch_finalize_kernel, dim3((P.ni * L.T + 255) / 256), dim3(256), 0, s,
                           (const double2 *)L.cpartial, L.citems, P.i0, P.ni, L.T, (double2 *)L.C);
    }
    return hipGetLastError();
}
const char *const kBatchKernelName[4] = {"blocks", "blocks_reduce", "contract", "contract_finalize"};
}  // namespace

hipError_t launch_batch(const BatchLaunch &L, hipStream_t s)
{
    // kernel by kernel over both phases (the per-kernel timings then cover the whole batch)
    for (int k = 0; k < 4; ++k) {
        Probe pr(kBatchKernelName[k], s);
        for (int ph = 0; ph < 2; ++ph) {
            const hipError_t e = batch_kernel(L, L.ph[ph], k, s);
            if (e != hipSuccess) return e;
        }
        pr.stop();
    }
    return hipSuccess;
}

hipError_t launch_batch_forked(const BatchLaunch &L, hipStream_t s0, hipStream_t s1, hipEvent_t fork,
                               hipEvent_t join)
{
    hipError_t e;
    for (int k = 0; k < 2; ++k)
        if ((e = batch_kernel(L, L.ph[0], k, s0)) != hipSuccess) return e;
    if ((e = hipEventRecord(fork, s0)) != hipSuccess || (e = hipStreamWaitEvent(s1, fork, 0)) != hipSuccess) return e;
    for (int k = 2; k < 4; ++k)
        if ((e = batch_kernel(L, L.ph[0], k, s0)) != hipSuccess) return e;
    for (int k = 0; k < 4; ++k)
        if ((e = batch_kernel(L, L.ph[1], k, s1)) != hipSuccess) return e;
    if ((e = hipEventRecord(join, s1)) != hipSuccess || (e = hipStreamWaitEvent(s0, join, 0)) != hipSuccess) return e;
    return hipSuccess;
}

}  // namespace wick
