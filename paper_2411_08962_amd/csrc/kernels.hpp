// Device-side descriptors and host launchers of the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace wick {

// One E group as the block kernel reads it (uniform per wave).
struct EGroupDev {
    int32_t f, g, R, nk, mt;
    int32_t kind_out[kMaxKindsPerGroup];
    int32_t nterm[kMaxRows];
    int8_t j2[kMaxRows][kMaxRowTerms];
    int8_t j3[kMaxRows][kMaxRowTerms];
    int8_t w[kMaxRows][kMaxRowTerms];
    int8_t aj1[kMaxKindsPerGroup][kMaxRows][kMaxAop];
    int8_t aa[kMaxKindsPerGroup][kMaxRows][kMaxAop];
};

constexpr int kNTiles = 9;  // 144 (i2, i3) columns = 9 MFMA tiles of 16

// All groups of a plan for the staged block kernel. Its workgroup has one
// wave per column tile; every wave accumulates every m-tile ("tile") of the
// groups of one pass. Groups are packed into passes of at most kPassTiles
// tiles (the accumulators of a pass stay in registers).
constexpr int kMaxGroupsStaged = 8;
constexpr int kMaxPasses = 8;
constexpr int kPassTiles = 4;
struct BlocksDesc {
    int32_t n_groups, n_passes;
    int32_t pass_tiles[kMaxPasses];
    int32_t pass_ngroups[kMaxPasses], pass_groups[kMaxPasses][kPassTiles];
    int32_t tile_group[kMaxPasses][kPassTiles], tile_mt[kMaxPasses][kPassTiles];  // group -1: unused
    EGroupDev groups[kMaxGroupsStaged];
};

// Nucleon-form groups (see NucGroup): E_r(x)[i2,i3] = sum over the nonzero
// M[s3][s2] of M * (colour cross product of S_g(x)[3 s2 + ., i2] and
// S_f(x)[3 s3 + ., i3])_r, and Aop_k(x, r)[i1] = S_f(x)[3 alpha_k + r, i1].
//
// A group may also carry the kinds of its twin: the group with flavors (g, f)
// and diquark entries (s3, s2, -M) for every (s2, s3, M) of this one, whose
// rows are E_r(x)[i3, i2] of this group's E_r(x)[i2, i3] (swap the two
// propagators in the colour cross product and relabel the spins). A twin
// kind reads its Aop row from S_g (flv = 1) and stores its columns
// transposed (tr = 1), so one E serves both groups.
struct NucGroupDev {
    int32_t f, g, npair, nk;
    int32_t npos, nneg;             // pairs with M = +1 first, then M = -1, then the rest
    int32_t s2[16], s3[16], m[16];  // 32-bit: read with scalar loads
    int32_t alpha[kMaxKindsPerGroup], kind_out[kMaxKindsPerGroup];
    int32_t flv[kMaxKindsPerGroup], tr[kMaxKindsPerGroup];
};
struct NucDesc {
    int32_t n_groups, n_passes;
    int32_t pass_ngroups[kMaxPasses], pass_groups[kMaxPasses][kPassTiles];
    int32_t pass_tiles[kMaxPasses];
    int32_t tile_group[kMaxPasses][kPassTiles], tile_mt[kMaxPasses][kPassTiles];  // group -1: unused
    NucGroupDev groups[kMaxGroupsStaged];
};

// Batched launches: one work entry per workgroup and one descriptor per
// (nucleus, configuration) item, so one launch covers items of different
// nuclei (different A, kinds and tables).
struct BatchBlockItem {
    const NucDesc *desc;   // the item's plan (split or FP64 packing)
    int64_t s_off;         // offset of the item's configuration in S_u / S_d (entries)
    int64_t part_off;      // offset of the item's partial blocks (double2 entries)
    int64_t b_off;         // offset of the item's blocks in B (double2 entries)
    int32_t K, n_chunks;
};
struct BatchBlockWork {
    int32_t item, t, chunk, pass;
};
// Term table on the device. Packed form (A <= 4, K <= 20, at most 256
// distinct coefficients): one 64-bit word per term holding the A block
// indices kind*792 + c in 14-bit fields (field a at bit 14a) and, in the top
// 8 bits, the index of the term's coefficient in a palette. Plain form:
// kidx[A][N] uint16 and coef[N] (real) or coef[N][2].
constexpr int kPackBits = 14;
constexpr int kMaxPalette = 256;
//
// Segmented form (2 <= A <= 4, K <= 12, at most 255 distinct coefficients),
// which shares the leading indices of the terms. The table sorted by index
// tuple is cut into nodes (terms sharing their first A-1 indices, at most
// kNodeLeaves = 2 of them, padded with a zero-coefficient term) and segments
// (at most seg_len / kNodeLeaves consecutive nodes sharing the first A-2
// indices, the segment prefix). A lane evaluates one segment as
//   P * sum_nodes B[node] * sum_leaves coef * B[leaf],   P = prod of the prefix entries,
// so every term costs one LDS gather and every node one more, instead of A
// per term; as every node is one word the lanes of a wave never diverge.
// Segments are sorted by length and dealt to the 64 lanes of a chunk; chunk
// c holds L = chunk_len[c] & 0xffff nodes per lane, interleaved (node j of
// lane l at chunk_base[c] + 64 j + l), shorter segments padded with zero
// words. Node word bits: leaf 0 [0,14), node index [14,28), palette index of
// leaf 0 [28,36), leaf 1 [36,50), palette index of leaf 1 [50,58); palette
// entry 0 is zero.
//
// Integer-coefficient words (coef_unit != 0: every coefficient is q *
// coef_unit for an integer q, |q| <= 1023, to within 2^-50 of it; true of
// every built-in nucleus, with coef_unit an integer, and of operators whose
// coefficients are multiples of one rational scale): leaf 0 [0,14), node
// index [14,28), leaf 1 [28,42), q of leaf 0 [42,53) and q of leaf 1
// [53,64), both two's complement. The lane sums with the integers q (exact
// in FP64) and multiplies by coef_unit once per segment, so no palette is
// read from LDS. q = 0 marks a missing leaf (index 0, weight zero) and a
// zero word is padding. Segments of equal length are sorted by their number
// of two-leaf nodes, and each lane holds its two-leaf nodes first, so a
// chunk's steps j >= chunk_len[c] >> 16 have no leaf 1 in any lane and the
// term sum skips that gather there.
//
// Factored form (A = 4 with integer words; chunk_g set). With the two index
// positions of fewest distinct pairs taken as the prefix (i, j) and the two
// others as node and leaf, the terms of each prefix form a list which,
// divided by g (gcd of its q, sign of the first), many prefixes share:
//   C = unit * sum_m G_m M_m,  G_m = sum over the prefixes of list m of g B[i] B[j].
// A lane's segment is a piece of one list (two-leaf words first): its first
// chunk_g[c] steps hold G_m as one-leaf words (node i, leaf j, q = g; zero
// words pad a shorter group), the later ones the piece's list words; the
// lane adds unit * G * (its piece's sum). seg_prefix is unused.
constexpr int kNodeLeaves = 2;
constexpr int kIntCoefMax = 1023;
struct TermTable {
    const uint64_t *words;  // packed [N] or segmented (interleaved chunks), or null
    const double2 *pal;     // packed / segmented: palette [n_pal]
    int32_t n_pal;
    int32_t coef_real;      // plain: coef is [N] (1) or [N][2] (0)
    const uint16_t *kidx;   // plain [A][N]
    const double *coef;
    // segmented form (seg_prefix != null)
    const uint32_t *seg_prefix;  // [n_chunks * 64]: A-2 indices of 14 bits
    const int64_t *chunk_base;   // [n_chunks]
    const int32_t *chunk_len;    // [n_chunks]: nodes per lane, plus (steps with a leaf 1) << 16
    const int32_t *chunk_g;      // [n_chunks]: factored form (A = 4), steps of prefix-group words
    int32_t n_chunks;
    double coef_unit;            // segmented form: 0 palette words, else integer-coefficient words
};

// The term sum stages the blocks of up to kMaxTG consecutive time slices of
// one (configuration or item) in LDS and reads each table word once for all
// of them: tg * K <= kMaxLdsKinds keeps a workgroup within 160 KiB of LDS.
constexpr int kCThreads = 1024;
constexpr int kMaxTG = 3;
constexpr int kMaxLdsKinds = 12;
constexpr int kPrefetch = 8;  // table words in flight per lane in the term sum
size_t contract_tg_lds_bytes(int K, int tg);  // palette + tg slices of K blocks

struct BatchContractItem {
    TermTable tab;
    int64_t N, slice_len, b_off, part_off;  // part_off: first partial of (item, t = 0); slice_len in chunks when segmented
    int32_t A, K, n_slices, tg;
    int32_t out_item;                       // the item's row of C (the caller's item index)
};
struct BatchContractWork {
    int32_t item, t0, slice, ntg;
};

struct BlockLaunch {
    const void *Su, *Sd;
    int dtype;               // 0 = complex128, 1 = complex64
    int prec;                // wick_precision
    const EGroupDev *groups; // device
    int n_groups;
    const BlocksDesc *desc;  // device; null when the plan exceeds the staged kernel's limits
    int n_tiles;             // most tiles in one pass (staged kernel)
    int n_passes;
    const NucDesc *nuc;      // device; set when every kind has nucleon form
    int nuc_tiles, nuc_passes;
    int64_t V;
    int T, n_cfg, K;
    int chunk_sites, n_chunks;
    double *partial;         // [n_cfg*T][n_chunks][K][12][144][2]
    double *B;               // [n_cfg*T][K][792][2]
};

hipError_t launch_blocks(const BlockLaunch &L, hipStream_t s);

// A batch runs in two phases of about equal work (items dealt alternately);
// each phase's work is a contiguous range of every work list, so phase 1's
// blocks can run while phase 0's term sum does (launch_batch_forked).
struct BatchPhase {
    int bw0, nbw;          // block work entries
    int i0, ni;            // items (internal order)
    int64_t bout0, nbout;  // block outputs
    int cw0, ncw;          // term-sum work entries
};
struct BatchLaunch {
    BatchPhase ph[2];
    const void *Su, *Sd;
    int dtype, prec, nt_max;
    int64_t V;
    int T, chunk_sites;
    int n_items;
    const BatchBlockItem *bitems;     // device
    const BatchBlockWork *bwork;      // device
    int n_bwork;
    const int64_t *bout_off;          // device [n_items + 1]: prefix of T*K*792
    int64_t n_bout;
    const BatchContractItem *citems;  // device
    const BatchContractWork *cwork;   // device
    int n_cwork;
    size_t contract_lds;              // dynamic LDS of the batched term sum
    double *partial;                  // workspace: raw partial blocks of every item
    double *B;                        // blocks of every item
    double *cpartial;                 // contraction partials
    double *C;                        // [n_items][T][2]
};
hipError_t launch_batch(const BatchLaunch &L, hipStream_t s);  // both phases in order on one stream
// Phase 0 on s0; phase 1 forked onto s1 after phase 0's blocks, so its blocks
// overlap phase 0's term sum; s0 then waits for s1 (graph capture makes the
// fork and join graph edges). fork/join: events owned by the caller.
hipError_t launch_batch_forked(const BatchLaunch &L, hipStream_t s0, hipStream_t s1, hipEvent_t fork,
                               hipEvent_t join);

struct ContractLaunch {
    const double *B;         // [n_ct][K][792][2]
    TermTable tab;
    int A, K;
    int64_t N;
    int n_ct;
    int tg;                  // time slices per workgroup (LDS kernel); 0: blocks read from global memory
    int n_slices;
    int64_t slice_len;       // terms per workgroup (chunks per workgroup for a segmented table)
    int share;               // groups of slices taking one table slice together (1: group-major)
    double *partial;         // [n_ct][n_slices][2]
    double *C;               // [n_ct][2]
};

hipError_t launch_contract(const ContractLaunch &L, hipStream_t s);
hipError_t launch_zero(double *p, int64_t n, hipStream_t s);  // p[0..n) = 0 (a kernel, so graph capture is safe)

// Optional per-kernel event timing (api.hip). A Probe records a start event
// on construction and a stop event on stop() when profiling is enabled.
struct Probe {
    Probe(const char *name, hipStream_t s);
    void stop();
    const char *name;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
};

}  // namespace wick
