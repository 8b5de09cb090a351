// Internal data structures shared by the planner, the C ABI and the kernels'
// host-side launchers. Not part of the public interface.
#pragma once

#include <array>
#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/wick.h"

namespace wick {

constexpr int kMaxA = 5;          // nucleons per operator
constexpr int kBlockLen = 792;    // compact antisymmetrised block: 66 pairs x 12
constexpr int kMaxTrials = 4;     // identity tests per term
constexpr int kMaxKindsPerGroup = 5;  // 12*5 = 60 <= 64 MFMA rows (4 tiles of 16)
constexpr int kMaxRows = 8;       // E rows per group
constexpr int kMaxRowTerms = 16;  // (j2, j3) terms per E row
constexpr int kMaxAop = 2;        // (j1, a) terms per (kind, row)

struct GInt {
    int64_t re = 0, im = 0;
};

struct KindDef {
    int flav[3] = {0, 0, 0};
    std::vector<std::array<int8_t, 3>> j;
    std::vector<GInt> w;
};

// One E row: E_r(x)[i2, i3] = sum_t w_t S_g(x)[j2_t, i2] S_f(x)[j3_t, i3].
struct ERow {
    std::vector<std::array<int8_t, 2>> jj;  // (j2, j3)
    std::vector<int8_t> w;                  // small integer weights
};

// Kinds of one flavor pattern (f, g, f) whose weights factor through common
// E rows: w_k(j1, j2, j3) = sum_r a_k(j1, r) E_r(j2, j3).
struct EGroup {
    int f = 0, g = 1;
    std::vector<ERow> rows;
    std::vector<int> kinds;  // block-kind indices
    // aop[(kk * R + r) * kMaxAop + e] = {j1, a}; a == 0 marks an unused entry
    std::vector<std::array<int8_t, 2>> aop;
};

// Kinds of nucleon form (Eqs. 2.2-2.3 and the projected forms of Sec. 3.3):
//   w_k(j1, j2, j3) = delta(spin j1 = alpha_k) eps[c(j1), c(j3), c(j2)] M[s(j3)][s(j2)]
// with one integer diquark matrix M shared by the group's kinds.
struct NucGroup {
    int f = 0, g = 1;
    std::vector<std::array<int8_t, 3>> pairs;  // (s2, s3, M[s3][s2]) for the nonzero entries of M
    std::vector<int> kinds, alpha;             // block-kind indices and their sink spins
};

// Kind weights on one device, for the per-site point-sink route (point.hip).
struct DeviceTable {
    int device = -1;
    void *kinds = nullptr;  // per-kind flavors and weight offsets, then the weights
};

struct wick_plan_impl;

}  // namespace wick

struct wick_plan_s {
    int A = 0;
    std::vector<wick::KindDef> kinds;   // block kinds (used by sink patterns)
    std::vector<wick::EGroup> egroups;
    std::vector<wick::NucGroup> nucgroups;  // empty unless every block kind has nucleon form
    int64_t n_terms = 0;
    std::vector<uint16_t> kidx;         // [A][n_terms]
    std::vector<double> coef_re, coef_im;
    bool coef_real = true;
    int64_t n_enumerated = 0, n_groups = 0;
    double bound = 0.0, scale = 1.0;
    // device copies of the kind weights for the per-site point-sink route, one per device
    std::mutex dev_mu;
    std::vector<wick::DeviceTable> dev;
    ~wick_plan_s();
};

// A point-sink plan (Eq. 2.9 and App. A): sink and source coefficient tensors
// antisymmetrised per flavor into groups (U, D) of sorted index lists, the
// distinct sink row sets, and the source column sets as ranks among the
// k-subsets of the 12 spin-colour indices.
struct wick_point_s {
    int n_u = 0, n_d = 0;               // quarks of each flavor
    double scale = 1.0;
    std::vector<std::array<int8_t, 8>> rows_u, rows_d;  // distinct sink row sets
    // sink groups, sorted by (u row set, d row set)
    std::vector<int32_t> g_u, g_d;      // indices into rows_u, rows_d
    std::vector<double> g_w;            // [2 G] exact integer weights (re, im)
    std::vector<int32_t> u_beg;         // [n rows_u + 1] sink groups of each u row set
    // source groups
    std::vector<uint16_t> h_ru, h_rd;   // colex ranks of the column sets U', D'
    std::vector<double> h_w;            // [2 H]
    int64_t n_cols_u = 0, n_cols_d = 0; // distinct source column sets
    std::mutex dev_mu;
    std::vector<void *> dev;            // device tables, one per device (point.hip)
    ~wick_point_s();
};

// A correlation matrix for the GEVP (Eqs. E1-E3): the union of the element
// tables, one coefficient per element and term.
struct wick_gevp_s {
    int n_ops = 0, A = 0;
    int64_t n_terms = 0, n_element_terms = 0;
    std::vector<uint16_t> kidx;   // [A][n_terms], kind * 792 + compact index, tuple sorted
    std::vector<double> coef;     // [n_terms][n_ops * n_ops][2], normalisation included
    bool coef_real = true;
    wick_plan_t carrier = nullptr;  // block kinds, no terms (drives the block kernels)
    std::mutex dev_mu;
    std::vector<void *> dev;      // device tables, one per device (gevp.hip)
    ~wick_gevp_s();
};

namespace wick {

void set_error(const std::string &msg);
wick_status fail(wick_status st, const std::string &msg);

// planner (plan.cpp)
wick_status build_plan(const wick_nucleus_desc *d, wick_plan_t *out);
void factor_kinds(wick_plan_s *p);  // fills p->egroups and p->nucgroups
wick_status save_plan(const wick_plan_s *p, const char *path);
wick_status load_plan(const char *path, wick_plan_t *out);

// important-term truncation (truncate.cpp)
int64_t truncation_count(int64_t n_terms, double keep);
wick_status truncate_plan(const wick_plan_s *p, const double *B_cal, int32_t n_slices, double keep,
                          wick_plan_t *out, double *dropped);

// built-in operators (nuclei.cpp)
wick_status std_plan(const char *name, int32_t J, wick_plan_t *out);
wick_status std_point_plan(const char *name, int32_t J, wick_point_t *out);
wick_status std_gevp_plan(const char *const *names, const int32_t *J, int32_t n_ops, wick_gevp_t *out);
wick_status std_pair_plan(const char *snk, int32_t J_snk, const char *src, int32_t J_src, wick_plan_t *out);

// GEVP union plan (gevp.cpp) and device tables (gevp.hip)
wick_status build_gevp(const wick_nucleus_desc *ops, int32_t n_ops, wick_gevp_t *out);
void release_gevp_tables(wick_gevp_s *g);

// point-sink planner (point.cpp) and device tables (point.hip)
wick_status build_point_plan(const wick_nucleus_desc *d, wick_point_t *out);
void release_point_tables(wick_point_s *p);
void release_plain_tables(wick_plan_s *p);

// device-table release (api.cpp)
void release_device_tables(wick_plan_s *p);

}  // namespace wick
