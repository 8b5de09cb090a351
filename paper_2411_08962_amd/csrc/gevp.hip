// Term sum of a GEVP correlation matrix (Eqs. E1-E3): every monomial of the
// union table is formed once per time slice and added to every element with
// that element's coefficient.
//
// gevp_contract_kernel: one workgroup per (configuration and time slice, term
// chunk). The slice's blocks are staged in LDS when they fit (up to 11 kinds),
// else read from global memory. Each thread forms prod_a B[kidx_{a,n}] for its
// terms and accumulates coef[n][e] times it for every element e in registers;
// the workgroup sums every element (wave shuffles, then the waves in order)
// into one partial per (slice, chunk, element). gevp_finalize_kernel adds
// the chunks in order (deterministic).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace wick {

wick_status workspace(hipStream_t s, size_t bytes, void **out);

namespace {

constexpr int kGvThreads = 512;
constexpr int kGvChunk = 8192;                  // terms per workgroup
constexpr int kGvMaxLdsKinds = 11;              // 11 * 792 * 16 B = 139 KB of LDS

struct GvDev {
    int device = -1;
    uint16_t *kidx = nullptr;
    double *coef = nullptr;   // [N][E] real or [N][E][2]
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

template <int A, int E, bool REAL, bool LDS>
__global__ __launch_bounds__(kGvThreads) void gevp_contract_kernel(const double2 *__restrict__ B, int K,
                                                                  const uint16_t *__restrict__ kidx,
                                                                  const double *__restrict__ coef, int64_t N,
                                                                  int n_chunks, double2 *__restrict__ partial)
{
    extern __shared__ double2 sB[];
    __shared__ double2 red[kGvThreads / 64][E];
    const int64_t slice = blockIdx.x / n_chunks;
    const int chunk = blockIdx.x % n_chunks;
    const double2 *Bs = B + slice * (int64_t)K * 792;
    if (LDS) {
        for (int e = threadIdx.x; e < K * 792; e += kGvThreads) sB[e] = Bs[e];
        __syncthreads();
    }
    const double2 *Bv = LDS ? sB : Bs;
    double2 acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = make_double2(0.0, 0.0);
    const int64_t n0 = (int64_t)chunk * kGvChunk, n1 = min(N, n0 + kGvChunk);
    for (int64_t n = n0 + threadIdx.x; n < n1; n += kGvThreads) {
        double2 p = Bv[kidx[n]];
#pragma unroll
        for (int a = 1; a < A; ++a) p = cmul(p, Bv[kidx[(int64_t)a * N + n]]);
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (REAL) {
                const double c = coef[n * E + e];
                acc[e].x += c * p.x;
                acc[e].y += c * p.y;
            } else {
                const double2 c = make_double2(coef[2 * (n * E + e)], coef[2 * (n * E + e) + 1]);
                const double2 t = cmul(c, p);
                acc[e].x += t.x;
                acc[e].y += t.y;
            }
        }
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
        double2 v = acc[e];
        for (int o = 32; o > 0; o >>= 1) {
            v.x += __shfl_down(v.x, o, 64);
            v.y += __shfl_down(v.y, o, 64);
        }
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][e] = v;
    }
    __syncthreads();
    if (threadIdx.x < E) {
        double2 v = red[0][threadIdx.x];
        for (int w = 1; w < kGvThreads / 64; ++w) { v.x += red[w][threadIdx.x].x; v.y += red[w][threadIdx.x].y; }
        partial[((int64_t)slice * n_chunks + chunk) * E + threadIdx.x] = v;
    }
}

__global__ void gevp_finalize_kernel(const double2 *__restrict__ partial, int n_chunks, int E, int64_t n_out,
                                     double2 *__restrict__ C)
{
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // slice * E + e
    if (o >= n_out) return;
    const int64_t slice = o / E;
    const int e = (int)(o % E);
    double2 s = make_double2(0.0, 0.0);
    for (int c = 0; c < n_chunks; ++c) {
        const double2 v = partial[(slice * n_chunks + c) * E + e];
        s.x += v.x;
        s.y += v.y;
    }
    C[o] = s;
}

wick_status gv_hip_fail(hipError_t e, const char *what)
{
    return fail(WICK_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

void free_gv(GvDev *d)
{
    (void)hipFree(d->kidx);
    (void)hipFree(d->coef);
    delete d;
}

wick_status gv_tables(wick_gevp_s *g, GvDev **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return gv_hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g->dev_mu);
    for (void *v : g->dev)
        if (((GvDev *)v)->device == dev) { *out = (GvDev *)v; return WICK_OK; }
    auto d = new GvDev();
    d->device = dev;
    const int E = g->n_ops * g->n_ops;
    std::vector<double> c;
    if (g->coef_real) {
        c.resize((size_t)g->n_terms * E);
        for (size_t i = 0; i < c.size(); ++i) c[i] = g->coef[2 * i];
    }
    const std::vector<double> &cv = g->coef_real ? c : g->coef;
    const size_t kb = std::max<size_t>(1, g->kidx.size()) * sizeof(uint16_t);
    const size_t cb = std::max<size_t>(1, cv.size()) * sizeof(double);
    if ((e = hipMalloc((void **)&d->kidx, kb)) != hipSuccess || (e = hipMalloc((void **)&d->coef, cb)) != hipSuccess) {
        free_gv(d);
        return fail(WICK_ENOMEM, std::string("wick_gevp_contract: hipMalloc: ") + hipGetErrorString(e));
    }
    if ((!g->kidx.empty() &&
         (e = hipMemcpy(d->kidx, g->kidx.data(), g->kidx.size() * sizeof(uint16_t), hipMemcpyHostToDevice)) != hipSuccess) ||
        (!cv.empty() && (e = hipMemcpy(d->coef, cv.data(), cv.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)) {
        free_gv(d);
        return gv_hip_fail(e, "wick_gevp_contract: hipMemcpy");
    }
    g->dev.push_back(d);
    *out = d;
    return WICK_OK;
}

template <int A, int E, bool REAL>
void launch_gv(bool lds, dim3 grid, size_t shmem, hipStream_t s, const double2 *B, int K, const uint16_t *kidx,
               const double *coef, int64_t N, int n_chunks, double2 *partial)
{
    if (lds)
        gevp_contract_kernel<A, E, REAL, true><<<grid, kGvThreads, shmem, s>>>(B, K, kidx, coef, N, n_chunks, partial);
    else
        gevp_contract_kernel<A, E, REAL, false><<<grid, kGvThreads, 0, s>>>(B, K, kidx, coef, N, n_chunks, partial);
}

template <int A, int E>
void launch_gv_e(bool real, bool lds, dim3 grid, size_t shmem, hipStream_t s, const double2 *B, int K,
                 const uint16_t *kidx, const double *coef, int64_t N, int n_chunks, double2 *partial)
{
    if (real) launch_gv<A, E, true>(lds, grid, shmem, s, B, K, kidx, coef, N, n_chunks, partial);
    else launch_gv<A, E, false>(lds, grid, shmem, s, B, K, kidx, coef, N, n_chunks, partial);
}

template <int A>
void launch_gv_a(int E, bool real, bool lds, dim3 grid, size_t shmem, hipStream_t s, const double2 *B, int K,
                 const uint16_t *kidx, const double *coef, int64_t N, int n_chunks, double2 *partial)
{
    switch (E) {
    case 1: launch_gv_e<A, 1>(real, lds, grid, shmem, s, B, K, kidx, coef, N, n_chunks, partial); break;
    case 4: launch_gv_e<A, 4>(real, lds, grid, shmem, s, B, K, kidx, coef, N, n_chunks, partial); break;
    case 9: launch_gv_e<A, 9>(real, lds, grid, shmem, s, B, K, kidx, coef, N, n_chunks, partial); break;
    default: launch_gv_e<A, 16>(real, lds, grid, shmem, s, B, K, kidx, coef, N, n_chunks, partial); break;
    }
}

}  // namespace

void release_gevp_tables(wick_gevp_s *g)
{
    std::lock_guard<std::mutex> lk(g->dev_mu);
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (void *v : g->dev) {
        GvDev *d = (GvDev *)v;
        (void)hipSetDevice(d->device);
        free_gv(d);
    }
    g->dev.clear();
    (void)hipSetDevice(cur);
}

}  // namespace wick

using namespace wick;

extern "C" wick_status wick_gevp_contract(wick_gevp_t g, const double *B, int32_t n_cfg, int32_t T,
                                          wick_stream_t stream, double *C)
{
    try {
        if (!g || !B || !C) return fail(WICK_EINVAL, "wick_gevp_contract: null pointer");
        if (((uintptr_t)B | (uintptr_t)C) & 15) return fail(WICK_EINVAL, "wick_gevp_contract: B and C must be 16-byte aligned");
        if (n_cfg < 1 || T < 1 || (int64_t)n_cfg * T > (1LL << 24)) return fail(WICK_EINVAL, "wick_gevp_contract: bad n_cfg or T");
        hipStream_t s = (hipStream_t)stream;
        const int E = g->n_ops * g->n_ops;
        const int64_t slices = (int64_t)n_cfg * T;
        if (g->n_terms == 0) {
            hipError_t e = launch_zero(C, slices * E * 2, s);
            return e == hipSuccess ? WICK_OK : gv_hip_fail(e, "zero_kernel");
        }
        GvDev *d = nullptr;
        wick_status st = gv_tables(g, &d);
        if (st != WICK_OK) return st;
        const int K = (int)g->carrier->kinds.size();
        const int n_chunks = (int)((g->n_terms + kGvChunk - 1) / kGvChunk);
        if (slices * n_chunks > (1LL << 31) - 1) return fail(WICK_ETOOBIG, "wick_gevp_contract: too many workgroups");
        void *ws = nullptr;
        st = workspace(s, (size_t)slices * n_chunks * E * sizeof(double2), &ws);
        if (st != WICK_OK) return st;
        const bool lds = K <= kGvMaxLdsKinds;
        const size_t shmem = lds ? (size_t)K * 792 * sizeof(double2) : 0;
        if (lds && shmem > 64 * 1024) {
            hipError_t e = hipSuccess;
#define GV_ATTR(a, ee, r)                                                                                        \
    e = hipFuncSetAttribute((const void *)gevp_contract_kernel<a, ee, r, true>,                                  \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);                              \
    if (e != hipSuccess) return gv_hip_fail(e, "hipFuncSetAttribute");
#define GV_ATTR_E(a) GV_ATTR(a, 1, true) GV_ATTR(a, 1, false) GV_ATTR(a, 4, true) GV_ATTR(a, 4, false)          \
    GV_ATTR(a, 9, true) GV_ATTR(a, 9, false) GV_ATTR(a, 16, true) GV_ATTR(a, 16, false)
            switch (g->A) {
            case 1: GV_ATTR_E(1) break;
            case 2: GV_ATTR_E(2) break;
            case 3: GV_ATTR_E(3) break;
            case 4: GV_ATTR_E(4) break;
            default: GV_ATTR_E(5) break;
            }
#undef GV_ATTR_E
#undef GV_ATTR
        }
        const dim3 grid((unsigned)(slices * n_chunks));
        double2 *partial = (double2 *)ws;
        Probe pr("gevp_contract", s);
        switch (g->A) {
        case 1: launch_gv_a<1>(E, g->coef_real, lds, grid, shmem, s, (const double2 *)B, K, d->kidx, d->coef, g->n_terms, n_chunks, partial); break;
        case 2: launch_gv_a<2>(E, g->coef_real, lds, grid, shmem, s, (const double2 *)B, K, d->kidx, d->coef, g->n_terms, n_chunks, partial); break;
        case 3: launch_gv_a<3>(E, g->coef_real, lds, grid, shmem, s, (const double2 *)B, K, d->kidx, d->coef, g->n_terms, n_chunks, partial); break;
        case 4: launch_gv_a<4>(E, g->coef_real, lds, grid, shmem, s, (const double2 *)B, K, d->kidx, d->coef, g->n_terms, n_chunks, partial); break;
        default: launch_gv_a<5>(E, g->coef_real, lds, grid, shmem, s, (const double2 *)B, K, d->kidx, d->coef, g->n_terms, n_chunks, partial); break;
        }
        pr.stop();
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return gv_hip_fail(e, "gevp_contract_kernel");
        const int64_t n_out = slices * E;
        gevp_finalize_kernel<<<dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, s>>>(partial, n_chunks, E, n_out,
                                                                                          (double2 *)C);
        e = hipGetLastError();
        return e == hipSuccess ? WICK_OK : gv_hip_fail(e, "gevp_finalize_kernel");
    } catch (const std::bad_alloc &) {
        return fail(WICK_ENOMEM, "wick_gevp_contract: out of host memory");
    } catch (...) {
        return fail(WICK_EINVAL, "wick_gevp_contract: internal error");
    }
}
