// dms_misc.hip -- status strings, the device check, table export, and the
// simplex values and backward scatter of the differentiable forms.
#include <atomic>
#include <cstring>

#include "dms_common.hpp"
#include "dms_internal.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

// Section 2.5: the birth and death of a pair are the highest vertex values
// of its two simplices, so their derivatives with respect to the field are
// indicator vectors at the max vertices (code >> 8).  The 2 npairs
// contributions (births c < npairs, deaths c = npairs + p) are keyed by
// their target vertex (targets outside [0, n) get the largest key and are
// dropped), ranked by a stable sort, and each run of equal target is summed
// by its first element in contribution order: every vertex gets the same
// sum, in the same order, on every run.
__global__ void k_backward_keys(const int64_t *__restrict__ bcode, const int64_t *__restrict__ dcode,
                                int64_t npairs, int64_t n, uint64_t *__restrict__ key)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= 2 * npairs) return;
    const int64_t v = (c < npairs ? bcode[c] : dcode[c - npairs]) >> 8;
    key[c] = v >= 0 && v < n ? (uint64_t)v : ~0ull;
}

__global__ void k_backward_place(const int32_t *__restrict__ rank, int64_t m, int32_t *__restrict__ at)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < m) at[rank[c]] = (int32_t)c;
}

__global__ void k_backward_sum(const int32_t *__restrict__ at, const uint64_t *__restrict__ key, int64_t m,
                               int64_t npairs, const double *__restrict__ gb, const double *__restrict__ gd,
                               double *__restrict__ grad)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const uint64_t v = key[at[j]];
    if (v == ~0ull || (j > 0 && key[at[j - 1]] == v)) return;
    double s = 0.0;
    for (int64_t q = j; q < m && key[at[q]] == v; ++q) {
        const int64_t c = at[q];
        s += c < npairs ? gb[c] : gd[c - npairs];
    }
    grad[v] = s;
}

template <typename T>
__global__ void k_simplex_values(const T *__restrict__ f, int64_t n, const int64_t *__restrict__ codes,
                                 int64_t count, double *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t v = codes[i] >> 8;
    out[i] = v >= 0 && v < n ? (double)f[v] : __longlong_as_double(0x7ff8000000000000ll);
}

__global__ void k_fill_zero(double *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

std::atomic<int> g_arch[64];  // per device: 0 unknown, 1 gfx950, 2 other

unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256); }

// Backward workspace: keys (8 B), ranks and positions (4 B each) per
// contribution, a flag word, then the ranking's own workspace.
struct BwdLayout {
    size_t key, rank, at, flags, rws, total;
};

BwdLayout bwd_layout(int64_t npairs)
{
    const int64_t m = 2 * npairs;
    BwdLayout L{};
    size_t off = 0;
    L.key = off; off += align_up((size_t)(m > 0 ? m : 1) * 8, 256);
    L.rank = off; off += align_up((size_t)(m > 0 ? m : 1) * 4, 256);
    L.at = off; off += align_up((size_t)(m > 0 ? m : 1) * 4, 256);
    L.flags = off; off += 256;
    L.rws = off; off += rank_u64_workspace_size(m > 0 ? m : 1);
    L.total = off;
    return L;
}

}  // namespace

int device_check()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
        (void)hipGetLastError();
        return DMS_E_UNSUPPORTED;
    }
    int st = g_arch[dev].load();
    if (st == 0) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) != hipSuccess) {
            (void)hipGetLastError();
            return DMS_E_UNSUPPORTED;
        }
        st = std::strncmp(p.gcnArchName, "gfx950", 6) == 0 ? 1 : 2;
        g_arch[dev].store(st);
    }
    return st == 1 ? DMS_OK : DMS_E_UNSUPPORTED;
}

}  // namespace dms

extern "C" const char *dms_status_str(int status)
{
    switch (status) {
    case DMS_OK: return "DMS_OK";
    case DMS_E_ARG: return "DMS_E_ARG: invalid argument";
    case DMS_E_SIZE: return "DMS_E_SIZE: grid too large for int32 orders";
    case DMS_E_WORKSPACE: return "DMS_E_WORKSPACE: workspace missing or too small";
    case DMS_E_UNSUPPORTED: return "DMS_E_UNSUPPORTED: the current device is not a gfx950";
    case DMS_E_HIP: return "DMS_E_HIP: HIP runtime error";
    case DMS_E_NOT_INITIALISED: return "DMS_E_NOT_INITIALISED: dms_init has not run on this device";
    default: return "unknown dms status";
    }
}

extern "C" const char *dms_version(void) { return "dms-mi355x 0.1 (gfx950)"; }

extern "C" int dms_star_tables(int32_t *nb, int32_t *tri, int32_t *tet, int32_t *edge_tris,
                               int32_t *tri_tets)
{
    const dms::Tables &T = dms::kTables;
    if (!nb || !tri || !tet || !edge_tris || !tri_tets) return DMS_E_ARG;
    for (int e = 0; e < 14; ++e) {
        for (int c = 0; c < 3; ++c) nb[3 * e + c] = T.nb[e][c];
        for (int s = 0; s < 6; ++s) edge_tris[6 * e + s] = T.edge_tris[e][s];
    }
    for (int t = 0; t < 36; ++t)
        for (int s = 0; s < 2; ++s) {
            tri[2 * t + s] = T.tri[t][s];
            tri_tets[2 * t + s] = T.tri_tets[t][s];
        }
    for (int q = 0; q < 24; ++q)
        for (int c = 0; c < 3; ++c) tet[3 * q + c] = T.tet[q][c];
    return DMS_OK;
}

extern "C" int dms_simplex_values(const void *values, int dtype, int64_t n, const int64_t *codes,
                                  int64_t count, double *out, void *stream)
{
    if ((dtype != DMS_F32 && dtype != DMS_F64) || n < 0 || count < 0) return DMS_E_ARG;
    if (count == 0) return DMS_OK;
    if (!values || !codes || !out) return DMS_E_ARG;
    if (const int dc = dms::device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    if (dtype == DMS_F32)
        hipLaunchKernelGGL(dms::k_simplex_values<float>, dim3(dms::blocks_of(count)), dim3(256), 0, s,
                           (const float *)values, n, codes, count, out);
    else
        hipLaunchKernelGGL(dms::k_simplex_values<double>, dim3(dms::blocks_of(count)), dim3(256), 0, s,
                           (const double *)values, n, codes, count, out);
    return dms::launch_status();
}

extern "C" size_t dms_gradient_backward_workspace_size(int64_t npairs)
{
    if (npairs < 0 || npairs > (1ll << 30)) return 0;
    return dms::bwd_layout(npairs).total;
}

extern "C" int dms_gradient_backward(const int64_t *birth_code, const int64_t *death_code,
                                     const double *g_birth, const double *g_death, int64_t npairs,
                                     double *grad, int64_t n, void *workspace, size_t workspace_bytes,
                                     void *stream)
{
    using namespace dms;
    if (npairs < 0 || n < 0 || npairs > (1ll << 30)) return DMS_E_ARG;
    if (n > 0 && !grad) return DMS_E_ARG;
    if (npairs > 0 && (!birth_code || !death_code || !g_birth || !g_death)) return DMS_E_ARG;
    if (n == 0) return DMS_OK;
    const BwdLayout L = bwd_layout(npairs);
    if (npairs > 0 && (!workspace || workspace_bytes < L.total)) return DMS_E_WORKSPACE;
    if (const int dc = device_check()) return dc;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks_of(n)), dim3(256), 0, s, grad, n);
    if (npairs > 0) {
        const int64_t m = 2 * npairs;
        char *ws = (char *)workspace;
        uint64_t *key = (uint64_t *)(ws + L.key);
        int32_t *rank = (int32_t *)(ws + L.rank), *at = (int32_t *)(ws + L.at);
        hipLaunchKernelGGL(k_backward_keys, dim3(blocks_of(m)), dim3(256), 0, s, birth_code, death_code,
                           npairs, n, key);
        const int st = launch_rank_u64(key, m, rank, ws + L.rws, (uint32_t *)(ws + L.flags), s);
        if (st) return st;
        hipLaunchKernelGGL(k_backward_place, dim3(blocks_of(m)), dim3(256), 0, s, rank, m, at);
        hipLaunchKernelGGL(k_backward_sum, dim3(blocks_of(m)), dim3(256), 0, s, at, key, m, npairs, g_birth,
                           g_death, grad);
    }
    return launch_status();
}
