// dms_misc.hip -- status strings, table export and the backward scatter of
// the differentiable D0 form.
#include "dms_common.hpp"
#include "dms_tables.hpp"

namespace dms {
namespace {

// Section 2.5: the birth and death of a pair are the highest vertex values
// of its two simplices, so their derivatives with respect to the field are
// indicator vectors at the max vertices (code >> 8).  Births are minima and
// deaths are edges with lower vertices, so the two target sets are disjoint;
// a death vertex may be the max vertex of several critical edges, whose
// contributions are summed by the first pair of each run of equal max
// vertex, in pair order, before a single atomic add.
__global__ void k_backward(const int64_t *__restrict__ bcode, const int64_t *__restrict__ dcode,
                           const double *__restrict__ gb, const double *__restrict__ gd, int64_t npairs,
                           double *__restrict__ grad, int64_t n)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npairs) return;
    const int64_t b = bcode[p] >> 8;
    if (b >= 0 && b < n) atomicAdd(&grad[b], gb[p]);
    const int64_t v = dcode[p] >> 8;
    if (p > 0 && (dcode[p - 1] >> 8) == v) return;
    double s = gd[p];
    for (int64_t q = p + 1; q < npairs && (dcode[q] >> 8) == v; ++q) s += gd[q];
    if (v >= 0 && v < n) atomicAdd(&grad[v], s);
}

__global__ void k_fill_zero(double *__restrict__ x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0;
}

}  // namespace
}  // namespace dms

extern "C" const char *dms_status_str(int status)
{
    switch (status) {
    case DMS_OK: return "DMS_OK";
    case DMS_E_ARG: return "DMS_E_ARG: invalid argument";
    case DMS_E_SIZE: return "DMS_E_SIZE: grid too large for int32 orders";
    case DMS_E_WORKSPACE: return "DMS_E_WORKSPACE: workspace missing or too small";
    case DMS_E_UNSUPPORTED: return "DMS_E_UNSUPPORTED: no gfx950 device";
    case DMS_E_HIP: return "DMS_E_HIP: HIP runtime error";
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

extern "C" int dms_gradient_backward(const int64_t *birth_code, const int64_t *death_code,
                                     const double *g_birth, const double *g_death, int64_t npairs,
                                     double *grad, int64_t n, void *stream)
{
    if (npairs < 0 || n < 0) return DMS_E_ARG;
    if (n > 0 && !grad) return DMS_E_ARG;
    if (npairs > 0 && (!birth_code || !death_code || !g_birth || !g_death)) return DMS_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (n > 0)
        hipLaunchKernelGGL(dms::k_fill_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, grad, n);
    if (npairs > 0)
        hipLaunchKernelGGL(dms::k_backward, dim3((unsigned)((npairs + 255) / 256)), dim3(256), 0, s,
                           birth_code, death_code, g_birth, g_death, npairs, grad, n);
    return dms::launch_status();
}
