// OP2-style indirect increment: every edge adds its value to the two cells
// it connects (an op_par_loop over edges with two OP_INC arguments through
// the edge-to-cell map, Sec. III-A).
//
// Two ways to run it:
//  * A plan (built once per mesh, on the host, like OP2's execution plans)
//    inverts the map: for each cell, the list of its incident edges in the
//    order the sequential loop visits them (edge index ascending; a
//    self-loop edge twice, its second cell first). The kernel then gives
//    each cell to one thread, which adds the cell's increments in exactly
//    that order: no atomics, no colouring, and the result equals the
//    sequential loop bit for bit.
//  * A scatter with float64 atomic adds: one thread per edge. Fast to set
//    up, but the order in which a cell's increments land varies from run
//    to run, so only a tolerance holds.
#include <string.h>

#include <vector>

#include "dev_common.h"
#include "pf_internal.h"

struct pf_inc_plan {
    int32_t ncells = 0, nedges = 0;
    int device = -1;
    void *dev = nullptr;  // offsets (ncells + 1) then edge lists (2 * nedges), int32
    const int32_t *off = nullptr, *idx = nullptr;
};

namespace pf {
namespace inc {

constexpr int kThreads = 256;


// cell[c] += edge[idx[k]] for k in off[c] .. off[c+1], in that order.
__global__ __launch_bounds__(kThreads) void k_gather(const int32_t *__restrict__ off, const int32_t *__restrict__ idx,
                                                     const double *__restrict__ edge, double *__restrict__ cell,
                                                     int32_t ncells) {
    const int64_t c = (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (c >= ncells) return;
    const int32_t k0 = off[c], k1 = off[c + 1];
    double v = cell[c];
    int32_t k = k0;
    // Four independent index/value loads in flight, added in order.
    for (; k + 4 <= k1; k += 4) {
        const int32_t i0 = idx[k], i1 = idx[k + 1], i2 = idx[k + 2], i3 = idx[k + 3];
        const double e0 = edge[i0], e1 = edge[i1], e2 = edge[i2], e3 = edge[i3];
        v = v + e0;
        v = v + e1;
        v = v + e2;
        v = v + e3;
    }
    for (; k < k1; ++k) v = v + edge[idx[k]];
    cell[c] = v;
}

// One thread per edge: cell[e2c[2i+1]] += edge[i]; cell[e2c[2i]] += edge[i].
__global__ __launch_bounds__(kThreads) void k_scatter(const int32_t *__restrict__ e2c, const double *__restrict__ edge,
                                                      double *__restrict__ cell, int32_t ncells, int32_t nedges) {
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= nedges) return;
    const double e = edge[i];
    const int32_t c1 = e2c[2 * i + 1], c0 = e2c[2 * i];
    // The map lives in device memory and is not validated by the host:
    // entries outside 0..ncells-1 are skipped rather than written through.
    if ((uint32_t)c1 < (uint32_t)ncells) unsafeAtomicAdd(&cell[c1], e);
    if ((uint32_t)c0 < (uint32_t)ncells) unsafeAtomicAdd(&cell[c0], e);
}

}  // namespace inc
}  // namespace pf

using namespace pf;

extern "C" {

pf_status pf_inc_plan_create(int32_t ncells, int32_t nedges, const int32_t *__restrict edge_to_cells,
                             pf_inc_plan **const __restrict plan) {
    clear_error();
    if (!plan) return fail(PF_EINVAL, "null plan out-parameter");
    *plan = nullptr;
    if (ncells < 1 || nedges < 0) return fail(PF_EINVAL, "need ncells >= 1 and nedges >= 0");
    if (nedges > (1 << 30)) return fail(PF_EUNSUPPORTED, "more than 2^30 edges");
    if (nedges > 0 && !edge_to_cells) return fail(PF_EINVAL, "null edge-to-cell map");
    for (int64_t j = 0; j < 2 * (int64_t)nedges; ++j)
        if (edge_to_cells[j] < 0 || edge_to_cells[j] >= ncells)
            return fail(PF_EINVAL, "edge " + std::to_string(j / 2) + " names a cell outside 0.." +
                                       std::to_string(ncells - 1));
    // Counting sort of the (edge, slot) visits by cell, in visit order.
    std::vector<int32_t> off((size_t)ncells + 1, 0);
    for (int64_t j = 0; j < 2 * (int64_t)nedges; ++j) ++off[(size_t)edge_to_cells[j] + 1];
    for (int32_t c = 0; c < ncells; ++c) off[(size_t)c + 1] += off[c];
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    std::vector<int32_t> idx((size_t)2 * nedges);
    for (int32_t i = 0; i < nedges; ++i) {
        idx[(size_t)fill[edge_to_cells[2 * (int64_t)i + 1]]++] = i;  // the second cell is incremented first
        idx[(size_t)fill[edge_to_cells[2 * (int64_t)i]]++] = i;
    }
    pf_inc_plan *p = new (std::nothrow) pf_inc_plan;
    if (!p) return fail(PF_ENOMEM, "plan allocation");
    p->ncells = ncells;
    p->nedges = nedges;
    (void)hipGetDevice(&p->device);
    const size_t bo = off.size() * sizeof(int32_t), bi = idx.size() * sizeof(int32_t);
    hipError_t e = hipMalloc(&p->dev, bo + bi + 4);
    if (e != hipSuccess) {
        delete p;
        return fail_hip(e, "plan allocation");
    }
    e = hipMemcpy(p->dev, off.data(), bo, hipMemcpyHostToDevice);
    if (e == hipSuccess && bi) e = hipMemcpy((char *)p->dev + bo, idx.data(), bi, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(p->dev);
        delete p;
        return fail_hip(e, "plan upload");
    }
    p->off = (const int32_t *)p->dev;
    p->idx = (const int32_t *)((char *)p->dev + bo);
    *plan = p;
    return PF_OK;
}

pf_status pf_inc_plan_run(const pf_inc_plan *p, int32_t ncells, int32_t nedges, const double *__restrict edge,
                          double *__restrict cell, void *stream) {
    clear_error();
    if (!p) return fail(PF_EINVAL, "null plan");
    if (ncells != p->ncells || nedges != p->nedges) return fail(PF_EINVAL, "sizes differ from the plan's");
    if (!cell || (nedges > 0 && !edge)) return fail(PF_EINVAL, "null array");
    if (((uintptr_t)edge | (uintptr_t)cell) % 8) return fail(PF_EINVAL, "arrays must be 8-byte aligned");
    const uintptr_t a = (uintptr_t)edge, b = (uintptr_t)cell;
    const uintptr_t na = (uintptr_t)nedges * 8, nb = (uintptr_t)ncells * 8;
    if (nedges > 0 && a < b + nb && b < a + na) return fail(PF_EALIAS, "edge and cell arrays overlap (restrict)");
    const int grid = (int)((ncells + inc::kThreads - 1) / inc::kThreads);
    hipLaunchKernelGGL(inc::k_gather, dim3(grid), dim3(inc::kThreads), 0, (hipStream_t)stream, p->off, p->idx, edge,
                       cell, ncells);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

pf_status pf_inc_plan_destroy(pf_inc_plan *p) {
    clear_error();
    if (!p) return PF_OK;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (p->device >= 0 && p->device != cur) (void)hipSetDevice(p->device);
    hipError_t e = hipFree(p->dev);
    if (p->device >= 0 && cur >= 0 && p->device != cur) (void)hipSetDevice(cur);
    delete p;
    if (e != hipSuccess) return fail_hip(e, "plan free");
    return PF_OK;
}

pf_status pf_edge_inc_atomic_f64(int32_t ncells, int32_t nedges, const int32_t *__restrict edge_to_cells,
                                 const double *__restrict edge, double *__restrict cell, void *stream) {
    clear_error();
    if (ncells < 1 || nedges < 0) return fail(PF_EINVAL, "need ncells >= 1 and nedges >= 0");
    if (nedges > (1 << 30)) return fail(PF_EUNSUPPORTED, "more than 2^30 edges");
    if (!cell || (nedges > 0 && (!edge || !edge_to_cells))) return fail(PF_EINVAL, "null array");
    if (((uintptr_t)edge | (uintptr_t)cell) % 8 || (uintptr_t)edge_to_cells % 4)
        return fail(PF_EINVAL, "misaligned array");
    const uintptr_t b = (uintptr_t)cell, nb = (uintptr_t)ncells * 8;
    const uintptr_t a = (uintptr_t)edge, na = (uintptr_t)nedges * 8;
    const uintptr_t m = (uintptr_t)edge_to_cells, nm = (uintptr_t)nedges * 8;
    if (nedges > 0 && ((a < b + nb && b < a + na) || (m < b + nb && b < m + nm)))
        return fail(PF_EALIAS, "cell array overlaps an input (restrict)");
    if (nedges == 0) return PF_OK;
    const int grid = (int)((nedges + inc::kThreads - 1) / inc::kThreads);
    hipLaunchKernelGGL(inc::k_scatter, dim3(grid), dim3(inc::kThreads), 0, (hipStream_t)stream, edge_to_cells, edge,
                       cell, ncells, nedges);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return PF_OK;
}

}  // extern "C"
