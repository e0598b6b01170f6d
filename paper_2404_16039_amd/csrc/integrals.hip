// integrals.hip -- integration points of a rule on every cell and the GI function
// (section 3.3 and 3.5: X_ip = amsm(coords3D, ip); section 3.4: GI(fip, w, sizes, normals)).
//
// A rule is given by the caller as barycentric points (nq x nv) and weights summing to 1,
// so any order the caller needs (the paper's Gauss_points for a chosen gqo) runs through
// the same kernels; both travel as kernel arguments (at most PF_RULE_MAX points).
// GI reduces in FP64 over a fixed grid: every block sums its share of the values in a fixed
// order, one block adds the block sums in block order, so the value is deterministic.
#include "common.hpp"

#include <string>

namespace pf {

constexpr int IBS = 256;

struct Rule {
    double lam[PF_RULE_MAX * 4];
    double w[PF_RULE_MAX];
};

// X[(c nq + q) dim + i] = sum_j lam_qj coords[cells[c nv + j] dim + i]; NaN for a bad node.
// A block takes pc consecutive cells (pc = min(PC_MAX, PB / nq), passed by the host): it
// stages their node coordinates (a bad node's as NaN, which every point of its cell then
// carries) and the rule in LDS with one load per value, then thread k makes output word k of
// the block's contiguous run of pc nq dim values (one coordinate of one point), so the
// stores are coalesced with no staging of the results.
#ifndef PF_POINTS_BS
#define PF_POINTS_BS 512
#endif
#ifndef PF_POINTS_PB
#define PF_POINTS_PB 8192
#endif
constexpr int SPT = PF_POINTS_BS;  // threads per block
constexpr int PB = PF_POINTS_PB;   // points per block at most
#ifndef PF_POINTS_CELLS
#define PF_POINTS_CELLS 256
#endif
constexpr int PC_MAX = PF_POINTS_CELLS;  // cells per block at most
template <int DIM, int NV>
__global__ __launch_bounds__(SPT) void k_simplex_points(int64_t nn, const double* __restrict__ coords, int64_t nc,
                                                        const int32_t* __restrict__ cells, int nq, int pc, Rule rule,
                                                        double* __restrict__ X) {
    __shared__ double xs[PC_MAX * NV * DIM];
    __shared__ double lam[PF_RULE_MAX * NV];
    const int64_t c0 = static_cast<int64_t>(blockIdx.x) * pc;
    const int ncb = static_cast<int>(nc - c0 < pc ? nc - c0 : pc);
    for (int u = threadIdx.x; u < ncb * NV * DIM; u += SPT) {
        const int c = u / (NV * DIM), j = (u / DIM) % NV, i = u % DIM;
        const int32_t v = cells[(c0 + c) * NV + j];
        xs[u] = v >= 0 && v < nn ? coords[static_cast<int64_t>(v) * DIM + i] : static_cast<double>(NAN);
    }
    for (int u = threadIdx.x; u < nq * NV; u += SPT) lam[u] = rule.lam[u];
    __syncthreads();
    const float rq = 1.0f / static_cast<float>(nq);
    double* out = X + c0 * nq * DIM;
    const int nw = ncb * nq * DIM;
    for (int k = threadIdx.x; k < nw; k += SPT) {
        const int u = k / DIM, i = k - u * DIM;  // point u of the block, coordinate i
        int c = static_cast<int>(static_cast<float>(u) * rq);  // u / nq (u < PB: one correction step)
        c += (c + 1) * nq <= u;
        c -= c * nq > u;
        const int q = u - c * nq;
        const double* xc = xs + c * (NV * DIM) + i;
        const double* lq = lam + q * NV;
        double x = lq[0] * xc[0];
#pragma unroll
        for (int j = 1; j < NV; ++j) x = __builtin_fma(lq[j], xc[j * DIM], x);
        out[k] = x;
    }
}

// Block sums of sizes[c] * f_c, f_c = sum_i n_ci sum_q w_q fip[c, q, i] (n = 1 without
// normals), reading fip as one flat array: value k of the grid-strided sweep belongs to cell
// k / (nq d) at position r = k mod (nq d); each lane advances (cell, r) by fixed steps, so
// consecutive lanes read consecutive values with no division in the loop.
template <typename T>
__global__ __launch_bounds__(IBS) void k_gi(int64_t nc, int nq, int d, const T* __restrict__ fip, Rule rule,
                                            const T* __restrict__ sizes, const T* __restrict__ normals,
                                            double* __restrict__ part) {
    __shared__ double wr[PF_RULE_MAX * 3];  // weight of position r: w[r / d]
    __shared__ double red[IBS / 64];
    const int nqd = nq * d;
    for (int r = threadIdx.x; r < nqd; r += IBS) wr[r] = rule.w[r / d];
    __syncthreads();
    const int64_t total = nc * nqd;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * IBS;
    int64_t k = static_cast<int64_t>(blockIdx.x) * IBS + threadIdx.x;
    int64_t c = k / nqd;
    int r = static_cast<int>(k - c * nqd);
    const int64_t dc = stride / nqd;
    const int dr = static_cast<int>(stride - dc * nqd);
    double sum = 0.0;
    for (; k < total; k += stride) {
        const int i = r % d;
        double v = wr[r] * static_cast<double>(fip[k]) * static_cast<double>(sizes[c]);
        if (normals) v *= static_cast<double>(normals[c * d + i]);
        sum += v;
        c += dc;
        r += dr;
        if (r >= nqd) {
            r -= nqd;
            ++c;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) sum += __shfl_xor(sum, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < IBS / 64; ++w) s += red[w];
        part[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(64) void k_gi_total(const double* __restrict__ part, int nblocks, double* __restrict__ value) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += 64) s += part[b];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) *value = s;
}

}  // namespace pf

using namespace pf;

pf_status pf_simplex_points(int dim, int nv, int64_t nn, const double* coords, int64_t nc, const int32_t* cells,
                            int nq, const double* lam, double* X, void* stream) {
    if (dim != 2 && dim != 3) return fail(PF_EORDER, "pf_simplex_points: dim must be 2 or 3");
    if (nv < 2 || nv > dim + 1) return fail(PF_EINVAL, "pf_simplex_points: nv must be 2..dim+1");
    if (nq < 1 || nq > PF_RULE_MAX) return fail(PF_EINVAL, "pf_simplex_points: nq must be 1..PF_RULE_MAX");
    if (nn < 0 || nc < 0) return fail(PF_EINVAL, "pf_simplex_points: negative size");
    if (nc == 0) return PF_OK;
    if (!coords || !cells || !lam || !X) return fail(PF_EINVAL, "pf_simplex_points: null argument");
    Rule rule{};
    for (int i = 0; i < nq * nv; ++i) rule.lam[i] = lam[i];
    hipStream_t s = as_stream(stream);
    const int pc = std::max(1, std::min(PC_MAX, PB / nq));  // cells per block: pc nq <= PB points
    const unsigned g = static_cast<unsigned>(ceil_div(nc, pc));
    if (dim == 3) {
        if (nv == 4) hipLaunchKernelGGL((k_simplex_points<3, 4>), dim3(g), dim3(SPT), 0, s, nn, coords, nc, cells, nq, pc, rule, X);
        else if (nv == 3) hipLaunchKernelGGL((k_simplex_points<3, 3>), dim3(g), dim3(SPT), 0, s, nn, coords, nc, cells, nq, pc, rule, X);
        else hipLaunchKernelGGL((k_simplex_points<3, 2>), dim3(g), dim3(SPT), 0, s, nn, coords, nc, cells, nq, pc, rule, X);
    } else {
        if (nv == 3) hipLaunchKernelGGL((k_simplex_points<2, 3>), dim3(g), dim3(SPT), 0, s, nn, coords, nc, cells, nq, pc, rule, X);
        else hipLaunchKernelGGL((k_simplex_points<2, 2>), dim3(g), dim3(SPT), 0, s, nn, coords, nc, cells, nq, pc, rule, X);
    }
    return launch_check("pf_simplex_points");
}

pf_status pf_gi(pf_dtype prec, int64_t nc, int nq, int d, const void* fip, const double* w, const void* sizes,
                const void* normals, double* value, double* work, void* stream) {
    if (prec != PF_F32 && prec != PF_F64) return fail(PF_EDTYPE, "pf_gi: prec must be PF_F32 or PF_F64");
    if (nq < 1 || nq > PF_RULE_MAX) return fail(PF_EINVAL, "pf_gi: nq must be 1..PF_RULE_MAX");
    if (d < 1 || d > 3) return fail(PF_EINVAL, "pf_gi: d must be 1..3");
    if (nc < 0) return fail(PF_EINVAL, "pf_gi: negative size");
    if (!w || !value || !work) return fail(PF_EINVAL, "pf_gi: null w, value or work");
    if (nc > 0 && (!fip || !sizes)) return fail(PF_EINVAL, "pf_gi: null fip or sizes");
    Rule rule{};
    for (int q = 0; q < nq; ++q) rule.w[q] = w[q];
    hipStream_t s = as_stream(stream);
    const int grid = static_cast<int>(std::max<int64_t>(std::min<int64_t>(ceil_div(nc * nq * d, IBS), PF_GI_WORK), 1));
    if (prec == PF_F32)
        hipLaunchKernelGGL(k_gi<float>, dim3(grid), dim3(IBS), 0, s, nc, nq, d, static_cast<const float*>(fip), rule,
                           static_cast<const float*>(sizes), static_cast<const float*>(normals), work);
    else
        hipLaunchKernelGGL(k_gi<double>, dim3(grid), dim3(IBS), 0, s, nc, nq, d, static_cast<const double*>(fip), rule,
                           static_cast<const double*>(sizes), static_cast<const double*>(normals), work);
    hipLaunchKernelGGL(k_gi_total, dim3(1), dim3(64), 0, s, work, grid, value);
    return launch_check("pf_gi");
}
