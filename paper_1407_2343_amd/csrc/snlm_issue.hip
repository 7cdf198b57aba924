// Issue-rate probe: how fast one SIMD issues the instruction mix of the pair
// body of the line kernels (the lifted difference, the two fused multiply-adds
// of the running window sum, the weight, and the two fused multiply-adds and
// two adds of the accumulation; Sec. 2.1 with eq. recursion), with and
// without the exp, from 1, 2 or 4 resident waves per SIMD.  It backs the
// roofline figures the benchmark reports: the peak the line kernels are
// measured against, and the rate their own instruction mix can reach.
//
// Each lane runs eight independent copies of the body in a loop (enough
// independent work that dependencies do not stall a lone wave).  Workgroups
// are one wave; their LDS request bounds residency to the chosen number of
// waves per SIMD, so that all of them run at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <vector>

#include "snlm.h"

namespace snlm {

constexpr int kIssueStreams = 8;

// rec[4 * wave]: start and end of the wave on the constant 100 MHz clock,
// shader-clock cycles between them, and the hardware ids of its SIMD.
template <int MODE>
__global__ __launch_bounds__(64) void snlm_issue_kernel(float* out, unsigned long long* rec, int iters,
                                                        float seed) {
    extern __shared__ float occupancy_pad[];
    float xa[kIssueStreams], xb[kIssueStreams], xc[kIssueStreams], xd[kIssueStreams];
    float R[kIssueStreams], P1[kIssueStreams], P2[kIssueStreams], Q1[kIssueStreams], Q2[kIssueStreams];
    const float t = seed * (float)(threadIdx.x + 1);
#pragma unroll
    for (int j = 0; j < kIssueStreams; ++j) {
        xa[j] = t + j;
        xb[j] = t * 0.5f + j;
        xc[j] = t * 0.25f - j;
        xd[j] = t * 0.125f;
        R[j] = P1[j] = P2[j] = 0.0f;
        Q1[j] = Q2[j] = 1.0f;
    }
    const unsigned long long r0 = wall_clock64();
    const unsigned long long c0 = clock64();
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < kIssueStreams; ++j) {
            // the samples change every iteration as far as the compiler knows
            asm volatile("" : "+v"(xa[j]), "+v"(xb[j]), "+v"(xc[j]), "+v"(xd[j]));
            if (MODE == 2) {  // the exp alone
                R[j] = __builtin_amdgcn_exp2f(-__builtin_fabsf(xa[j]));
                asm volatile("" : "+v"(R[j]));
                continue;
            }
            const float de = xa[j] - xb[j], dl = xc[j] - xd[j];
            R[j] = __builtin_fmaf(de, de, R[j]);
            R[j] = __builtin_fmaf(-dl, dl, R[j]);
            const float w = MODE == 1 ? __builtin_amdgcn_exp2f(-__builtin_fabsf(R[j])) : R[j];
            P1[j] = __builtin_fmaf(w, xa[j], P1[j]);
            Q1[j] += w;
            P2[j] = __builtin_fmaf(w, xb[j], P2[j]);
            Q2[j] += w;
        }
    }
    const unsigned long long c1 = clock64();
    const unsigned long long r1 = wall_clock64();
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kIssueStreams; ++j) s += R[j] + P1[j] + P2[j] + Q1[j] + Q2[j];
    out[blockIdx.x * 64 + threadIdx.x] = s;
    if (seed < 0.0f) occupancy_pad[threadIdx.x] = s;  // never: keeps the LDS request
    if (threadIdx.x == 0) {
        rec[4 * blockIdx.x + 0] = r0;
        rec[4 * blockIdx.x + 1] = r1;
        rec[4 * blockIdx.x + 2] = c1 - c0;
        // HW_ID (SIMD [5:4], CU [11:8], shader engine [14:13]) and XCC_ID (the XCD)
        rec[4 * blockIdx.x + 3] = ((unsigned long long)__builtin_amdgcn_s_getreg(0xF814) << 32) |
                                  __builtin_amdgcn_s_getreg(0xF804);
    }
}

}  // namespace snlm

extern "C" int snlm_issue_rate(int mode, int waves_per_simd, int iters, double* clk_per_pair,
                               double* clock_ghz) {
    if (mode < 0 || mode > 2 || waves_per_simd < 1 || waves_per_simd > 4 || iters < 1 || !clk_per_pair)
        return SNLM_EINVAL;
    int dev = 0, ncu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
        return SNLM_EDEVICE;
    const int nb = ncu * 4 * waves_per_simd;
    // LDS per one-wave workgroup such that at most 4 * waves_per_simd fit a CU
    const size_t lds = (size_t)(163840 / (4 * waves_per_simd)) / 256 * 256;
    float* out = nullptr;
    unsigned long long* rec = nullptr;
    if (hipMalloc(&out, (size_t)nb * 64 * sizeof(float)) != hipSuccess) return SNLM_EDEVICE;
    if (hipMalloc(&rec, (size_t)nb * 4 * sizeof(unsigned long long)) != hipSuccess) {
        (void)hipFree(out);
        return SNLM_EDEVICE;
    }
    const void* fns[3] = {(const void*)&snlm::snlm_issue_kernel<0>, (const void*)&snlm::snlm_issue_kernel<1>,
                          (const void*)&snlm::snlm_issue_kernel<2>};
    float seed = 1.0001f;
    void* args[] = {(void*)&out, (void*)&rec, (void*)&iters, (void*)&seed};
    int rc = SNLM_OK;
    for (int rep = 0; rep < 2 && rc == SNLM_OK; ++rep)  // the first launch warms up
        if (hipLaunchKernel(fns[mode], dim3(nb), dim3(64), args, lds, nullptr) != hipSuccess ||
            hipDeviceSynchronize() != hipSuccess)
            rc = SNLM_EDEVICE;
    std::vector<unsigned long long> h((size_t)nb * 4);
    if (rc == SNLM_OK &&
        hipMemcpy(h.data(), rec, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess)
        rc = SNLM_EDEVICE;
    if (rc == SNLM_OK) {
        // shader clock from cycles over constant-clock ticks (100 MHz), all waves
        double cyc = 0.0, ticks = 0.0;
        for (int b = 0; b < nb; ++b) {
            cyc += (double)h[4 * b + 2];
            ticks += (double)(h[4 * b + 1] - h[4 * b + 0]);
        }
        const double ghz = ticks > 0.0 ? cyc / ticks / 10.0 : 0.0;
        // per SIMD (waves grouped by XCD, shader engine, CU and SIMD): the
        // pair bodies its waves retired over the span from its first wave's
        // start to its last wave's end, in cycles
        std::map<unsigned long long, std::pair<unsigned long long, unsigned long long>> span;
        std::map<unsigned long long, int> count;
        for (int b = 0; b < nb; ++b) {
            const unsigned long long id = h[4 * b + 3] & 0x0000000F00007FF0ull;
            auto it = span.find(id);
            if (it == span.end())
                span[id] = {h[4 * b + 0], h[4 * b + 1]};
            else
                it->second = {std::min(it->second.first, h[4 * b + 0]), std::max(it->second.second, h[4 * b + 1])};
            count[id] += 1;
        }
        std::vector<double> per;
        for (auto& kv : span) {
            const double cycles = (double)(kv.second.second - kv.second.first) * 10.0 * ghz;
            per.push_back(cycles / ((double)iters * snlm::kIssueStreams * count[kv.first]));
        }
        std::sort(per.begin(), per.end());
        *clk_per_pair = per.empty() ? 0.0 : per[per.size() / 2];
        if (clock_ghz) *clock_ghz = ghz;
    }
    (void)hipFree(out);
    (void)hipFree(rec);
    return rc;
}
