// Instantiates every kernel variant for one search half-width S, given on the
// compiler command line as -DSNLM_S=<S>, and registers their entry points.
#include "snlm_registry.hpp"

#ifndef SNLM_S
#error "compile with -DSNLM_S=<0..16>"
#endif

namespace snlm {
namespace {

template <int K>
void register_k(KernelRegistry* reg) {
    if constexpr (SNLM_S == 0) {
        const void* f = (const void*)&snlm_kernel<0, 0, false, false, false, false>;
        for (int v = 0; v < kNumVariants; ++v)
            for (int r = 0; r < 2; ++r) reg->fn[0][K][v][r] = f;
        for (int g = 0; g < 2; ++g)
            for (int r = 0; r < 2; ++r) reg->div[0][K][g][r] = (const void*)&snlm_div_kernel<0, 0, false, false>;
    } else {
        // snlm_kernel<S, K, GAUSS, KAHAN, RESTART, ROWS>
        // snlm_div_kernel<S, K, GAUSS, ROWS>
        reg->div[SNLM_S][K][0][0] = (const void*)&snlm_div_kernel<SNLM_S, K, false, false>;
        reg->div[SNLM_S][K][0][1] = (const void*)&snlm_div_kernel<SNLM_S, K, false, true>;
        reg->div[SNLM_S][K][1][0] = (const void*)&snlm_div_kernel<SNLM_S, K, true, false>;
        reg->div[SNLM_S][K][1][1] = (const void*)&snlm_div_kernel<SNLM_S, K, true, true>;
        reg->fn[SNLM_S][K][kVarBox][0] = (const void*)&snlm_kernel<SNLM_S, K, false, false, true, false>;
        reg->fn[SNLM_S][K][kVarBox][1] = (const void*)&snlm_kernel<SNLM_S, K, false, false, true, true>;
        reg->fn[SNLM_S][K][kVarBoxKahan][0] = (const void*)&snlm_kernel<SNLM_S, K, false, true, false, false>;
        reg->fn[SNLM_S][K][kVarBoxKahan][1] = (const void*)&snlm_kernel<SNLM_S, K, false, true, false, true>;
        reg->fn[SNLM_S][K][kVarGauss][0] = (const void*)&snlm_kernel<SNLM_S, K, true, false, false, false>;
        reg->fn[SNLM_S][K][kVarGauss][1] = (const void*)&snlm_kernel<SNLM_S, K, true, false, false, true>;
        reg->fn[SNLM_S][K][kVarBoxPlain][0] = (const void*)&snlm_kernel<SNLM_S, K, false, false, false, false>;
        reg->fn[SNLM_S][K][kVarBoxPlain][1] = (const void*)&snlm_kernel<SNLM_S, K, false, false, false, true>;
    }
    if constexpr (K < kMaxK) register_k<K + 1>(reg);
}

}  // namespace
}  // namespace snlm

#define SNLM_CAT2(a, b) a##b
#define SNLM_CAT(a, b) SNLM_CAT2(a, b)
extern "C" void SNLM_CAT(snlm_register_s, SNLM_S)(snlm::KernelRegistry* reg) {
    snlm::register_k<0>(reg);
#if SNLM_S > 0
    reg->iir[SNLM_S] = (const void*)&snlm::snlm_iir_nlm_kernel<SNLM_S>;
    reg->iir_fwd[SNLM_S][0] = (const void*)&snlm::snlm_iir_fwd_kernel<SNLM_S, false>;
    reg->iir_fwd[SNLM_S][1] = (const void*)&snlm::snlm_iir_fwd_kernel<SNLM_S, true>;
#endif
}
