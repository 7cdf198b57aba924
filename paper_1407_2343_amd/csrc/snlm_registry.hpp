// Table of compiled kernel entry points, filled by one registration function per
// search half-width S (each compiled in its own translation unit).
#pragma once

#include "snlm_device.hpp"
#include "snlm_sure.hpp"
#include "snlm_carry.hpp"
#include "snlm_iir.hpp"

namespace snlm {

// Running-sum / patch-kernel variants of the line kernels: box with block
// restarts (the default), box with Kahan-compensated whole-line sums, the
// exact Gaussian FIR, box with plain whole-line sums.
enum Variant { kVarBox = 0, kVarBoxKahan = 1, kVarGauss = 2, kVarBoxPlain = 3, kNumVariants = 4 };

// fn[S][K][variant][rows]: rows = 1 is the variant for passes whose lines are
// contiguous in memory (LDS transpose tiles), rows = 0 for column passes.
// div[S][K][gauss][rows]: divergence-carrying passes (block-restarted box, or
// Gauss); rows as for fn.
// iir[S]: the recursive-Gaussian pass's backward recursion and 1D NLM (S >= 1);
// iir_fwd[S][f16]: its forward recursion.
struct KernelRegistry {
    const void* fn[kMaxS + 1][kMaxK + 1][kNumVariants][2];
    const void* div[kMaxS + 1][kMaxK + 1][2][2];
    const void* iir[kMaxS + 1];
    const void* iir_fwd[kMaxS + 1][2];
};

}  // namespace snlm

extern "C" {
#define SNLM_DECLARE_REG(n) void snlm_register_s##n(snlm::KernelRegistry* reg);
SNLM_DECLARE_REG(0)
SNLM_DECLARE_REG(1)
SNLM_DECLARE_REG(2)
SNLM_DECLARE_REG(3)
SNLM_DECLARE_REG(4)
SNLM_DECLARE_REG(5)
SNLM_DECLARE_REG(6)
SNLM_DECLARE_REG(7)
SNLM_DECLARE_REG(8)
SNLM_DECLARE_REG(9)
SNLM_DECLARE_REG(10)
SNLM_DECLARE_REG(11)
SNLM_DECLARE_REG(12)
SNLM_DECLARE_REG(13)
SNLM_DECLARE_REG(14)
SNLM_DECLARE_REG(15)
SNLM_DECLARE_REG(16)
#undef SNLM_DECLARE_REG
}
