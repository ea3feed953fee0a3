// Kernel table of the chain kernels (templates in step_kernels.h) with the
// Hamiltonian Monte Carlo small-step kernel, the third local dynamics of
// the paper's study (Sec. 9), for the Gaussian-mixture targets with the
// uniform regeneration distribution.  A translation unit of its own, so the
// library's kernels compile in parallel.
#include "step_kernels.h"

namespace restore {

KernelSet find_kernels_hmc(int tgt, int d, int mu) {
    if (mu != MU_UNIFORM) return KernelSet{};
    if (tgt == TGT_ISO) {
        switch (d) { RESTORE_SETS_FOR(TGT_ISO, LOC_HMC, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_FULL) {
        switch (d) { RESTORE_SETS_FOR(TGT_FULL, LOC_HMC, MU_UNIFORM) default: break; }
    }
    return KernelSet{};
}

}  // namespace restore
