// Kernel table of the chain kernels (templates in step_kernels.h) with local
// dynamics that are not pi-invariant: the unadjusted random-walk jump
// process, whose killing rate carries the adjoint generator term of Sec.
// 6.2, eq. (killing-rate).  Built for the isotropic mixtures (Q^T p in
// closed form) with the uniform regeneration distribution.  A translation
// unit of its own, so the library's kernels compile in parallel.
#include "step_kernels.h"

namespace restore {

KernelSet find_kernels_rwu(int tgt, int d, int mu) {
    if (mu != MU_UNIFORM || tgt != TGT_ISO) return KernelSet{};
    switch (d) { RESTORE_SETS_FOR(TGT_ISO, LOC_RWU, MU_UNIFORM) default: break; }
    return KernelSet{};
}

}  // namespace restore
