// Kernel table of the chain kernels (templates in step_kernels.h) for the
// random-walk and Langevin small-step kernels, the rendering-shaped
// integrand and the learned regeneration distribution; the Hamiltonian
// kernels are instantiated in step_kernels_hmc.hip.
#include "step_kernels.h"

namespace restore {

KernelSet find_kernels(int tgt, int d, int loc, int mu) {
    if (loc == LOC_HMC) return find_kernels_hmc(tgt, d, mu);
    if (loc == LOC_RWU) return find_kernels_rwu(tgt, d, mu);
    if (mu == MU_GMM) {
        // learned regeneration distribution: the mixtures of the learned-mu workloads
        if (tgt == TGT_FULL && loc == LOC_MALA) {
            switch (d) { case 2: return make_set<2, TGT_FULL, LOC_MALA, MU_GMM>();
                         case 8: return make_set<8, TGT_FULL, LOC_MALA, MU_GMM>(); default: break; }
        }
        if (tgt == TGT_FULL && loc == LOC_RWMH) {
            switch (d) { case 2: return make_set<2, TGT_FULL, LOC_RWMH, MU_GMM>();
                         case 8: return make_set<8, TGT_FULL, LOC_RWMH, MU_GMM>(); default: break; }
        }
        if (tgt == TGT_ISO && loc == LOC_RWMH && d == 2) return make_set<2, TGT_ISO, LOC_RWMH, MU_GMM>();
        // the rendering-shaped integrand (image splats, binned or direct)
        if (tgt == TGT_PSS && loc == LOC_RWMH && d == 12) return make_set<12, TGT_PSS, LOC_RWMH, MU_GMM>();
        return KernelSet{};
    }
    if (tgt == TGT_PSS) {
        if (d == 12 && loc == LOC_RWMH) return make_set<12, TGT_PSS, LOC_RWMH, MU_UNIFORM>();
        return KernelSet{};
    }
    if (tgt == TGT_ISO && loc == LOC_RWMH) {
        switch (d) { RESTORE_SETS_FOR(TGT_ISO, LOC_RWMH, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_ISO && loc == LOC_MALA) {
        switch (d) { RESTORE_SETS_FOR(TGT_ISO, LOC_MALA, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_FULL && loc == LOC_RWMH) {
        switch (d) { RESTORE_SETS_FOR(TGT_FULL, LOC_RWMH, MU_UNIFORM) default: break; }
    } else if (tgt == TGT_FULL && loc == LOC_MALA) {
        switch (d) { RESTORE_SETS_FOR(TGT_FULL, LOC_MALA, MU_UNIFORM) default: break; }
    }
    return KernelSet{};
}

}  // namespace restore
