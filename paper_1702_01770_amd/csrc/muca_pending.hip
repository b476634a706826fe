// Entry points whose kernels live in other translation units still being written.
#include "../../include/muca.h"
#include "muca_internal.h"
#include <string>
extern "C" {
int muca_energy_fwd(muca_ctx *, int32_t, const float *, int64_t, const double *, double *) { return MUCA_E_STATE; }
int muca_energy_bwd(muca_ctx *, int32_t, const float *, int64_t, const double *, const double *, float *, double *) { return MUCA_E_STATE; }
size_t muca_reweight_workspace_bytes(int64_t, int32_t) { return 0; }
int muca_reweight_fwd(const double *, const double *, int64_t, const double *, int32_t, double *, double *, double *, void *, size_t, void *) { return MUCA_E_STATE; }
int muca_reweight_bwd(const double *, const double *, int64_t, const double *, int32_t, const double *, const double *, const double *, double *, void *) { return MUCA_E_STATE; }
int microcanonical_analyze(const muca_analysis_in *, muca_analysis_out *) { return MUCA_E_STATE; }
}
