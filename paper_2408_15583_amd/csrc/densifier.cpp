// Learned densifier (U-Net) host side.
#include "pe_runtime.h"

using namespace pe;

extern "C" {
pe_status pe_densifier_create(pe_ctx, int32_t, uint64_t, pe_densifier*) { return set_error(PE_EUNSUPPORTED, "densifier not built"); }
pe_status pe_densifier_destroy(pe_densifier) { return PE_OK; }
pe_status pe_densifier_save(pe_densifier, const char*) { return set_error(PE_EUNSUPPORTED, "densifier not built"); }
pe_status pe_densifier_load(pe_densifier, const char*) { return set_error(PE_EUNSUPPORTED, "densifier not built"); }
pe_status pe_densifier_num_params(pe_densifier, uint64_t*) { return set_error(PE_EUNSUPPORTED, "densifier not built"); }
pe_status pe_densifier_train_step(pe_densifier, int32_t, int32_t, int32_t, const float*, const float*, const float*, const float*, float, float, double*, void*) { return set_error(PE_EUNSUPPORTED, "densifier not built"); }
pe_status pe_densifier_infer(pe_densifier, int32_t, int32_t, int32_t, const float*, float*, float*, float*, void*) { return set_error(PE_EUNSUPPORTED, "densifier not built"); }
}
