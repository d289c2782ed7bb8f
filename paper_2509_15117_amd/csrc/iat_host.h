// Host-side helpers shared by the libiat entry points (validation, parameter blocks, errors).
#pragma once

#include "iat.h"
#include "iat_device.h"

namespace iat {

int set_error(int code, const char* fmt, ...);
const char* last_error();
int device_state(int* n_cu, unsigned long long** queue_slot);
void release_devices();
int validate_common(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch);
void fill_params(KParams& P, const iat_system* sys, const iat_species* species, int n_species,
                 const iat_batch* batch);
void fill_outputs(KParams& P, const iat_obs* obs);
int resolve_launch(const iat_launch* launch, iat_launch* out);

}  // namespace iat
