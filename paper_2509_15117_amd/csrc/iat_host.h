// Host-side helpers shared by the libiat entry points (validation, parameter blocks, errors).
#pragma once

#include "iat.h"
#include "iat_device.h"

namespace iat {

int set_error(int code, const char* fmt, ...);
const char* last_error();
int device_state(int* n_cu);
void release_devices();
int validate_common(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch);
void fill_params(KParams& P, const iat_system* sys, const iat_species* species, int n_species,
                 const iat_batch* batch);
void fill_outputs(KParams& P, const iat_obs* obs);
int resolve_launch(const iat_launch* launch, iat_launch* out);
// setup (ids -> start states, lane constants) and observables kernels over a work buffer
void launch_setup(const KParams& P, const Work& W, hipStream_t st);
void launch_observe(const KParams& P, const Work& W, hipStream_t st);
// device bytes that iat_integrate and iat_reduce allocate for a batch (host only, nothing launched)
int integrate_ws_bytes(const iat_system* sys, const iat_species* species, int n_species, const iat_batch* batch,
                       const iat_launch* launch, size_t* bytes);
int reduce_ws_bytes(const iat_batch* batch, int kind, size_t* bytes);

// HIP-event timing of a call's phases into a host float[kMarks - 1] (no-op when out is NULL).
class PhaseTimer {
public:
    static constexpr int kMarks = 6;
    PhaseTimer(float* out, hipStream_t st);
    ~PhaseTimer();
    // k = 0..5: before setup, after setup, after main, after tail, after solo, after observe
    void mark(int k);
    int finish();          // waits for the last mark; 0 or an error code
private:
    float* out_;
    hipStream_t st_;
    hipEvent_t ev_[kMarks] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
};

}  // namespace iat
