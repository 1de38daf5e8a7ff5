// Library-internal calls between the simulation handle (icwf_api.cpp) and the
// server (icwf_server.cpp); not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/icwf.h"

// The shape key of a simulation that icwf_step_batch can advance together
// with others of the same key (false: it can only step alone).
bool icwf_internal_batch_key(const icwf_sim *sim, std::string *key);

// Move a handle's later work to another stream (its earlier work must be
// complete: the caller synchronises the old stream first).
void icwf_internal_set_stream(icwf_sim *sim, hipStream_t stream);
