// Library-internal calls the serving runtime makes on a scene beyond the
// public C ABI (host declarations only; defined in api.hip).
#pragma once

#include <string>

#include "icr.h"

namespace icr {

// The argument checks icr_step applies to (obs, opt), without running a
// step; returns ICR_OK or the status icr_step would return, with a message.
icr_status check_step_request(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt, std::string &msg);

// Enqueue on the scene's stream a copy of the final eps of the first
// n_newton Newton iterations of the last enqueued step into host memory
// `dst` (pinned: the copy completes in stream order).
icr_status enqueue_eps_readback(icr_scene *s, int n_newton, double *dst);

// Contacts the scene's step buffers hold without growing (icr_reserve).
int reserved_contacts(const icr_scene *s);

// Contact candidates of the scene (0 before icr_set_candidates).
int candidate_count(const icr_scene *s);

// The HIP stream the scene enqueues on (as void*).
void *scene_stream(const icr_scene *s);

// Whether the buffers of an ICR_FP32_IR step are allocated for the reserved contacts.
bool mixed_reserved(const icr_scene *s);

}  // namespace icr
