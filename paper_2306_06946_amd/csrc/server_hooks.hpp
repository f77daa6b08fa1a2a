// Library-internal calls the serving runtime makes on a scene beyond the
// public C ABI (host declarations only; defined in api.hip).
#pragma once

#include <cstddef>
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

// Batched Newton loops (the serving path).  A step whose Newton loop can run
// in the batched launch (fast scheme, FP64, no pair contacts, 1..512
// contacts, untimed): newton_batchable.  step_begin applies icr_step's
// checks and enqueues the step up to its Newton loop on the scene's stream,
// and writes the scene's task (newton_task_bytes() bytes, the device table
// entry) to `task`; newton_batch runs the Newton loops of the table entries
// idx[0..n) (n <= 64; entry k at byte k * newton_task_bytes() of the device
// table `tasks`) in one launch on `stream`, after every step_begin of
// those scenes completed (the caller orders the streams); step_end enqueues
// the rest of the step on the scene's stream after the batch.
size_t newton_task_bytes();
bool newton_batchable(const icr_scene *s, const icr_step_opts *opt);
icr_status step_begin(icr_scene *s, const icr_obstacle *obs, const icr_step_opts *opt, void *task);
icr_status step_end(icr_scene *s, const icr_step_opts *opt);
icr_status newton_batch(void *stream, const void *tasks, const int *idx, int n, std::string &msg);

}  // namespace icr
