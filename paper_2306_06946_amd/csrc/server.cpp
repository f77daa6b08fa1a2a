// Serving runtime: admitted scenes, a FIFO of step requests and a fixed set
// of slots (one HIP stream each).  A request is icr_step(scene, obstacle,
// opts, NULL) enqueued on the slot's stream, followed by a copy of its PGS
// eps values into the slot's pinned host buffer (the step's convergence
// status) and an event that marks its completion.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <deque>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "icr.h"
#include "server_hooks.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_since(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Request {
  uint64_t tag = 0;
  int scene = -1;
  icr_obstacle obs{};
  icr_step_opts opt{};
  Clock::time_point t_submit, t_launch;
};

struct SceneEntry {
  icr_scene *s = nullptr;
  void *own_stream = nullptr;   // the scene's stream at admission, restored when a request ends
  int64_t bytes = 0;
  int reserved = 0;    // contacts its buffers hold (reserved at admission)
  bool admitted = false;
  bool busy = false;   // a request of this scene is in flight
  int queued = 0;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  double *eps = nullptr;   // pinned host: eps of every Newton iteration of the request
  bool running = false;
  Request req;
};

constexpr int kEpsSlots = 256;   // Newton iterations per step at most

struct ServerError : std::runtime_error {
  icr_status code;
  ServerError(icr_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) throw ServerError(ICR_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

struct icr_server {
  int64_t budget = 0, used = 0;
  std::vector<Slot> slots;
  std::vector<SceneEntry> scenes;
  std::deque<Request> queue;
  std::deque<icr_completion> failed;   // requests whose launch failed, reported by the next poll
  std::string err;
};

namespace {

template <class F>
icr_status guarded_srv(icr_server *srv, F &&body) {
  if (!srv) return ICR_E_ARG;
  srv->err.clear();
  try {
    return body();
  } catch (const ServerError &e) {
    srv->err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    srv->err = "host allocation failed";
    return ICR_E_OOM;
  } catch (const std::exception &e) {
    srv->err = e.what();
    return ICR_E_HIP;
  }
}

SceneEntry &entry(icr_server *srv, int id) {
  if (id < 0 || id >= (int)srv->scenes.size() || !srv->scenes[id].admitted)
    throw ServerError(ICR_E_ARG, "unknown scene id " + std::to_string(id));
  return srv->scenes[id];
}

// Start queued requests on free slots: the oldest request whose scene is idle.
// A request whose launch fails becomes a completion with the failing status
// (its scene stays usable) and the slot takes the next request.
void launch_ready(icr_server *srv) {
  for (auto &sl : srv->slots) {
    while (!sl.running) {
      auto it = srv->queue.begin();
      while (it != srv->queue.end() && srv->scenes[it->scene].busy) ++it;
      if (it == srv->queue.end()) return;
      Request r = *it;
      srv->queue.erase(it);
      SceneEntry &se = srv->scenes[r.scene];
      se.queued--;
      icr_status st = icr_set_stream(se.s, sl.stream);
      if (st == ICR_OK) st = icr_step(se.s, &r.obs, &r.opt, nullptr);
      if (st == ICR_OK) st = icr::enqueue_eps_readback(se.s, r.opt.n_newton, sl.eps);
      if (st != ICR_OK) {
        // whatever was enqueued on the slot stream finishes before the
        // scene goes back to its own stream
        (void)hipStreamSynchronize(sl.stream);
        (void)icr_set_stream(se.s, se.own_stream);
        icr_completion c{};
        c.tag = r.tag;
        c.scene = r.scene;
        c.status = st;
        c.latency_ms = c.queue_ms = ms_since(r.t_submit, Clock::now());
        srv->failed.push_back(c);
        continue;
      }
      hip_check(hipEventRecord(sl.done, sl.stream), "hipEventRecord");
      r.t_launch = Clock::now();
      sl.req = r;
      sl.running = true;
      se.busy = true;
    }
  }
}

// Status of a completed request: ICR_WARN_NOT_CONVERGED when tol > 0 and a
// Newton iteration's PGS ended with eps > tol (tol = 0 asks for a fixed
// sweep count: no convergence test), else ICR_OK.
int32_t step_status(const Slot &sl) {
  const icr_step_opts &o = sl.req.opt;
  if (!(o.tol > 0)) return ICR_OK;
  for (int k = 0; k < o.n_newton; ++k)
    if (!(sl.eps[k] <= o.tol)) return ICR_WARN_NOT_CONVERGED;
  return ICR_OK;
}

}  // namespace

extern "C" {

icr_status icr_server_create(icr_server **out, int64_t hbm_budget, int32_t slots) {
  if (!out) return ICR_E_ARG;
  *out = nullptr;
  if (hbm_budget <= 0 || slots < 1 || slots > 32) return ICR_E_ARG;
  icr_server *srv = new (std::nothrow) icr_server;
  if (!srv) return ICR_E_OOM;
  srv->budget = hbm_budget;
  srv->slots.resize(slots);
  for (auto &sl : srv->slots) {
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&sl.eps, sizeof(double) * kEpsSlots, hipHostMallocDefault) != hipSuccess) {
      icr_server_destroy(srv);
      return ICR_E_HIP;
    }
  }
  *out = srv;
  return ICR_OK;
}

void icr_server_destroy(icr_server *srv) {
  if (!srv) return;
  for (auto &sl : srv->slots) {
    if (sl.running && sl.done) (void)hipEventSynchronize(sl.done);
    if (sl.running) {
      SceneEntry &se = srv->scenes[sl.req.scene];
      if (se.s) (void)icr_set_stream(se.s, se.own_stream);
    }
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.eps) (void)hipHostFree(sl.eps);
  }
  delete srv;
}

const char *icr_server_last_error(const icr_server *srv) { return srv ? srv->err.c_str() : "null server"; }

icr_status icr_server_admit(icr_server *srv, icr_scene *scene, int32_t *scene_id) {
  return guarded_srv(srv, [&] {
    if (!scene || !scene_id) throw ServerError(ICR_E_ARG, "NULL scene or id pointer");
    for (const auto &e : srv->scenes)
      if (e.admitted && e.s == scene) throw ServerError(ICR_E_ARG, "scene already admitted");
    // the scene's own stream may still hold its set-up work; requests will run
    // on the slot streams, so drain the device once here
    hip_check(hipDeviceSynchronize(), "hipDeviceSynchronize");
    icr_factor_info info{};
    icr_status st = icr_get_factor_info(scene, &info);
    if (st != ICR_OK) throw ServerError(st, std::string("scene not ready: ") + icr_last_error(scene));
    // every buffer a step allocates is allocated now and charged: the
    // contacts reserved with icr_reserve, else the candidate count
    int reserve = icr::reserved_contacts(scene);
    if (reserve < 1) {
      const int cand = icr::candidate_count(scene);
      if (cand < 1) throw ServerError(ICR_E_STATE, "scene has no contact candidates");
      st = icr_reserve(scene, cand < 4096 ? cand : 4096, ICR_FP64);
      if (st != ICR_OK) throw ServerError(st, std::string("reservation failed: ") + icr_last_error(scene));
      st = icr_get_factor_info(scene, &info);
      if (st != ICR_OK) throw ServerError(st, icr_last_error(scene));
      reserve = icr::reserved_contacts(scene);
    }
    if (srv->used + info.device_bytes > srv->budget)
      throw ServerError(ICR_E_OOM, "admission refused: " + std::to_string(info.device_bytes) + " bytes with " +
                                       std::to_string(srv->used) + " of " + std::to_string(srv->budget) +
                                       " in use");
    // one stream per request: the scene's second stream would only contend
    // with the slots for the hardware queues
    const icr_status so = icr_set_overlap(scene, 0);
    if (so != ICR_OK) throw ServerError(so, icr_last_error(scene));
    SceneEntry e;
    e.s = scene;
    e.own_stream = icr::scene_stream(scene);
    e.bytes = info.device_bytes;
    e.reserved = reserve;
    e.admitted = true;
    srv->scenes.push_back(e);
    srv->used += info.device_bytes;
    *scene_id = (int32_t)srv->scenes.size() - 1;
    return ICR_OK;
  });
}

icr_status icr_server_evict(icr_server *srv, int32_t scene_id) {
  return guarded_srv(srv, [&] {
    SceneEntry &e = entry(srv, scene_id);
    if (e.busy || e.queued > 0) throw ServerError(ICR_E_STATE, "scene has requests queued or in flight");
    srv->used -= e.bytes;
    e.admitted = false;
    e.s = nullptr;
    return ICR_OK;
  });
}

icr_status icr_server_used(const icr_server *srv, int64_t *bytes) {
  if (!srv || !bytes) return ICR_E_ARG;
  *bytes = srv->used;
  return ICR_OK;
}

icr_status icr_server_submit(icr_server *srv, int32_t scene_id, const icr_obstacle *obs, const icr_step_opts *opt,
                             uint64_t tag) {
  return guarded_srv(srv, [&] {
    SceneEntry &e = entry(srv, scene_id);
    if (!obs || !opt) throw ServerError(ICR_E_ARG, "NULL obstacle or options");
    std::string msg;
    const icr_status st = icr::check_step_request(e.s, obs, opt, msg);
    if (st != ICR_OK) throw ServerError(st, "request refused: " + msg);
    if (opt->precision == ICR_FP32_IR && !icr::mixed_reserved(e.s))
      throw ServerError(ICR_E_ARG, "request refused: ICR_FP32_IR steps need icr_reserve(scene, n, ICR_FP32_IR) "
                                   "before admission");
    if (opt->n_contacts > e.reserved)
      throw ServerError(ICR_E_ARG, "request refused: n_contacts " + std::to_string(opt->n_contacts) +
                                       " exceeds the " + std::to_string(e.reserved) + " contacts reserved at admission");
    Request r;
    r.tag = tag;
    r.scene = scene_id;
    r.obs = *obs;
    r.opt = *opt;
    r.t_submit = Clock::now();
    srv->queue.push_back(r);
    e.queued++;
    return ICR_OK;
  });
}

icr_status icr_server_poll(icr_server *srv, icr_completion *out, int32_t cap, int32_t *n_out, int32_t wait,
                           int32_t *pending_out) {
  return guarded_srv(srv, [&] {
    if (!n_out || (cap > 0 && !out) || cap < 0) throw ServerError(ICR_E_ARG, "bad output arguments");
    int n = 0;
    while (true) {
      launch_ready(srv);
      while (n < cap && !srv->failed.empty()) {
        out[n++] = srv->failed.front();
        srv->failed.pop_front();
      }
      bool any_running = false;
      for (auto &sl : srv->slots) {
        if (!sl.running) continue;
        if (n >= cap) {
          any_running = true;
          continue;
        }
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) {
          any_running = true;
          continue;
        }
        hip_check(q, "hipEventQuery");
        const auto now = Clock::now();
        icr_completion &c = out[n++];
        c.tag = sl.req.tag;
        c.scene = sl.req.scene;
        c.status = step_status(sl);
        c.latency_ms = ms_since(sl.req.t_submit, now);
        c.queue_ms = ms_since(sl.req.t_submit, sl.req.t_launch);
        SceneEntry &se = srv->scenes[sl.req.scene];
        (void)icr_set_stream(se.s, se.own_stream);   // its request is complete on the slot stream
        se.busy = false;
        sl.running = false;
      }
      if (n > 0) launch_ready(srv);   // freed slots take the next requests at once
      if (n > 0 || !wait || n >= cap || (!any_running && srv->queue.empty() && srv->failed.empty())) break;
      // wait for whichever slot finishes first (not the oldest: a long step
      // must not hold the other slots idle)
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    *n_out = n;
    if (pending_out) {
      int p = (int)srv->queue.size() + (int)srv->failed.size();
      for (auto &sl : srv->slots) p += sl.running ? 1 : 0;
      *pending_out = p;
    }
    return ICR_OK;
  });
}

}  // extern "C"
