// Serving runtime: admitted scenes, a FIFO of step requests and a fixed set
// of slots (one HIP stream each).  The startable requests (the oldest of
// idle scenes) are spread over the free slots, up to the group size per
// slot, and each slot runs its group in its stream's order: with batching on, every request whose Newton loop
// can run batched (fast scheme, FP64, no pair contacts, at most 512
// contacts) enqueues its step up to the Newton loop, one launch runs all
// their Newton loops (one workgroup per scene, k_newton_batch), then each
// finishes its step; other requests run icr_step whole.  Each request ends
// with a copy of its PGS eps values into its pinned host buffer (the step's
// convergence status) and an event that marks its completion; the slot is
// free again once its whole group completed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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

constexpr int kEpsSlots = 256;   // Newton iterations per step at most
constexpr int kGroupMax = 64;    // requests per slot and round at most (one batched launch)

struct Member {                  // one request of a slot's group
  hipEvent_t done = nullptr;
  double *eps = nullptr;         // pinned host: eps of every Newton iteration of the request
  bool pending = false;          // in flight, not yet reported
  Request req;
};

struct Slot {
  hipStream_t stream = nullptr;
  void *task = nullptr;          // pinned host: the group's Newton tasks (kGroupMax entries)
  Member mem[kGroupMax];
  int n = 0;                     // requests of the current group
  bool running = false;          // a group is in flight
};

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
  int group = 8;             // requests per slot and round; 0: one whole step per slot (no batching)
  double max_wait_ms = 0.0;  // a short group waits this long for more requests while another slot runs
  void *d_tasks = nullptr;   // device table of Newton tasks, kGroupMax entries per slot
  size_t task_bytes = 0;
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

// A request whose launch failed becomes a completion with the failing
// status; whatever was enqueued on the slot stream finishes before the scene
// goes back to its own stream, and the scene stays usable.
void fail_request(icr_server *srv, Slot &sl, const Request &r, icr_status st) {
  SceneEntry &se = srv->scenes[r.scene];
  (void)hipStreamSynchronize(sl.stream);
  (void)icr_set_stream(se.s, se.own_stream);
  se.busy = false;
  icr_completion c{};
  c.tag = r.tag;
  c.scene = r.scene;
  c.status = st;
  c.latency_ms = c.queue_ms = ms_since(r.t_submit, Clock::now());
  srv->failed.push_back(c);
}

// Take a group for every free slot and enqueue it (see the top of the file).
// The startable requests (the oldest of idle scenes) are spread evenly over
// the free slots, at most `group` per slot: short rounds while the load is
// light, full launches under load.  With max_wait_ms > 0, fewer startable
// requests than a full group wait until the oldest of them has waited that
// long, or until no slot runs.
void launch_ready(icr_server *srv) {
  const int gmax = srv->group > 0 ? srv->group : 1;
  int nfree = 0;
  for (const Slot &sl : srv->slots) nfree += sl.running ? 0 : 1;
  if (nfree == 0) return;
  int ready = 0;
  const Request *oldest = nullptr;
  std::vector<char> seen(srv->scenes.size(), 0);
  for (const Request &r : srv->queue)
    if (!srv->scenes[r.scene].busy && !seen[r.scene]) {
      seen[r.scene] = 1;
      if (!oldest) oldest = &r;
      if (++ready >= nfree * gmax) break;
    }
  if (ready == 0) return;
  if (srv->group > 1 && srv->max_wait_ms > 0 && ready < gmax && nfree < (int)srv->slots.size() &&
      ms_since(oldest->t_submit, Clock::now()) < srv->max_wait_ms)
    return;
  const int per_slot = std::min(gmax, (ready + nfree - 1) / nfree);
  for (int k = 0; k < (int)srv->slots.size(); ++k) {
    Slot &sl = srv->slots[k];
    if (sl.running) continue;
    std::vector<Request> grp;
    for (auto it = srv->queue.begin(); it != srv->queue.end() && (int)grp.size() < per_slot;) {
      if (srv->scenes[it->scene].busy) {
        ++it;
        continue;
      }
      srv->scenes[it->scene].busy = true;
      srv->scenes[it->scene].queued--;
      grp.push_back(*it);
      it = srv->queue.erase(it);
    }
    if (grp.empty()) return;
    sl.n = 0;
    std::vector<int> batched;   // member indices whose Newton loops run in the group's launch
    auto task_of = [&](int j) { return static_cast<char *>(sl.task) + (size_t)j * srv->task_bytes; };
    // whole steps, and the batched steps up to their Newton loops
    for (const Request &r : grp) {
      SceneEntry &se = srv->scenes[r.scene];
      const int j = sl.n;
      icr_status st = icr_set_stream(se.s, sl.stream);
      const bool b = srv->group > 0 && icr::newton_batchable(se.s, &r.opt);
      if (b) {
        if (st == ICR_OK) st = icr::step_begin(se.s, &r.obs, &r.opt, task_of(j));
        if (st == ICR_OK) {
          void *dst = static_cast<char *>(srv->d_tasks) + ((size_t)k * kGroupMax + j) * srv->task_bytes;
          if (hipMemcpyAsync(dst, task_of(j), srv->task_bytes, hipMemcpyHostToDevice, sl.stream) != hipSuccess)
            st = ICR_E_HIP;
        }
      } else {
        if (st == ICR_OK) st = icr_step(se.s, &r.obs, &r.opt, nullptr);
        if (st == ICR_OK) st = icr::enqueue_eps_readback(se.s, r.opt.n_newton, sl.mem[j].eps);
        if (st == ICR_OK && hipEventRecord(sl.mem[j].done, sl.stream) != hipSuccess) st = ICR_E_HIP;
      }
      if (st != ICR_OK) {
        fail_request(srv, sl, r, st);
        continue;
      }
      Member &m = sl.mem[j];
      m.req = r;
      m.req.t_launch = Clock::now();
      m.pending = !b;   // a batched member is pending once its step is complete
      if (b) batched.push_back(j);
      sl.n++;
    }
    if (!batched.empty()) {
      std::vector<int> idx(batched.size());
      for (size_t q = 0; q < batched.size(); ++q) idx[q] = k * kGroupMax + batched[q];
      std::string msg;
      const icr_status bst = icr::newton_batch(sl.stream, srv->d_tasks, idx.data(), (int)idx.size(), msg);
      for (int j : batched) {
        Member &m = sl.mem[j];
        SceneEntry &se = srv->scenes[m.req.scene];
        icr_status st = bst;
        if (st == ICR_OK) st = icr::step_end(se.s, &m.req.opt);
        if (st == ICR_OK) st = icr::enqueue_eps_readback(se.s, m.req.opt.n_newton, m.eps);
        if (st == ICR_OK && hipEventRecord(m.done, sl.stream) != hipSuccess) st = ICR_E_HIP;
        if (st != ICR_OK) {
          fail_request(srv, sl, m.req, st);
          continue;
        }
        m.pending = true;
      }
    }
    int live = 0;
    for (int j = 0; j < sl.n; ++j) live += sl.mem[j].pending ? 1 : 0;
    sl.running = live > 0;
  }
}

// Status of a completed request: ICR_WARN_NOT_CONVERGED when tol > 0 and a
// Newton iteration's PGS ended with eps > tol (tol = 0 asks for a fixed
// sweep count: no convergence test), else ICR_OK.
int32_t step_status(const Member &m) {
  const icr_step_opts &o = m.req.opt;
  if (!(o.tol > 0)) return ICR_OK;
  for (int k = 0; k < o.n_newton; ++k)
    if (!(m.eps[k] <= o.tol)) return ICR_WARN_NOT_CONVERGED;
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
  srv->task_bytes = icr::newton_task_bytes();   // the table's entry stride, as the kernel indexes it
  if (hipMalloc(&srv->d_tasks, srv->task_bytes * kGroupMax * slots) != hipSuccess) {
    srv->d_tasks = nullptr;
    icr_server_destroy(srv);
    return ICR_E_HIP;
  }
  for (auto &sl : srv->slots) {
    bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
              hipHostMalloc(&sl.task, srv->task_bytes * kGroupMax, hipHostMallocDefault) == hipSuccess;
    for (int j = 0; ok && j < kGroupMax; ++j)
      ok = hipEventCreateWithFlags(&sl.mem[j].done, hipEventDisableTiming) == hipSuccess &&
           hipHostMalloc((void **)&sl.mem[j].eps, sizeof(double) * kEpsSlots, hipHostMallocDefault) == hipSuccess;
    if (!ok) {
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
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    for (int j = 0; j < sl.n; ++j) {
      Member &m = sl.mem[j];
      if (!m.pending) continue;
      SceneEntry &se = srv->scenes[m.req.scene];
      if (se.s) (void)icr_set_stream(se.s, se.own_stream);
    }
    for (auto &m : sl.mem) {
      if (m.done) (void)hipEventDestroy(m.done);
      if (m.eps) (void)hipHostFree(m.eps);
    }
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.task) (void)hipHostFree(sl.task);
  }
  if (srv->d_tasks) (void)hipFree(srv->d_tasks);
  delete srv;
}

const char *icr_server_last_error(const icr_server *srv) { return srv ? srv->err.c_str() : "null server"; }

icr_status icr_server_set_batching(icr_server *srv, int32_t group, double max_wait_ms) {
  return guarded_srv(srv, [&] {
    if (group < 0 || group > kGroupMax) throw ServerError(ICR_E_ARG, "group size in [0, 64]");
    if (!(max_wait_ms >= 0.0) || !std::isfinite(max_wait_ms)) throw ServerError(ICR_E_ARG, "max_wait_ms >= 0");
    srv->group = group;
    srv->max_wait_ms = max_wait_ms;
    return ICR_OK;
  });
}

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
        int live = 0;
        for (int j = 0; j < sl.n; ++j) {
          Member &m = sl.mem[j];
          if (!m.pending) continue;
          if (n >= cap) {
            live++;
            continue;
          }
          const hipError_t q = hipEventQuery(m.done);
          if (q == hipErrorNotReady) {
            live++;
            continue;
          }
          hip_check(q, "hipEventQuery");
          const auto now = Clock::now();
          icr_completion &c = out[n++];
          c.tag = m.req.tag;
          c.scene = m.req.scene;
          c.status = step_status(m);
          c.latency_ms = ms_since(m.req.t_submit, now);
          c.queue_ms = ms_since(m.req.t_submit, m.req.t_launch);
          SceneEntry &se = srv->scenes[m.req.scene];
          (void)icr_set_stream(se.s, se.own_stream);   // its request is complete on the slot stream
          se.busy = false;
          m.pending = false;
        }
        sl.running = live > 0;
        any_running = any_running || sl.running;
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
      for (auto &sl : srv->slots)
        for (int j = 0; j < sl.n; ++j) p += sl.mem[j].pending ? 1 : 0;
      *pending_out = p;
    }
    return ICR_OK;
  });
}

}  // extern "C"
