// Grouped stepping of several solves: each handle advances by one SVT step
// (Alg. 6), and the fresh rSVD-BKI calls (Alg. 5) of all the handles run in
// lock-step stages whose sparse products -- one per solve and stage -- go out
// together, in one launch per lane form and value type, instead of one
// launch per solve.  Each solve's other work stays on its own stream; a
// grouped launch runs on a stream of its own after the participants' stage
// work (stream waits on their events), and every participant's stream waits
// for it before its next stage.  The products run the same per-segment code
// as a solo launch, so every result is the one the solve gets alone.
#include <mutex>
#include <vector>

#include "solver.hpp"

namespace mcsvt {

namespace {

// Device resources of the grouped launches, one set per device, kept for the
// process: a stream, the task tables (pinned staging and device copy) and an
// event that the participants' streams wait on.
struct GroupRes {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  SpmmTask* staging = nullptr;
  SpmmTask* table = nullptr;
  int64_t cap = 0;
  std::vector<hipEvent_t> evs;
};

constexpr int64_t kGroupTasks = 4096;   // task-table entries per stage loop

std::mutex g_mu;
GroupRes g_res[64];

GroupRes& resources() {
  int dev = 0;
  MC_HIP(hipGetDevice(&dev));
  MC_REQUIRE(dev >= 0 && dev < 64, kEDEVICE, "device ordinal out of range");
  GroupRes& r = g_res[dev];
  if (!r.st) {
    MC_HIP(hipStreamCreateWithFlags(&r.st, hipStreamNonBlocking));
    MC_HIP(hipEventCreateWithFlags(&r.done, hipEventDisableTiming));
    MC_HIP(hipHostMalloc((void**)&r.staging, kGroupTasks * sizeof(SpmmTask)));
    r.table = static_cast<SpmmTask*>(dev_alloc(kGroupTasks * sizeof(SpmmTask), r.st));
    r.cap = kGroupTasks;
  }
  return r;
}

hipEvent_t event_at(GroupRes& r, size_t i) {
  while (r.evs.size() <= i) {
    hipEvent_t e;
    MC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    r.evs.push_back(e);
  }
  return r.evs[i];
}

}  // namespace

// One step of every solver in `ss` (all on the current device).  A solver that
// fails gets its status and message in status[i] / err[i] and takes no
// further part; the others go on.  Returns when every live solver has
// finished its step.
void step_group(const std::vector<Solver*>& ss, std::vector<int>& status,
                std::vector<std::string>& err) {
  std::lock_guard<std::mutex> lk(g_mu);
  GroupRes& res = resources();
  const size_t n = ss.size();
  struct Undefer {
    const std::vector<Solver*>& ss;
    ~Undefer() {
      for (Solver* s : ss) s->set_deferred(false);
    }
  } undefer{ss};
  std::vector<bool> live(n, true);
  auto fail = [&](size_t i, int st, const char* what) {
    live[i] = false;
    status[i] = st;
    err[i] = what;
  };
  auto guard = [&](size_t i, auto&& f) {
    try {
      f();
    } catch (const Error& e) {
      fail(i, e.status, e.what());
    } catch (const std::exception& e) {
      fail(i, kEDEVICE, e.what());
    }
  };
  for (size_t i = 0; i < n; ++i) {
    ss[i]->set_deferred(true);
    guard(i, [&] { ss[i]->step_begin(); });
  }
  for (;;) {
    // the pending SVD calls: recycled ones (and solves that cannot share a
    // launch) go out alone, fresh ones in grouped stages
    std::vector<size_t> fresh;
    for (size_t i = 0; i < n; ++i) {
      if (!live[i] || !ss[i]->svd_pending()) continue;
      if (ss[i]->pending_fresh() && ss[i]->group_kind() >= 0)
        fresh.push_back(i);
      else
        guard(i, [&] { ss[i]->launch_pending(); });
    }
    for (size_t i : fresh) guard(i, [&] { ss[i]->fresh_group_begin(); });
    int64_t used = 0;                          // task-table entries this loop
    for (int t = 0; !fresh.empty(); ++t) {
      std::vector<SpmmTask> tasks[2];          // by value type: FP64, FP32
      std::vector<size_t> part[2];
      std::vector<size_t> next;
      for (size_t i : fresh) {
        if (!live[i]) continue;
        std::vector<SpmmTask> sink;
        bool more = false;
        guard(i, [&] { more = ss[i]->fresh_group_stage(t, &sink); });
        if (!live[i]) continue;
        if (!more) {
          guard(i, [&] { ss[i]->fresh_group_end(); });
          continue;
        }
        next.push_back(i);
        if (sink.empty()) continue;
        const int kind = ss[i]->group_kind();
        tasks[kind].insert(tasks[kind].end(), sink.begin(), sink.end());
        part[kind].push_back(i);
      }
      for (int kind = 0; kind < 2; ++kind) {
        if (tasks[kind].empty()) continue;
        // the group stream waits for the participants' stage work
        for (size_t j = 0; j < part[kind].size(); ++j) {
          hipEvent_t e = event_at(res, j);
          MC_HIP(hipEventRecord(e, ss[part[kind][j]]->stream()));
          MC_HIP(hipStreamWaitEvent(res.st, e, 0));
        }
        const int64_t need = (int64_t)tasks[kind].size();
        MC_REQUIRE(used + need <= res.cap, kEINVAL, "grouped SpMM: task table full");
        if (kind == 0)
          launch_spmm_group<double, double, double, double>(
              tasks[kind], res.staging + used, res.table + used, res.cap - used, res.st);
        else
          launch_spmm_group<float, float, float, float>(
              tasks[kind], res.staging + used, res.table + used, res.cap - used, res.st);
        used += need;
        MC_HIP(hipEventRecord(res.done, res.st));
        for (size_t i : part[kind]) MC_HIP(hipStreamWaitEvent(ss[i]->stream(), res.done, 0));
      }
      fresh.swap(next);
    }
    // every live solve now has work in flight (or has finished its step):
    // wait for each and let it decide its next move
    bool pending = false;
    for (size_t i = 0; i < n; ++i) {
      if (!live[i]) continue;
      guard(i, [&] { ss[i]->step_poll(true); });
      if (live[i] && ss[i]->step_busy()) pending = true;
    }
    if (!pending) break;
    // solves in their SDDMM phase are polled again on the next pass; the
    // staging entries were all consumed by the waits above
  }
}

}  // namespace mcsvt
