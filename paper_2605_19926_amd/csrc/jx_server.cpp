// jx_server.cpp -- serving form: a request loop that keeps many clients' env
// batches resident on one device and coalesces their step requests into shared
// persistent launches (continuous batching).
//
// Threads:
//   caller threads  jx_server_open / submit / wait / close (any number); open
//                   generates the client's layouts on the caller's thread
//   admitter        admits queued clients in FIFO order as the HBM budget
//                   allows: upload of the state image and the episode-0 reset
//   scheduler       packs every ready request (its client has no step in
//                   flight, its results fit the staging buffers) into one
//                   launch on the next free stream.  A launch's descriptors,
//                   work items and actions sit in one range of the pinned
//                   host arena, copied to the same range of that stream's
//                   device staging buffer, and the kernel writes the results
//                   of host-result clients straight into the pinned range, so
//                   a launch is one H2D copy, the serving kernel and an
//                   event, whatever the number of clients in it; the HIP calls
//                   are made without the server lock
//   completion      polls the in-flight launches and retires each as it
//                   completes (any stream order), stamping its requests
// A caller's wait copies a request's results out of the staging arena and
// releases its range.  A request that arrives while launches are in flight
// joins the next launch, which can start on another stream before the earlier
// ones finish.
#include <hip/hip_runtime_api.h>
#include <sys/prctl.h>

#include <algorithm>
#include <cstdlib>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "jx.h"
#include "jx_common.h"
#include "jx_internal.h"

using namespace jx;

namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

int64_t align256(int64_t v) { return (v + 255) / 256 * 256; }

// First-fit allocator over one device arena with coalescing of free ranges.
class Arena {
 public:
  void init(int64_t bytes) { free_[0] = bytes; }
  int64_t alloc(int64_t bytes) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const int64_t off = it->first;
        const int64_t rest = it->second - bytes;
        free_.erase(it);
        if (rest > 0) free_[off + bytes] = rest;
        used_ += bytes;
        return off;
      }
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = align256(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  int64_t used() const { return used_; }

 private:
  std::map<int64_t, int64_t> free_;
  int64_t used_ = 0;
};

// One launch's range of the pinned host arena, shared by its requests and
// released when the last of them is collected.
struct StageRange {
  int64_t off = -1, len = 0;
  int left = 0;  // requests not yet collected
};

struct Request {
  uint64_t ticket = 0;
  int client = -1;
  std::vector<uint8_t> actions;
  // results inside the launch's pinned range (set when the request is launched)
  std::shared_ptr<StageRange> range;
  uint8_t* h_obs = nullptr;
  float* h_rew = nullptr;
  uint8_t* h_done = nullptr;
  int64_t obs_bytes = 0;
  int n = 0;
  double t_submit = 0, t_done = 0;
  int status = 0;  // 0 queued, 1 launched, 2 done, 3 failed
  int slot = -1;   // device-result clients: the ring slot its results went to
  bool dev = false;  // the client's results stay in its device ring
};

// PENDING: in the admission queue; ADMITTING: memory reserved, being
// uploaded and reset (without the server lock); ACTIVE: served.
enum ClientState { PENDING, ADMITTING, ACTIVE, CLOSED };

struct Client {
  int id = -1;
  int n = 0;
  jx_env_cfg cfg{};
  std::vector<uint64_t> seeds;
  std::string ascii;  // copy of the configuration's ASCII map, if any
  // state image (layouts generated on the host at open), uploaded on admission
  std::vector<uint8_t> img;
  std::vector<int32_t> idx;
  ClientState st = PENDING;
  bool closing = false;
  bool in_flight = false;
  // device memory: one arena range holding workspace | obs | act | rew | done
  int64_t arena_off = -1, bytes = 0;
  Layout L{};
  DevState S{};
  int64_t obs_bytes = 0;
  std::deque<std::shared_ptr<Request>> queue;
  // device-result clients: the caller's rings of `slots` steps; request k of
  // the client writes slot k mod slots (requests of one client run in order)
  uint8_t* dev_obs = nullptr;
  float* dev_rew = nullptr;
  uint8_t* dev_done = nullptr;
  int slots = 0;
  int64_t launched = 0;  // requests of this client issued so far
  bool failed = false;   // a launch holding this client failed: its state is unknown
};

struct Launch {
  int stream = 0;
  hipEvent_t ev = nullptr;
  std::vector<std::shared_ptr<Request>> reqs;
};

struct StreamSlot {
  hipStream_t s = nullptr;
  bool busy = false;
  uint8_t* d_stage = nullptr;       // launch staging: descriptors, items, actions, results
  uint32_t* d_counters = nullptr;   // queue counter sets of this stream
  uint32_t seq = 0;                  // serving launches issued on this stream
  hipEvent_t ev = nullptr;
};

constexpr int kMaxClientsPerLaunch = 1024;
constexpr int kMaxItemsPerLaunch = 1 << 18;
// Device staging per stream slot (outside the HBM budget, which covers the
// clients' resident state).
constexpr int64_t kSlotStageBytes = int64_t(128) << 20;

}  // namespace

// Pinned staging arena for requests' actions and results: allocated once, so
// that no pinned allocation or free (which can synchronise the device) happens
// while serving.
constexpr int64_t kStagingMaxBytes = int64_t(2) << 30;

struct jx_server {
  int device = 0;
  uint8_t* host_base = nullptr;  // pinned staging arena
  uint8_t* host_dev = nullptr;   // its device view: the serving kernels write host clients' results there
  int64_t host_bytes = 0;
  Arena host;
  int mode = JX_SERVE_COALESCE;
  int max_batch_envs = 0;
  int n_cu = 1;
  int64_t budget = 0;
  uint8_t* arena_base = nullptr;
  Arena arena;
  std::vector<StreamSlot> streams;
  hipStream_t admin = nullptr;
  int next_stream = 0;

  std::mutex mu;
  std::condition_variable cv_sched;   // scheduler: new work / stream freed / stop
  // Bumped, with mu held, at every change that can give the scheduler work; an
  // idle scheduler polls it before sleeping on cv_sched (see sched_idle).
  std::atomic<uint64_t> sched_epoch{0};
  // Launches appended to `inflight` so far (bumped under mu): the completion
  // thread polls its snapshot of the in-flight events without the lock until
  // this moves or one of them completes.
  std::atomic<uint64_t> launches_pushed{0};
  std::condition_variable cv_admit;   // admitter: a client queued / memory freed / stop
  std::condition_variable cv_done;    // waiters: a request completed
  std::condition_variable cv_comp;    // completion thread: a launch was issued
  std::map<int, std::unique_ptr<Client>> clients;
  std::deque<int> pending;            // admission FIFO
  std::map<uint64_t, std::shared_ptr<Request>> requests;
  std::deque<Launch> inflight;
  std::deque<std::pair<uint64_t, int>> completed;  // (ticket, client) in completion order
  uint64_t next_ticket = 1;
  int next_client = 0;
  bool stop = false;
  // testing hook (JX_SERVER_FAIL_LAUNCH): the launch with this index is treated
  // as failed before any HIP call is made for it; -1 = none
  int64_t fail_launch = -1;
  int64_t launches_issued = 0;
  std::string fatal;
  jx_server_stats stats{};
  std::thread sched, comp, admitter;
};

// Tells the scheduler there may be new work; call with s->mu held.
void wake_sched(jx_server* s) {
  s->sched_epoch.fetch_add(1, std::memory_order_release);
  s->cv_sched.notify_one();
}

namespace {

// Device bytes of a client (its workspace: state and maps); its frames,
// actions, rewards and dones live in the launch staging.
int64_t client_bytes(int n, const jx_env_cfg& cfg, Layout* L, int64_t* obs_bytes) {
  *L = make_layout(n, 1, (int64_t)n * map_bytes_of(cfg.side));
  *obs_bytes = (int64_t)n * cfg.obs_h * cfg.obs_w * 3;
  return align256(L->total);
}

// Offsets (identical in the device staging and the pinned range) of one
// launch: descriptors | work items | actions | results, each 256-byte aligned.
struct LaunchPlan {
  int64_t states = 0, ios = 0, items = 0, acts = 0, results = 0, total = 0;
  std::vector<int64_t> act, obs, rew, done;
};

LaunchPlan plan_launch(const std::vector<Client*>& batch) {
  LaunchPlan P;
  int64_t o = 0, n_items = 0;
  for (Client* c : batch) n_items += c->n;
  P.states = o;
  o += align256((int64_t)sizeof(DevState) * (int64_t)batch.size());
  P.ios = o;
  o += align256((int64_t)sizeof(DevIo) * (int64_t)batch.size());
  P.items = o;
  o += align256((int64_t)sizeof(ServeItem) * n_items);
  P.acts = o;
  for (Client* c : batch) {
    P.act.push_back(o);
    o += align256(c->n);
  }
  P.results = o;
  for (Client* c : batch) {
    if (c->dev_obs) {  // results go to the client's device ring: no staging
      P.obs.push_back(-1);
      P.rew.push_back(-1);
      P.done.push_back(-1);
      continue;
    }
    P.obs.push_back(o);
    o += align256(c->obs_bytes);
    P.rew.push_back(o);
    o += align256(4 * (int64_t)c->n);
    P.done.push_back(o);
    o += align256(c->n);
  }
  P.total = o;
  return P;
}

// Upper bound of what one more client adds to a launch's staging.
int64_t stage_bound(const Client* c) {
  const int64_t results = c->dev_obs ? 0 : align256(c->obs_bytes) + align256(4 * (int64_t)c->n) + align256(c->n);
  return align256(sizeof(DevState)) + align256(sizeof(DevIo)) + align256(8 * (int64_t)c->n) + align256(c->n) +
         results;
}

// Uploads the client's image (built at open) and runs the episode-0 reset.
// Called without the server lock; the client's arena range is already reserved.
jx_status activate(jx_server* s, Client* c) {
  const Layout L = c->L;
  uint8_t* ws = s->arena_base + c->arena_off;
  c->L = L;
  c->S = bind_state(ws, L, c->n);
  set_uniform(&c->S, &c->cfg, 1, c->idx);
  if (hipMemcpyAsync(ws, c->img.data(), c->img.size(), hipMemcpyHostToDevice, s->admin) != hipSuccess)
    return set_error(JX_EDEVICE, "client upload failed");
  DevIo io{};
  io.mode = MODE_RESET;
  int rc = launch_batch(c->S, io, nullptr, 0, LaunchCfg{0, 1, 1, 0}, c->cfg.side, s->n_cu, 0, s->admin);
  if (rc) return set_error(JX_EDEVICE, std::string("client reset: ") + kernel_error_string(rc));
  if (hipStreamSynchronize(s->admin) != hipSuccess) return set_error(JX_EDEVICE, "client reset sync failed");
  std::vector<uint8_t>().swap(c->img);
  return JX_OK;
}

void free_client_memory(jx_server* s, Client* c) {
  if (c->arena_off >= 0) s->arena.release(c->arena_off, c->bytes);
  c->arena_off = -1;
}

// A request is collected: its launch's pinned range goes back to the arena
// with the last of the launch's requests (lock held).
void release_staging(jx_server* s, Request* r) {
  if (r->range && --r->range->left == 0) s->host.release(r->range->off, r->range->len);
  r->range.reset();
  r->h_obs = r->h_done = nullptr;
  r->h_rew = nullptr;
}

// Admitter thread: admits queued clients in FIFO order while the budget
// allows, uploading and resetting each without the server lock, so the
// scheduler keeps issuing launches meanwhile.
void admitter_main(jx_server* s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    if (s->pending.empty()) {
      s->cv_admit.wait(lk);
      continue;
    }
    Client* c = s->clients[s->pending.front()].get();
    const int64_t off = s->arena.alloc(c->bytes);
    if (off < 0) {
      s->cv_admit.wait(lk);  // woken when a client's memory is released
      continue;
    }
    c->arena_off = off;
    c->st = ADMITTING;
    s->pending.pop_front();
    lk.unlock();
    jx_status st = activate(s, c);
    lk.lock();
    s->stats.clients_pending -= 1;
    if (st != JX_OK) {
      s->fatal = "admission failed: " + std::string(jx_last_error());
      c->st = CLOSED;
      for (auto& r : c->queue) {
        r->status = 3;
        s->completed.emplace_back(r->ticket, r->client);
      }
      c->queue.clear();
      free_client_memory(s, c);
      s->cv_done.notify_all();
      continue;
    }
    c->st = ACTIVE;
    s->stats.clients_active += 1;
    wake_sched(s);
  }
}

void reap_closed(jx_server* s) {
  bool freed = false;
  for (auto& kv : s->clients) {
    Client* c = kv.second.get();
    if (c->closing && c->st == ACTIVE && !c->in_flight && c->queue.empty()) {
      free_client_memory(s, c);
      c->st = CLOSED;
      s->stats.clients_active -= 1;
      freed = true;
    }
  }
  if (freed) {
    s->cv_admit.notify_one();
    for (auto it = s->clients.begin(); it != s->clients.end();) {
      if (it->second->st == CLOSED && it->second->queue.empty()) it = s->clients.erase(it);
      else ++it;
    }
  }
}

// Builds and issues one launch on stream slot k from the batch, whose pinned
// range (at host_off, plan P) is already reserved.  Called with the lock held;
// the HIP calls run without it (the slot is marked busy and the clients in
// flight first, so nothing else touches them meanwhile).
void issue(jx_server* s, std::unique_lock<std::mutex>& lk, int k, const std::vector<Client*>& batch,
           const LaunchPlan& P, int64_t host_off) {
  StreamSlot& ss = s->streams[k];
  Launch L;
  L.stream = k;
  L.ev = ss.ev;
  uint8_t* h = s->host_base + host_off;
  uint8_t* hd = s->host_dev + host_off;
  uint8_t* d = ss.d_stage;
  auto range = std::make_shared<StageRange>();
  range->off = host_off;
  range->len = P.total;
  range->left = (int)batch.size();
  std::vector<DevState> states(batch.size());
  std::vector<DevIo> dev_io(batch.size());  // I/O of each client, device addresses
  int n_items = 0;
  for (size_t j = 0; j < batch.size(); ++j) {
    Client* c = batch[j];
    std::shared_ptr<Request> r = c->queue.front();
    c->queue.pop_front();
    c->in_flight = true;
    r->status = 1;
    r->n = c->n;
    r->obs_bytes = c->obs_bytes;
    r->range = range;
    DevIo io{};
    io.mode = MODE_STEP;
    io.act = d + P.act[j];
    if (c->dev_obs) {
      // the client's k-th request writes ring slot k mod slots
      r->slot = (int)(c->launched % c->slots);
      io.obs = c->dev_obs + (int64_t)r->slot * c->obs_bytes;
      io.rew = c->dev_rew + (int64_t)r->slot * c->n;
      io.done = c->dev_done + (int64_t)r->slot * c->n;
    } else {
      r->h_obs = h + P.obs[j];
      r->h_rew = (float*)(h + P.rew[j]);
      r->h_done = h + P.done[j];
      // the kernel writes the results straight into the pinned range (through
      // its device view), where jx_server_wait copies them out: no device
      // staging and no copy back (measured: the median at 2000 req/s fell
      // from 0.064 to 0.046 ms and at 8000 req/s from 0.091 to 0.066 ms,
      // with the saturated rate unchanged)
      io.obs = hd + P.obs[j];
      io.rew = reinterpret_cast<float*>(hd + P.rew[j]);
      io.done = hd + P.done[j];
    }
    c->launched += 1;
    dev_io[j] = io;
    L.reqs.push_back(r);
    states[j] = c->S;
    n_items += c->n;
  }
  ss.busy = true;
  const bool plain = s->mode == JX_SERVE_PLAIN;
  const int side = batch[0]->cfg.side;
  const bool inject = s->launches_issued++ == s->fail_launch;
  lk.unlock();
  TraceRange trace(plain ? "jx_server launch (plain)" : "jx_server launch (coalesced)");
  // descriptors, work items and actions into the pinned range
  DevIo* ios = reinterpret_cast<DevIo*>(h + P.ios);
  ServeItem* items = reinterpret_cast<ServeItem*>(h + P.items);
  int it = 0;
  for (size_t j = 0; j < batch.size(); ++j) {
    Request* r = L.reqs[j].get();
    std::memcpy(h + P.act[j], r->actions.data(), (size_t)r->n);
    ios[j] = dev_io[j];
    if (!plain)
      for (int e = 0; e < r->n; ++e) items[it++] = ServeItem{(int32_t)j, e};
  }
  hipStream_t st = ss.s;
  // an injected failure makes no HIP call for this launch
  bool ok = false;
  bool ran = false;  // the serving kernel was enqueued: it used counter set seq
  if (!inject) {
    if (plain) {
      // the per-request kernel takes its state and I/O by value: copy the actions only
      ok = hipMemcpyAsync(d + P.acts, h + P.acts, (size_t)(P.results - P.acts), hipMemcpyHostToDevice, st) ==
           hipSuccess;
      ok = ok && launch_batch(states[0], ios[0], nullptr, 0, LaunchCfg{0, 1, 1, 0}, side, s->n_cu, 0, st) == 0;
    } else {
      std::memcpy(h + P.states, states.data(), sizeof(DevState) * states.size());
      ok = hipMemcpyAsync(d, h, (size_t)P.results, hipMemcpyHostToDevice, st) == hipSuccess;
      const int wpb = 2;
      int groups = std::min((n_items + wpb - 1) / wpb, s->n_cu * 4);
      groups = std::max(groups, 1);
      ran = ok && launch_serve(reinterpret_cast<DevState*>(d + P.states), reinterpret_cast<DevIo*>(d + P.ios),
                               reinterpret_cast<ServeItem*>(d + P.items), n_items, ss.d_counters, ss.seq, wpb,
                               groups, st) == 0;
      ok = ran;
    }
    ok = ok && hipEventRecord(ss.ev, st) == hipSuccess;
    // a launch that failed part-way may still have work queued on the stream:
    // drain it before the slot and the staging range can be reused
    if (!ok) hipStreamSynchronize(st);
  }
  lk.lock();
  if (ran) ss.seq += 1;
  if (!ok) {
    // the launch's requests fail and its clients' state is unknown: those
    // clients fail (their queued requests too), every other client goes on
    for (auto& r : L.reqs) {
      r->status = 3;
      s->completed.emplace_back(r->ticket, r->client);
    }
    for (Client* c : batch) {
      c->in_flight = false;
      c->failed = true;
      for (auto& r : c->queue) {
        r->status = 3;
        s->completed.emplace_back(r->ticket, r->client);
      }
      c->queue.clear();
    }
    s->stats.failed_launches += 1;
    ss.busy = false;
    s->cv_done.notify_all();
    wake_sched(s);
    return;
  }
  s->stats.launches += 1;
  s->stats.env_steps += n_items;
  s->inflight.push_back(std::move(L));
  s->launches_pushed.fetch_add(1, std::memory_order_release);
  s->cv_comp.notify_one();
}

// An idle scheduler (with poll set) polls the wake counter for up to
// kSchedSpin without the lock, so that a request arriving then is picked up
// within about a microsecond instead of after a thread wake-up (about 10 us
// here), and then sleeps until the counter moves.  Every bump happens with the
// lock held, and the counter is read under it before the sleep, so no wake-up
// is lost.  The polling keeps one host core busy while requests arrive less
// than kSchedSpin apart (at 2000 requests/s, 86% of Poisson gaps are shorter
// than 1 ms).
constexpr auto kSchedSpin = std::chrono::microseconds(1000);
void sched_idle(jx_server* s, std::unique_lock<std::mutex>& lk, bool poll) {
  const uint64_t seen = s->sched_epoch.load(std::memory_order_acquire);
  lk.unlock();
  const auto until = std::chrono::steady_clock::now() + (poll ? kSchedSpin : std::chrono::microseconds(0));
  while (s->sched_epoch.load(std::memory_order_acquire) == seen && std::chrono::steady_clock::now() < until)
    std::this_thread::yield();
  lk.lock();
  s->cv_sched.wait(lk, [&] { return s->stop || s->sched_epoch.load(std::memory_order_acquire) != seen; });
}

void scheduler_main(jx_server* s) {
  hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    reap_closed(s);
    // ready clients, oldest request first
    std::vector<Client*> ready;
    for (auto& kv : s->clients) {
      Client* c = kv.second.get();
      if (c->st == ACTIVE && !c->in_flight && !c->queue.empty()) ready.push_back(c);
    }
    int k = -1;
    for (int j = 0; j < (int)s->streams.size(); ++j) {
      int cand = (s->next_stream + j) % (int)s->streams.size();
      if (!s->streams[cand].busy) {
        k = cand;
        break;
      }
    }
    if (ready.empty() || k < 0) {
      // poll only when the device is idle too: under load a completion or a
      // submit wakes the scheduler soon anyway, and polling threads then
      // contend for the lock and the host cores (measured: a p99 of several
      // milliseconds at 64,000 requests/s against 0.3-1.2 ms without)
      sched_idle(s, lk, ready.empty() && s->inflight.empty());
      continue;
    }
    std::sort(ready.begin(), ready.end(), [](Client* a, Client* b) {
      return a->queue.front()->ticket < b->queue.front()->ticket;
    });
    std::vector<Client*> batch;
    int envs = 0;
    int64_t bound = 0;
    for (Client* c : ready) {
      if (s->mode == JX_SERVE_PLAIN && !batch.empty()) break;
      if (!batch.empty() && s->max_batch_envs > 0 && envs + c->n > s->max_batch_envs) continue;
      if ((int)batch.size() >= kMaxClientsPerLaunch || envs + c->n > kMaxItemsPerLaunch) break;
      if (bound + stage_bound(c) > kSlotStageBytes) continue;
      batch.push_back(c);
      envs += c->n;
      bound += stage_bound(c);
    }
    // the launch's results must fit the pinned arena; else it shrinks, and a
    // single request that does not fit waits for callers to collect results
    LaunchPlan P;
    int64_t off = -1;
    while (!batch.empty()) {
      P = plan_launch(batch);
      off = s->host.alloc(P.total);
      if (off >= 0) break;
      batch.resize(batch.size() / 2);
    }
    if (batch.empty()) {
      sched_idle(s, lk, false);
      continue;
    }
    s->next_stream = (k + 1) % (int)s->streams.size();
    issue(s, lk, k, batch, P, off);
  }
}

// Retires launches in the order they complete (any stream), stamping their
// requests' completion time.  Results are already in the requests' pinned
// buffers; the caller's wait copies them out, so nothing here delays the next
// launch's timestamp.
void completion_main(jx_server* s) {
  hipSetDevice(s->device);
  // This thread polls at a granularity of a few microseconds.  Linux's default
  // timer slack (50 us) would stretch every short sleep below to about 60 us
  // and add that to the latency of each request, so it is cut to 1 us for this
  // thread only.
  prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<hipEvent_t> evs;
  std::vector<hipError_t> res;
  while (true) {
    while (s->inflight.empty() && !s->stop) s->cv_comp.wait(lk);
    if (s->inflight.empty() && s->stop) return;
    // The events are queried without the lock, which submits, waits and the
    // scheduler need far more often than this thread (taking it at every poll
    // pushed the 64,000 requests/s p99 from 0.2 to 1-2.5 ms).  Only this thread
    // removes launches, and a stream's event is not recorded again before its
    // launch is retired here, so the first evs.size() launches are the same
    // ones when the lock is taken back (the scheduler only appends).
    evs.clear();
    for (const Launch& L : s->inflight) evs.push_back(L.ev);
    const uint64_t pushed = s->launches_pushed.load(std::memory_order_acquire);
    lk.unlock();
    res.resize(evs.size());
    // poll the snapshot every 2 us (launches take tens of microseconds and up)
    // without touching the lock, until a launch completes or a new one starts
    bool any = false;
    while (true) {
      for (size_t i = 0; i < evs.size(); ++i) {
        res[i] = hipEventQuery(evs[i]);
        any = any || res[i] != hipErrorNotReady;
      }
      if (any || s->launches_pushed.load(std::memory_order_acquire) != pushed) break;
      std::this_thread::sleep_for(std::chrono::microseconds(2));
    }
    if (!any) {
      lk.lock();
      continue;
    }
    const double t = now_s();
    lk.lock();
    auto it = s->inflight.begin();
    for (size_t i = 0; i < res.size(); ++i) {
      const hipError_t e = res[i];
      if (e == hipErrorNotReady) {
        ++it;
        continue;
      }
      for (auto& r : it->reqs) {
        r->status = (e == hipSuccess) ? 2 : 3;
        r->t_done = t;
        s->completed.emplace_back(r->ticket, r->client);
        auto c = s->clients.find(r->client);
        if (c != s->clients.end()) c->second->in_flight = false;
        s->stats.requests += 1;
      }
      if (e != hipSuccess) s->fatal = std::string("device error: ") + hipGetErrorString(e);
      s->streams[it->stream].busy = false;
      it = s->inflight.erase(it);
      // requests collected through jx_server_wait leave stale entries in the
      // completion queue: prune them once they dominate (amortised O(1))
      if (s->completed.size() > 2 * s->requests.size() + 1024) {
        std::deque<std::pair<uint64_t, int>> keep;
        for (auto& tc : s->completed)
          if (s->requests.count(tc.first)) keep.push_back(tc);
        s->completed.swap(keep);
      }
    }
    s->cv_done.notify_all();
    wake_sched(s);
  }
}

}  // namespace

#define SRV_CHK(expr, msg)                          \
  do {                                              \
    if ((expr) != hipSuccess) {                     \
      jx_server_destroy(s);                         \
      return set_error(JX_EDEVICE, msg);            \
    }                                               \
  } while (0)

extern "C" {

jx_status jx_server_create(jx_server** out, int32_t device, size_t hbm_budget_bytes, int32_t n_streams,
                           int32_t mode, int32_t max_batch_envs) {
  if (!out) return set_error(JX_EINVAL, "out is null");
  *out = nullptr;
  if (n_streams < 1 || n_streams > 8) return set_error(JX_EINVAL, "n_streams must be in 1..8");
  if (mode != JX_SERVE_COALESCE && mode != JX_SERVE_PLAIN) return set_error(JX_EINVAL, "bad mode");
  if (hbm_budget_bytes < 4096) return set_error(JX_EINVAL, "budget too small");
  if (max_batch_envs < 0) return set_error(JX_EINVAL, "max_batch_envs < 0");
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 || device >= n_dev)
    return set_error(JX_EINVAL, "bad device index");
  hipSetDevice(device);
  jx_server* s = new jx_server();
  s->device = device;
  s->mode = mode;
  s->max_batch_envs = max_batch_envs;
  s->budget = (int64_t)hbm_budget_bytes;
  // testing hook: JX_SERVER_FAIL_LAUNCH=k treats this server's k-th launch
  // (0-based) as failed without making any HIP call for it
  if (const char* f = std::getenv("JX_SERVER_FAIL_LAUNCH")) {
    char* end = nullptr;
    const long long k = std::strtoll(f, &end, 10);
    if (end != f && *end == '\0' && k >= 0) s->fail_launch = (int64_t)k;
  }
  hipDeviceProp_t p;
  SRV_CHK(hipGetDeviceProperties(&p, device), "device properties");
  s->n_cu = std::max(1, p.multiProcessorCount);
  SRV_CHK(hipMalloc((void**)&s->arena_base, hbm_budget_bytes), "HBM budget allocation failed");
  s->arena.init((int64_t)hbm_budget_bytes);
  s->host_bytes = std::min<int64_t>((int64_t)hbm_budget_bytes, kStagingMaxBytes);
  SRV_CHK(hipHostMalloc((void**)&s->host_base, (size_t)s->host_bytes), "pinned staging allocation failed");
  SRV_CHK(hipHostGetDevicePointer((void**)&s->host_dev, s->host_base, 0), "pinned staging device view failed");
  s->host.init(s->host_bytes);
  SRV_CHK(hipStreamCreateWithFlags(&s->admin, hipStreamNonBlocking), "stream");
  const int ns = (mode == JX_SERVE_PLAIN) ? 1 : n_streams;
  s->streams.resize(ns);
  for (auto& ss : s->streams) {
    SRV_CHK(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking), "stream");
    SRV_CHK(hipEventCreateWithFlags(&ss.ev, hipEventDisableTiming), "event");
    SRV_CHK(hipMalloc((void**)&ss.d_stage, (size_t)kSlotStageBytes), "staging allocation failed");
    SRV_CHK(hipMalloc((void**)&ss.d_counters, 4 * kQueueWords), "alloc");
    SRV_CHK(hipMemset(ss.d_counters, 0, 4 * kQueueWords), "memset");
  }
  SRV_CHK(hipDeviceSynchronize(), "sync");
  s->sched = std::thread(scheduler_main, s);
  s->comp = std::thread(completion_main, s);
  s->admitter = std::thread(admitter_main, s);
  *out = s;
  return JX_OK;
}

void jx_server_destroy(jx_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
    s->sched_epoch.fetch_add(1, std::memory_order_release);
  }
  s->cv_sched.notify_all();
  s->cv_comp.notify_all();
  s->cv_admit.notify_all();
  if (s->sched.joinable()) s->sched.join();
  if (s->comp.joinable()) s->comp.join();
  if (s->admitter.joinable()) s->admitter.join();
  hipSetDevice(s->device);
  hipDeviceSynchronize();
  for (auto& kv : s->clients) free_client_memory(s, kv.second.get());
  if (s->host_base) hipHostFree(s->host_base);
  for (auto& ss : s->streams) {
    if (ss.s) hipStreamDestroy(ss.s);
    if (ss.ev) hipEventDestroy(ss.ev);
    if (ss.d_stage) hipFree(ss.d_stage);
    if (ss.d_counters) hipFree(ss.d_counters);
  }
  if (s->admin) hipStreamDestroy(s->admin);
  if (s->arena_base) hipFree(s->arena_base);
  delete s;
}

}  // extern "C"

namespace {

// Opens a client; dev_obs != nullptr: its results go to the caller's device
// rings of `slots` steps.
jx_status open_client(jx_server* s, int32_t n_envs, const uint64_t* seeds, const jx_env_cfg* cfg,
                      uint8_t* dev_obs, float* dev_rew, uint8_t* dev_done, int32_t slots, int32_t* client) {
  if (!s || !seeds || !cfg || !client) return set_error(JX_EINVAL, "null argument");
  if (n_envs < 1 || n_envs > kMaxItemsPerLaunch) return set_error(JX_EINVAL, "n_envs out of range");
  std::string why;
  if (!validate_cfg(*cfg, &why)) return set_error(JX_EINVAL, why);
  if (obs_fmt_of(*cfg) != 0) return set_error(JX_EINVAL, "serving takes the default frame format (NHWC, U8) only");
  auto c = std::make_unique<Client>();
  c->n = n_envs;
  c->cfg = *cfg;
  if (cfg->ascii_map) {  // the caller's text need not outlive this call
    c->ascii = cfg->ascii_map;
    c->cfg.ascii_map = c->ascii.c_str();
  }
  c->seeds.assign(seeds, seeds + n_envs);
  c->dev_obs = dev_obs;
  c->dev_rew = dev_rew;
  c->dev_done = dev_done;
  c->slots = dev_obs ? slots : 0;
  c->bytes = client_bytes(n_envs, *cfg, &c->L, &c->obs_bytes);
  if (c->bytes > s->budget) return set_error(JX_ENOMEM, "client exceeds the HBM budget on its own");
  {
    const int64_t one = plan_launch(std::vector<Client*>{c.get()}).total;
    if (one > kSlotStageBytes || one > s->host_bytes)
      return set_error(JX_ENOMEM, "one step of this client exceeds the launch staging (" +
                                      std::to_string(std::min(kSlotStageBytes, s->host_bytes)) + " bytes)");
  }
  {
    // layouts are generated here, on the caller's thread, so that admission
    // only uploads and resets
    Layout L;
    std::vector<int64_t> oo;
    jx_status st = build_image(n_envs, c->seeds.data(), &c->cfg, 1, nullptr, &c->img, &L, &oo, &c->idx);
    if (st) return st;
    if (L.total != c->L.total || (int64_t)c->img.size() > L.total)
      return set_error(JX_ESTATE, "client image does not match its reserved layout");
    c->L = L;
  }
  std::unique_lock<std::mutex> lk(s->mu);
  const int id = s->next_client++;
  c->id = id;
  Client* cp = c.get();
  s->clients[id] = std::move(c);
  *client = id;
  const bool fifo_empty = s->pending.empty();
  const int64_t off = fifo_empty ? s->arena.alloc(cp->bytes) : -1;
  if (off < 0) {
    s->pending.push_back(id);
    s->stats.clients_pending += 1;
    s->stats.admission_waits += 1;
    s->cv_admit.notify_one();
    return JX_EBUSY;
  }
  cp->arena_off = off;
  cp->st = ADMITTING;
  lk.unlock();
  jx_status st = activate(s, cp);
  lk.lock();
  if (st != JX_OK) {
    free_client_memory(s, cp);
    for (auto& r : cp->queue) {
      r->status = 3;
      s->completed.emplace_back(r->ticket, r->client);
    }
    s->clients.erase(id);
    s->cv_done.notify_all();
    return st;
  }
  cp->st = ACTIVE;
  s->stats.clients_active += 1;
  wake_sched(s);
  return JX_OK;
}

}  // namespace

extern "C" {

jx_status jx_server_open(jx_server* s, int32_t n_envs, const uint64_t* seeds, const jx_env_cfg* cfg,
                         int32_t* client) {
  return open_client(s, n_envs, seeds, cfg, nullptr, nullptr, nullptr, 0, client);
}

jx_status jx_server_open_dev(jx_server* s, int32_t n_envs, const uint64_t* seeds, const jx_env_cfg* cfg,
                             uint8_t* obs_dev, float* reward_dev, uint8_t* done_dev, int32_t slots,
                             int32_t* client) {
  if (!obs_dev || !reward_dev || !done_dev) return set_error(JX_EINVAL, "device result rings must not be null");
  if (slots < 1) return set_error(JX_EINVAL, "slots must be >= 1");
  if (((uintptr_t)obs_dev & 3) || ((uintptr_t)reward_dev & 3))
    return set_error(JX_EINVAL, "obs and reward rings must be 4-byte aligned");
  return open_client(s, n_envs, seeds, cfg, obs_dev, reward_dev, done_dev, slots, client);
}

jx_status jx_server_submit(jx_server* s, int32_t client, const uint8_t* actions, uint64_t* ticket) {
  if (!s || !actions || !ticket) return set_error(JX_EINVAL, "null argument");
  auto r = std::make_shared<Request>();
  std::unique_lock<std::mutex> lk(s->mu);
  if (!s->fatal.empty()) return set_error(JX_EDEVICE, s->fatal);
  auto it = s->clients.find(client);
  if (it == s->clients.end() || it->second->closing || it->second->st == CLOSED)
    return set_error(JX_EINVAL, "unknown or closed client");
  Client* c = it->second.get();
  if (c->failed) return set_error(JX_EDEVICE, "client failed: a launch holding one of its steps failed");
  r->ticket = s->next_ticket++;
  r->dev = c->dev_obs != nullptr;
  r->client = client;
  r->actions.assign(actions, actions + c->n);
  r->t_submit = now_s();
  c->queue.push_back(r);
  s->requests[r->ticket] = r;
  *ticket = r->ticket;
  wake_sched(s);
  return JX_OK;
}

jx_status jx_server_wait(jx_server* s, uint64_t ticket, double timeout_s, uint8_t* obs, float* rew,
                         uint8_t* done, double* latency) {
  if (!s) return set_error(JX_EINVAL, "null server");
  std::shared_ptr<Request> r;
  std::string fatal;
  {
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->requests.find(ticket);
    if (it == s->requests.end()) return set_error(JX_EINVAL, "unknown ticket");
    r = it->second;
    if (r->dev && (obs || rew || done))
      return set_error(JX_EINVAL, "the client keeps its results in its device rings: pass no host buffers");
    auto finished = [&] { return r->status >= 2; };
    if (timeout_s < 0) {
      s->cv_done.wait(lk, finished);
    } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
      return JX_EBUSY;
    }
    s->requests.erase(ticket);
    fatal = s->fatal;
  }
  // the request is ours alone now: copy without the lock, then give its
  // staging range back
  const bool failed = r->status == 3;
  if (!failed) {
    if (obs) std::memcpy(obs, r->h_obs, (size_t)r->obs_bytes);
    if (rew) std::memcpy(rew, r->h_rew, 4 * (size_t)r->n);
    if (done) std::memcpy(done, r->h_done, (size_t)r->n);
    if (latency) *latency = r->t_done - r->t_submit;
  }
  {
    std::lock_guard<std::mutex> g(s->mu);
    release_staging(s, r.get());
    s->sched_epoch.fetch_add(1, std::memory_order_release);
  }
  s->cv_sched.notify_one();
  if (failed)
    return set_error(JX_EDEVICE, fatal.empty() ? "request failed: the launch holding it (or an earlier step of its "
                                                 "client) failed"
                                               : fatal);
  return JX_OK;
}

jx_status jx_server_wait_any(jx_server* s, double timeout_s, uint64_t* ticket, int32_t* client) {
  if (!s || !ticket) return set_error(JX_EINVAL, "null argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto next = [&] {
    // drop entries already collected through jx_server_wait
    while (!s->completed.empty() && !s->requests.count(s->completed.front().first))
      s->completed.pop_front();
    return !s->completed.empty();
  };
  if (timeout_s < 0) {
    s->cv_done.wait(lk, next);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), next)) {
    return JX_EBUSY;
  }
  *ticket = s->completed.front().first;
  if (client) *client = s->completed.front().second;
  s->completed.pop_front();
  return JX_OK;
}

jx_status jx_server_close(jx_server* s, int32_t client) {
  if (!s) return set_error(JX_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->clients.find(client);
  if (it == s->clients.end()) return set_error(JX_EINVAL, "unknown client");
  Client* c = it->second.get();
  if (c->st == PENDING && c->queue.empty()) {
    // never admitted and nothing to run: leave the admission FIFO at once
    s->pending.erase(std::remove(s->pending.begin(), s->pending.end(), client), s->pending.end());
    c->st = CLOSED;
    s->stats.clients_pending -= 1;
    s->clients.erase(it);
  } else {
    // admitted (or still to be admitted, with queued requests): released once
    // its queued requests have run
    c->closing = true;
  }
  wake_sched(s);
  return JX_OK;
}

jx_status jx_server_replay(jx_server* s, int32_t n, const double* t_arrival_s, const int32_t* client,
                           const uint8_t* const* actions_host, const uint8_t* close_after,
                           int32_t n_collectors, double timeout_s, double* latency_s, double* submitted_s,
                           double* wall_s) {
  if (!s || n < 0 || (n > 0 && (!t_arrival_s || !client || !actions_host || !latency_s)))
    return set_error(JX_EINVAL, "null argument");
  if (n_collectors < 1 || n_collectors > 64) return set_error(JX_EINVAL, "n_collectors must be in 1..64");
  if (n == 0) return JX_OK;
  // result buffers of each collector, sized for the largest client of the trace
  int64_t max_n = 1, max_obs = 1;
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (int32_t k = 0; k < n; ++k) {
      auto it = s->clients.find(client[k]);
      if (it == s->clients.end()) return set_error(JX_EINVAL, "trace names a client that is not open");
      max_n = std::max<int64_t>(max_n, it->second->n);
      max_obs = std::max<int64_t>(max_obs, it->second->obs_bytes);
    }
  }
  std::vector<uint64_t> ticket_of(n, 0);
  std::atomic<int32_t> left(n);
  std::atomic<bool> failed(false);
  std::mutex err_mu;
  std::string err;
  std::vector<std::vector<std::pair<uint64_t, double>>> got(n_collectors);
  std::atomic<double> t_last(0.0);
  const double t0 = now_s();
  const double deadline = t0 + (timeout_s > 0 ? timeout_s : 1e30);
  auto fail = [&](const std::string& m) {
    std::lock_guard<std::mutex> g(err_mu);
    if (err.empty()) err = m;
    failed = true;
  };
  auto collector = [&](int id) {
    std::vector<uint8_t> obs((size_t)max_obs);
    std::vector<float> rew((size_t)max_n);
    std::vector<uint8_t> dn((size_t)max_n);
    while (!failed && left.fetch_sub(1) > 0) {
      uint64_t tk = 0;
      int32_t cid = -1;
      jx_status st = JX_EBUSY;
      while (st == JX_EBUSY && !failed) {
        if (now_s() > deadline) {
          fail("replay did not complete within the timeout");
          return;
        }
        st = jx_server_wait_any(s, 0.05, &tk, &cid);
      }
      if (failed) return;
      if (st != JX_OK) {
        fail("wait_any failed");
        return;
      }
      bool dev = false;
      {
        // the buffers are sized for the trace's clients: a request of another
        // caller (which the replay must not run beside) would not fit
        std::lock_guard<std::mutex> g(s->mu);
        auto it = s->requests.find(tk);
        if (it == s->requests.end() || it->second->n > max_n || it->second->obs_bytes > max_obs) {
          fail("replay: a request not of the trace completed during the replay");
          return;
        }
        dev = it->second->dev;
      }
      double lat = 0.0;
      // device-result clients: the results stay in their rings, nothing to copy
      if (jx_server_wait(s, tk, -1.0, dev ? nullptr : obs.data(), dev ? nullptr : rew.data(),
                         dev ? nullptr : dn.data(), &lat) != JX_OK) {
        fail("a request failed");
        return;
      }
      got[id].emplace_back(tk, lat);
      double prev = t_last.load();
      const double t = now_s();
      while (t > prev && !t_last.compare_exchange_weak(prev, t)) {
      }
    }
  };
  std::vector<std::thread> th;
  for (int i = 0; i < n_collectors; ++i) th.emplace_back(collector, i);
  for (int32_t k = 0; k < n && !failed; ++k) {
    for (;;) {  // sleep through long gaps, spin through short ones
      const double w = t0 + t_arrival_s[k] - now_s();
      if (w <= 0) break;
      if (w > 2e-4) std::this_thread::sleep_for(std::chrono::duration<double>(w - 1e-4));
    }
    if (jx_server_submit(s, client[k], actions_host[k], &ticket_of[k]) != JX_OK) {
      fail("submit failed: " + std::string(jx_last_error()));
      break;
    }
    if (close_after && close_after[k]) jx_server_close(s, client[k]);
  }
  const double t_sub = now_s() - t0;
  for (auto& t : th) t.join();
  if (failed) return set_error(JX_EDEVICE, err);
  std::map<uint64_t, double> lat_of;
  for (auto& v : got)
    for (auto& p : v) lat_of[p.first] = p.second;
  for (int32_t k = 0; k < n; ++k) {
    auto it = lat_of.find(ticket_of[k]);
    latency_s[k] = it == lat_of.end() ? -1.0 : it->second;
  }
  if (submitted_s) *submitted_s = t_sub;
  if (wall_s) *wall_s = t_last.load() - t0;
  return JX_OK;
}

jx_status jx_server_get_stats(jx_server* s, jx_server_stats* out) {
  if (!s || !out) return set_error(JX_EINVAL, "null argument");
  std::lock_guard<std::mutex> g(s->mu);
  *out = s->stats;
  out->bytes_in_use = s->arena.used();
  return JX_OK;
}

}  // extern "C"
