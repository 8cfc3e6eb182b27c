// laim_batch.cpp -- batched plans (one persistent launch over shots of
// several codes, replayed from a HIP graph) and the continuous-batching
// server (requests resident in device memory, one round per step).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <vector>

#include "laim_internal.h"

using namespace laim;

namespace {

struct DeviceGuard {
  int prev = 0;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(dev);
  }
  ~DeviceGuard() { (void)hipSetDevice(prev); }
};

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

int cu_count(int device) {
  int cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  return cus > 0 ? cus : 256;
}

// Resolves one code + parameters into the device record of the multi-code
// kernels (shape, variant) and its LDS/block needs.
laim_status make_item(const laim_code* code, const laim_decode_params* params, BatchItemDev* it,
                      size_t* lds, int* block) {
  KParams kp;
  laim_status st = resolve_params(params, &kp);
  if (st != LAIM_OK) return st;
  if (kp.bp == 0 && kp.alpha > 1.0f) {
    set_error("the batched form runs min-sum with alpha <= 1 only");
    return LAIM_EUNSUP;
  }
  memset(it, 0, sizeof(*it));
  it->c = code->dev;
  it->kp = kp;
  const laim_resident_cfg* want = code->has_cfg[kp.bp] ? &code->cfg[kp.bp] : nullptr;
  if (!batch_variant(code->dev, kp.bp, want, code->device, kp.conflict == kConflictSequential,
                     reg_dv2_ok(kp), &it->u, &it->variant, lds, block))
    return LAIM_EUNSUP;
  it->u.rounds = kp.rounds;
  return LAIM_OK;
}

}  // namespace

// ===================================================================== plan
struct laim_batch_plan {
  int device = 0;
  hipStream_t cap = nullptr;
  void* dev_mem = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

laim_status laim_batch_plan_create(const laim_batch_item* items, int32_t nitems, laim_stream stream,
                                   laim_batch_plan** out) {
  (void)stream;
  if (!out || nitems < 1 || !items) {
    set_error("laim_batch_plan_create: bad arguments");
    return LAIM_EINVAL;
  }
  *out = nullptr;
  const int device = items[0].code ? items[0].code->device : 0;
  // Items that run resident are grouped by code and parameters: each group
  // is one persistent launch of the resident kernel specialised for that
  // code (its own launch shape, registers and LDS), walking the shots of all
  // its items from one queue.
  struct Group {
    const laim_code* code;
    KParams kp;
    ResidentShape sh;
    std::vector<GroupItemDev> items;
    int32_t total = 0;
    double cost = 0.0;
  };
  std::vector<Group> groups;
  std::vector<int> fallback_fail;  // items whose failure test runs in its own kernel
  struct StreamItem {
    int32_t index;
    KParams kp;
  };
  std::vector<StreamItem> stream_items;  // items run in the stream form
  for (int32_t i = 0; i < nitems; ++i) {
    const laim_batch_item& b = items[i];
    if (!b.code || b.nshots < 0 ||
        (b.nshots > 0 && (!b.e0 || !b.z_out || !b.s_out || !b.tclr_out))) {
      set_error("batch item %d: bad arguments", i);
      return LAIM_EINVAL;
    }
    if (b.code->device != device) {
      set_error("batch item %d: every code must live on the same device", i);
      return LAIM_EINVAL;
    }
    KParams kp = {};  // zero padding: groups compare the whole struct
    laim_status st = resolve_params(&b.params, &kp);
    if (st != LAIM_OK) return st;
    ResidentShape sh;
    const laim_resident_cfg* want = b.code->has_cfg[kp.bp] ? &b.code->cfg[kp.bp] : nullptr;
    const bool resident = !(kp.bp == 0 && kp.alpha > 1.0f) &&
                          resident_shape(b.code->dev, kp.bp, want, &sh, device,
                                         kp.conflict == kConflictSequential, reg_dv2_ok(kp));
    if (!resident) {
      // no resident variant (the shot's state exceeds the LDS, degrees
      // beyond the compiled variants, or min-sum with alpha > 1): the item
      // runs in the stream form, recorded in the same graph
      stream_items.push_back({i, kp});
      continue;
    }
    if (b.nshots == 0) continue;
    Group* g = nullptr;
    for (auto& gg : groups)
      if (gg.code == b.code && memcmp(&gg.kp, &kp, sizeof(KParams)) == 0) g = &gg;
    if (!g) {
      groups.push_back(Group{b.code, kp, sh, {}, 0, 0.0});
      g = &groups.back();
    }
    GroupItemDev it;
    it.e0 = b.e0;
    it.shot0 = b.shot0;
    it.first = g->total;
    it.nshots = b.nshots;
    it.z = b.z_out;
    it.s = b.s_out;
    it.tclr = b.tclr_out;
    it.fail = (b.fail_out && b.code->dev.kw <= 4) ? b.fail_out : nullptr;
    if (b.fail_out && !it.fail) fallback_fail.push_back(i);
    g->items.push_back(it);
    if ((int64_t)g->total + b.nshots > INT32_MAX) {
      set_error("more than 2^31 - 1 shots of one code in a plan");
      return LAIM_EINVAL;
    }
    g->total += b.nshots;
    g->cost += (double)b.nshots * kp.rounds * std::max(kp.iters, 1) * b.code->E;
  }
  // the largest groups first
  std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.cost > b.cost; });
  laim_batch_plan* plan = new (std::nothrow) laim_batch_plan();
  if (!plan) {
    set_error("out of host memory");
    return LAIM_ENOMEM;
  }
  plan->device = device;
  DeviceGuard g(device);
  std::vector<size_t> goff;
  size_t total = 0;
  for (const Group& gr : groups) {
    goff.push_back(total);
    total += 256 + al256(gr.items.size() * sizeof(GroupItemDev));  // queue word, then the item table
  }
  std::vector<size_t> stream_off;
  for (const StreamItem& si : stream_items) {
    const laim_batch_item& b = items[si.index];
    stream_off.push_back(total);
    total += al256(stream_workspace_bytes(b.code->dev, b.nshots,
                                          si.kp.conflict == kConflictSequential));
  }
  hipError_t e = hipMalloc(&plan->dev_mem, std::max<size_t>(total, 256));
  if (e != hipSuccess) {
    delete plan;
    set_error("hipMalloc of %zu bytes for the plan failed", total);
    return LAIM_ENOMEM;
  }
  char* base = (char*)plan->dev_mem;
  for (size_t k = 0; k < groups.size() && e == hipSuccess; ++k)
    e = hipMemcpy(base + goff[k] + 256, groups[k].items.data(), groups[k].items.size() * sizeof(GroupItemDev),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipStreamCreate(&plan->cap);
  if (e == hipSuccess) e = hipStreamBeginCapture(plan->cap, hipStreamCaptureModeThreadLocal);
  for (size_t k = 0; k < groups.size() && e == hipSuccess; ++k) {
    const Group& gr = groups[k];
    e = launch_resident_group(gr.code->dev, gr.kp, gr.sh, (const GroupItemDev*)(base + goff[k] + 256),
                              (int32_t)gr.items.size(), gr.total, base + goff[k], plan->cap);
  }
  for (int i : fallback_fail) {
    if (e != hipSuccess) break;
    const laim_batch_item& b = items[i];
    e = launch_failure(b.code->dev, b.e0, b.z_out, b.nshots, b.fail_out, plan->cap);
  }
  for (size_t k = 0; k < stream_items.size() && e == hipSuccess; ++k) {
    const laim_batch_item& b = items[stream_items[k].index];
    if (b.nshots == 0) continue;
    e = launch_stream(b.code->dev, stream_items[k].kp, b.e0, b.shot0, b.nshots, base + stream_off[k], b.z_out,
                      b.s_out, b.tclr_out, nullptr, plan->cap);
    if (e == hipSuccess && b.fail_out)
      e = launch_failure(b.code->dev, b.e0, b.z_out, b.nshots, b.fail_out, plan->cap);
  }
  if (plan->cap) {
    hipGraph_t gph = nullptr;
    hipError_t e2 = hipStreamEndCapture(plan->cap, &gph);
    if (e == hipSuccess) e = e2;
    plan->graph = gph;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&plan->exec, plan->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    laim_status st = hip_fail(e, "building the batched plan");
    laim_batch_plan_destroy(plan);
    return st;
  }
  *out = plan;
  return LAIM_OK;
}

laim_status laim_batch_plan_launch(laim_batch_plan* plan, laim_stream stream) {
  if (!plan || !plan->exec) {
    set_error("plan is NULL");
    return LAIM_EINVAL;
  }
  DeviceGuard g(plan->device);
  hipError_t e = hipGraphLaunch(plan->exec, (hipStream_t)stream);
  return e == hipSuccess ? LAIM_OK : hip_fail(e, "hipGraphLaunch");
}

void laim_batch_plan_destroy(laim_batch_plan* plan) {
  if (!plan) return;
  DeviceGuard g(plan->device);
  if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
  if (plan->graph) (void)hipGraphDestroy(plan->graph);
  if (plan->cap) (void)hipStreamDestroy(plan->cap);
  if (plan->dev_mem) (void)hipFree(plan->dev_mem);
  delete plan;
}

}  // extern "C"

// =================================================================== server
namespace {

// First-fit allocator over one device arena (offsets, 256-byte granules).
struct Arena {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used = 0;
  void init(size_t s) {
    size = s;
    free_.clear();
    if (s) free_[0] = s;
    used = 0;
  }
  bool alloc(size_t n, size_t* off) {
    n = al256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const size_t rest = it->second - n;
        const size_t roff = it->first + n;
        free_.erase(it);
        if (rest) free_[roff] = rest;
        used += n;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t n) {
    n = al256(n);
    used -= n;
    auto it = free_.emplace(off, n).first;
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
};

struct Request {
  uint64_t ticket;
  const laim_code* code;
  int item;  // index into the server's item table
  int bp;
  uint64_t shot;
  int32_t rounds_total;
  int32_t round = 0;
  int32_t retire = 1;
  std::vector<uint8_t> e0;  // the caller's error, or empty when it is sampled on the device
  uint64_t noise_bound = 0;  // floor(p 2^32) of a sampled error
  uint64_t noise_seed = 0;
  bool resident = false, done = false;
  size_t off = 0, bytes = 0;  // arena block
  size_t o_e0, o_msg, o_z, o_s, o_hdr;
  int32_t tclr = -1, fail = 0;
  int64_t t_ready = 0;
};

// Arena bytes of one request: e0 [n], messages [m][dcmax], z [n], s [m] and
// a 256-byte header, each part 256-byte aligned.
struct RequestLayout {
  size_t b_e0, b_msg, b_z, b_s, b_hdr, total;
};

RequestLayout request_layout(const laim_code* c) {
  RequestLayout l;
  l.b_e0 = al256(c->n);
  l.b_msg = al256((size_t)c->m * c->dcmax * 4);
  l.b_z = al256(c->n);
  l.b_s = al256(c->m);
  l.b_hdr = 256;
  l.total = l.b_e0 + l.b_msg + l.b_z + l.b_s + l.b_hdr;
  return l;
}

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct laim_server {
  int device = 0;
  int max_slots = 0;
  hipStream_t st = nullptr;
  void* arena_mem = nullptr;
  Arena arena;
  // item table (one record per distinct code + parameters), on host and device
  std::vector<BatchItemDev> items;
  std::vector<std::vector<char>> item_keys;
  std::vector<size_t> item_lds;
  std::vector<int> item_block;
  BatchItemDev* items_dev = nullptr;
  size_t items_dev_cap = 0;
  bool items_dirty = false;
  // per-step tables (pinned host, device)
  ServerReqDev* reqs_h = nullptr;
  ServerUnitDev* units_h = nullptr;
  int32_t* ev_h = nullptr;
  ServerReqDev* reqs_d = nullptr;
  ServerUnitDev* units_d = nullptr;
  int32_t* ev_d = nullptr;
  std::map<uint64_t, Request> reqs;
  std::deque<uint64_t> waiting;
  uint64_t next_ticket = 1;
};

extern "C" {

laim_status laim_server_create(int32_t device, size_t mem_budget_bytes, int32_t max_slots,
                               laim_server** out) {
  if (!out || max_slots < 1 || mem_budget_bytes < 4096) {
    set_error("laim_server_create: bad arguments");
    return LAIM_EINVAL;
  }
  *out = nullptr;
  laim_server* s = new (std::nothrow) laim_server();
  if (!s) {
    set_error("out of host memory");
    return LAIM_ENOMEM;
  }
  s->device = device;
  s->max_slots = max_slots;
  DeviceGuard g(device);
  hipError_t e = hipStreamCreate(&s->st);
  if (e == hipSuccess) e = hipMalloc(&s->arena_mem, mem_budget_bytes);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->reqs_h, sizeof(ServerReqDev) * max_slots, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->units_h, sizeof(ServerUnitDev) * max_slots, 0);
  if (e == hipSuccess) e = hipHostMalloc((void**)&s->ev_h, sizeof(int32_t) * 4 * max_slots, 0);
  if (e == hipSuccess) e = hipMalloc((void**)&s->reqs_d, sizeof(ServerReqDev) * max_slots);
  if (e == hipSuccess) e = hipMalloc((void**)&s->units_d, sizeof(ServerUnitDev) * max_slots);
  if (e == hipSuccess) e = hipMalloc((void**)&s->ev_d, sizeof(int32_t) * 4 * max_slots);
  if (e != hipSuccess) {
    laim_status st = hip_fail(e, "creating the server");
    laim_server_destroy(s);
    return st == LAIM_EHIP ? LAIM_ENOMEM : st;
  }
  s->arena.init(mem_budget_bytes);
  *out = s;
  return LAIM_OK;
}

void laim_server_destroy(laim_server* s) {
  if (!s) return;
  DeviceGuard g(s->device);
  if (s->st) (void)hipStreamSynchronize(s->st);
  if (s->reqs_h) (void)hipHostFree(s->reqs_h);
  if (s->units_h) (void)hipHostFree(s->units_h);
  if (s->ev_h) (void)hipHostFree(s->ev_h);
  if (s->reqs_d) (void)hipFree(s->reqs_d);
  if (s->units_d) (void)hipFree(s->units_d);
  if (s->ev_d) (void)hipFree(s->ev_d);
  if (s->items_dev) (void)hipFree(s->items_dev);
  if (s->arena_mem) (void)hipFree(s->arena_mem);
  if (s->st) (void)hipStreamDestroy(s->st);
  delete s;
}

laim_status laim_server_submit(laim_server* s, const laim_code* code,
                               const laim_decode_params* params, uint64_t shot_id,
                               const uint8_t* e0_host, double p, uint64_t* ticket) {
  if (!s || !code || !params || !ticket) {
    set_error("laim_server_submit: bad arguments");
    return LAIM_EINVAL;
  }
  if (!e0_host && p != p) {
    set_error("p is NaN");
    return LAIM_EINVAL;
  }
  if (code->device != s->device) {
    set_error("the code lives on another device than the server");
    return LAIM_EINVAL;
  }
  // a request larger than the whole arena could never be admitted and would
  // hold up the FIFO for good
  const size_t need = request_layout(code).total;
  if (need > s->arena.size) {
    set_error("a request of this code needs %zu bytes of device state; the server's budget is %zu",
              need, s->arena.size);
    return LAIM_ENOMEM;
  }
  // one item per distinct (code, parameters); the key is built field by
  // field so that padding bytes of the caller's struct do not enter it
  laim_decode_params kp_key;
  memset(&kp_key, 0, sizeof(kp_key));
  kp_key.bp = params->bp;
  kp_key.alpha = params->alpha;
  kp_key.q = params->q;
  kp_key.clamp = params->clamp;
  kp_key.iters = params->iters;
  kp_key.rounds = params->rounds;
  kp_key.mask_density = params->mask_density;
  kp_key.gauge = params->gauge;
  kp_key.evidence = params->evidence;
  kp_key.retire = params->retire;
  kp_key.seed = params->seed;
  kp_key.conflict = params->conflict;
  kp_key.skip_fixed = params->skip_fixed;
  kp_key.move = params->move;
  std::vector<char> key(sizeof(void*) + sizeof(laim_decode_params));
  memcpy(key.data(), &code, sizeof(void*));
  memcpy(key.data() + sizeof(void*), &kp_key, sizeof(laim_decode_params));
  int item = -1;
  for (size_t i = 0; i < s->item_keys.size(); ++i)
    if (s->item_keys[i] == key) item = (int)i;
  if (item < 0) {
    BatchItemDev it;
    size_t lds = 0;
    int block = 0;
    laim_status st = make_item(code, params, &it, &lds, &block);
    if (st != LAIM_OK) return st;
    item = (int)s->items.size();
    s->items.push_back(it);
    s->item_keys.push_back(key);
    s->item_lds.push_back(lds);
    s->item_block.push_back(block);
    s->items_dirty = true;
  }
  Request r;
  r.ticket = s->next_ticket++;
  r.code = code;
  r.item = item;
  r.bp = s->items[item].kp.bp;
  r.shot = shot_id;
  r.rounds_total = params->rounds;
  r.retire = params->retire ? 1 : 0;
  if (e0_host) {
    r.e0.assign(e0_host, e0_host + code->n);
    for (auto& b : r.e0) b &= 1u;
  } else {
    r.noise_bound = bernoulli_bound(p);
    r.noise_seed = params->seed;
  }
  r.t_ready = now_ns();
  *ticket = r.ticket;
  s->waiting.push_back(r.ticket);
  s->reqs.emplace(r.ticket, std::move(r));
  return LAIM_OK;
}

laim_status laim_server_step(laim_server* s, laim_server_event* events, int32_t max_events,
                             int32_t* n_events) {
  if (!s || !n_events || (max_events > 0 && !events)) {
    set_error("laim_server_step: bad arguments");
    return LAIM_EINVAL;
  }
  *n_events = 0;
  DeviceGuard g(s->device);
  hipError_t e = hipSuccess;
  // ---- admission, FIFO, while slots and memory allow
  int resident = 0;
  for (auto& kv : s->reqs)
    if (kv.second.resident && !kv.second.done) ++resident;
  while (!s->waiting.empty() && resident < s->max_slots) {
    Request& r = s->reqs.at(s->waiting.front());
    const laim_code* c = r.code;
    const RequestLayout lay = request_layout(c);
    size_t off;
    if (!s->arena.alloc(lay.total, &off)) break;
    r.off = off;
    r.bytes = lay.total;
    r.o_e0 = off;
    r.o_msg = r.o_e0 + lay.b_e0;
    r.o_z = r.o_msg + lay.b_msg;
    r.o_s = r.o_z + lay.b_z;
    r.o_hdr = r.o_s + lay.b_s;
    uint8_t* e0_dev = (uint8_t*)s->arena_mem + r.o_e0;
    if (r.e0.empty())  // sampled from (seed, shot id, p), as laim_sample_noise draws it
      e = launch_noise(c->dev, r.noise_bound, r.noise_seed, r.shot, 1, e0_dev, s->st);
    else
      e = hipMemcpyAsync(e0_dev, r.e0.data(), c->n, hipMemcpyHostToDevice, s->st);
    if (e != hipSuccess) {
      s->arena.release(r.off, r.bytes);
      return hip_fail(e, "admitting a request");
    }
    r.resident = true;
    s->waiting.pop_front();
    ++resident;
  }
  if (s->items_dirty) {
    if (s->items.size() > s->items_dev_cap) {
      if (s->items_dev) {
        (void)hipStreamSynchronize(s->st);
        (void)hipFree(s->items_dev);
      }
      s->items_dev_cap = std::max<size_t>(16, s->items.size() * 2);
      e = hipMalloc((void**)&s->items_dev, s->items_dev_cap * sizeof(BatchItemDev));
      if (e != hipSuccess) return hip_fail(e, "server item table");
    }
    e = hipMemcpyAsync(s->items_dev, s->items.data(), s->items.size() * sizeof(BatchItemDev),
                       hipMemcpyHostToDevice, s->st);
    if (e != hipSuccess) return hip_fail(e, "server item table");
    s->items_dirty = false;
  }
  // ---- units: resident requests grouped by (BP, item, first round or not)
  // At most max_events requests advance, the oldest first, so that every
  // advanced request reports its event (and a finished one its done flag).
  std::vector<uint64_t> order;
  for (auto& kv : s->reqs)
    if (kv.second.resident && !kv.second.done && (int32_t)order.size() < std::max(max_events, 0))
      order.push_back(kv.first);
  if (order.empty()) return LAIM_OK;
  // a unit holds requests of one item in the same phase: first round, later
  // round, or no round at all (rounds = 0: only the start state and result)
  auto phase = [](const Request& r) { return r.rounds_total == 0 ? 2 : (r.round > 0 ? 1 : 0); };
  std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) {
    const Request &x = s->reqs.at(a), &y = s->reqs.at(b);
    const int kx = x.bp * 1000000 + x.item * 3 + phase(x);
    const int ky = y.bp * 1000000 + y.item * 3 + phase(y);
    return kx < ky;
  });
  int nreq = 0, nunit = 0;
  int unit_first[2] = {-1, -1}, unit_count[2] = {0, 0};
  size_t lds[2] = {0, 0};
  int block[2] = {0, 0};
  for (size_t k = 0; k < order.size(); ++k) {
    Request& r = s->reqs.at(order[k]);
    char* A = (char*)s->arena_mem;
    ServerReqDev q;
    q.shot = r.shot;
    q.round = r.round;
    q.pad = 0;
    q.e0 = (const uint8_t*)(A + r.o_e0);
    q.msg = (float*)(A + r.o_msg);
    q.z = (uint8_t*)(A + r.o_z);
    q.s = (uint8_t*)(A + r.o_s);
    q.hdr = (int32_t*)(A + r.o_hdr);
    q.fail = (uint8_t*)(A + r.o_hdr + 16);
    q.ev = s->ev_d + 4 * nreq;
    s->reqs_h[nreq] = q;
    const BatchItemDev& it = s->items[r.item];
    const bool resume = r.round > 0;
    const int32_t nround = r.rounds_total > 0 ? 1 : 0;
    const bool new_unit = nunit == 0 || s->units_h[nunit - 1].item != r.item ||
                          s->units_h[nunit - 1].resume != (resume ? 1 : 0) ||
                          s->units_h[nunit - 1].rounds != nround ||
                          s->units_h[nunit - 1].count >= it.u.spb;
    if (new_unit) {
      if (unit_first[r.bp] < 0) unit_first[r.bp] = nunit;
      ++unit_count[r.bp];
      s->units_h[nunit++] = ServerUnitDev{r.item, nreq, 0, resume ? 1 : 0, nround};
      lds[r.bp] = std::max(lds[r.bp], s->item_lds[r.item]);
      block[r.bp] = std::max(block[r.bp], s->item_block[r.item]);
    }
    s->units_h[nunit - 1].count++;
    ++nreq;
  }
  e = hipMemcpyAsync(s->reqs_d, s->reqs_h, sizeof(ServerReqDev) * nreq, hipMemcpyHostToDevice, s->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->units_d, s->units_h, sizeof(ServerUnitDev) * nunit, hipMemcpyHostToDevice, s->st);
  for (int bp = 0; bp < 2 && e == hipSuccess; ++bp)
    if (unit_count[bp])
      e = launch_server(bp, s->items_dev, s->units_d + unit_first[bp], unit_count[bp], s->reqs_d,
                        lds[bp], block[bp], s->st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->ev_h, s->ev_d, sizeof(int32_t) * 4 * nreq, hipMemcpyDeviceToHost, s->st);
  if (e == hipSuccess) e = hipStreamSynchronize(s->st);
  if (e != hipSuccess) return hip_fail(e, "server step");
  const int64_t t = now_ns();
  int32_t ne = 0;
  for (int i = 0; i < nreq; ++i) {
    Request& r = s->reqs.at(order[i]);
    if (r.rounds_total > 0) r.round += 1;
    r.tclr = s->ev_h[4 * i + 2];
    r.fail = s->ev_h[4 * i + 3] & 1;
    // a frozen request (its state can no longer change) is finished: the
    // remaining rounds would leave z, s, t_clr and the failure as they are
    const bool frozen = (s->ev_h[4 * i + 3] >> 1) & 1;
    r.done = (r.retire && r.tclr >= 0) || r.round >= r.rounds_total || frozen;
    {
      laim_server_event& ev = events[ne++];
      ev.ticket = r.ticket;
      ev.round = r.round;
      ev.done = r.done ? 1 : 0;
      ev.tclr = r.tclr;
      ev.flips = s->ev_h[4 * i + 0];
      ev.defects = s->ev_h[4 * i + 1];
      ev.fail = r.fail;
      ev.latency_ns = t - r.t_ready;
    }
    r.t_ready = t;
  }
  *n_events = ne;
  return LAIM_OK;
}

laim_status laim_server_result(laim_server* s, uint64_t ticket, uint8_t* z_host, uint8_t* s_host,
                               int32_t* tclr) {
  if (!s) {
    set_error("server is NULL");
    return LAIM_EINVAL;
  }
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    set_error("unknown ticket");
    return LAIM_EINVAL;
  }
  Request& r = it->second;
  if (!r.done) {
    set_error("request %llu is not finished", (unsigned long long)ticket);
    return LAIM_EBUSY;
  }
  DeviceGuard g(s->device);
  hipError_t e = hipSuccess;
  char* A = (char*)s->arena_mem;
  if (z_host) e = hipMemcpy(z_host, A + r.o_z, r.code->n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && s_host) e = hipMemcpy(s_host, A + r.o_s, r.code->m, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "reading a result");
  if (tclr) *tclr = r.tclr;
  s->arena.release(r.off, r.bytes);
  s->reqs.erase(it);
  return LAIM_OK;
}

laim_status laim_server_stats(const laim_server* s, int32_t* resident, int32_t* waiting,
                              size_t* bytes_in_use) {
  if (!s) {
    set_error("server is NULL");
    return LAIM_EINVAL;
  }
  int32_t res = 0;
  for (auto& kv : s->reqs)
    if (kv.second.resident && !kv.second.done) ++res;
  if (resident) *resident = res;
  if (waiting) *waiting = (int32_t)s->waiting.size();
  if (bytes_in_use) *bytes_in_use = s->arena.used;
  return LAIM_OK;
}

}  // extern "C"
