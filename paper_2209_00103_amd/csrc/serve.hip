// Served mode: a host request loop over resident arrays with continuous batching.
//
// The request semantics are the single-array operations (insertion round, r/w,
// flatten of Sec. IV and VI-B); what this file adds is the scheduling: per-array
// FIFO order, steps that carry one request of many arrays each, several steps in
// flight on their own streams, and admission by a byte budget.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <new>
#include <queue>
#include <utility>
#include <vector>

#include "gga_internal.h"

using namespace gga;

namespace {

constexpr uint64_t kNone = ~0ull;
constexpr uint64_t kAlign = 256;

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Flatten outputs: a ring over the arena; space comes back in allocation order
// and is handed out again only after the ring has gone all the way round, so an
// output stays readable as long as the arena allows.
struct Ring {
  struct Span {
    uint64_t off, bytes;
    bool done;
  };
  uint64_t size = 0, head = 0, live = 0, wraps = 0;
  std::deque<Span> q;

  bool alloc(uint64_t n, uint64_t* off) {
    if (n > size) return false;
    if (q.empty()) {
      if (size - head >= n) *off = head;
      else {
        *off = 0;
        ++wraps;
      }
    } else {
      const uint64_t tail = q.front().off;
      if (head > tail) {  // live data in [tail, head): free space at the end, then at the start
        if (size - head >= n) *off = head;
        else if (tail >= n) {
          *off = 0;
          ++wraps;
        } else return false;
      } else {  // wrapped: free space is [head, tail) (none when equal)
        if (tail - head >= n) *off = head;
        else return false;
      }
    }
    head = *off + n;
    live += n;
    q.push_back(Span{*off, n, false});
    return true;
  }

  void release(uint64_t off) {
    for (Span& sp : q)
      if (sp.off == off && !sp.done) {
        sp.done = true;
        break;
      }
    while (!q.empty() && q.front().done) {
      live -= q.front().bytes;
      q.pop_front();
    }
  }
};

struct Lane {
  hipStream_t s = nullptr;
  hipEvent_t ev_a = nullptr;     // the step's appends (and scans) are done
  hipEvent_t ev = nullptr;       // the whole step is done
  uint8_t* h_stage = nullptr;    // pinned staging of the step table
  uint8_t* d_block = nullptr;    // device copy of the table, then the scan outputs
  std::vector<uint32_t> a_reqs;  // appends of the step in flight
  std::vector<uint32_t> reqs;    // its r/w and flatten requests
  bool busy = false;
  bool a_done = false;
};

uint64_t now_ns(std::chrono::steady_clock::time_point t0) {
  return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now() - t0)
      .count();
}

}  // namespace

struct gga_server {
  std::vector<ggarray*> arrays;
  uint32_t elem_bytes = 0;
  uint8_t* arena = nullptr;
  uint64_t arena_bytes = 0;
  gga_server_config cfg{};
  std::vector<Lane> lanes;
  uint64_t table_bytes = 0;  // fixed part of a lane block: the largest step table
  uint64_t* h_sizes = nullptr;
  std::vector<hipEvent_t> rq_events;  // per-request mode
};

namespace {

// Layout of one step table: [append items][append block offsets][stream items].
struct TableLayout {
  uint64_t begins, sitems, used;
};
TableLayout layout(uint32_t n_a, uint32_t n_s) {
  TableLayout L;
  L.begins = align_up((uint64_t)n_a * sizeof(BatchArr), 16);
  L.sitems = align_up(L.begins + ((uint64_t)n_a + 1) * sizeof(uint64_t), 16);
  L.used = L.sitems + (uint64_t)n_s * sizeof(ServeItem);
  return L;
}

void destroy_server(gga_server* sv) {
  for (Lane& l : sv->lanes) {
    if (l.s) hipStreamSynchronize(l.s);
    if (l.ev) hipEventDestroy(l.ev);
    if (l.ev_a) hipEventDestroy(l.ev_a);
    if (l.h_stage) hipHostFree(l.h_stage);
    if (l.d_block) hipFree(l.d_block);
    if (l.s) hipStreamDestroy(l.s);
  }
  for (hipEvent_t e : sv->rq_events) hipEventDestroy(e);
  if (sv->h_sizes) hipHostFree(sv->h_sizes);
  delete sv;
}

// Per-run bookkeeping shared by both modes.
struct RunState {
  gga_server* sv;
  const gga_trace* tr;
  uint64_t *t_issue, *t_done, *out_offset, *dev_out_len;
  int32_t* status;
  std::vector<uint64_t> size;  // host bound of each array's size
  uint64_t charged = 0;        // sum of the arrays' capacity bounds, bytes
  Ring ring;
  uint64_t done = 0, rejected = 0, waits = 0, peak = 0, steps = 0, largest = 0, issued = 0;
  std::chrono::steady_clock::time_point t0;

  uint64_t vf(uint32_t a) const { return (uint64_t)sv->arrays[a]->V << sv->arrays[a]->log2F; }

  // 0: admitted (flatten space reserved at *off), 1: wait, 2: reject.
  int admit(uint32_t r, uint64_t* off) {
    const uint32_t a = tr->target[r];
    const uint8_t kind = tr->kind[r];
    const uint64_t cap = sv->cfg.cap_bytes;
    const uint64_t need_arr = kind == GGA_REQ_APPEND ? 2ull * tr->length[r] * sv->elem_bytes : 0;
    const uint64_t need_out = kind == GGA_REQ_FLATTEN ? align_up(size[a] * sv->elem_bytes, kAlign) : 0;
    *off = kNone;
    if (charged + need_arr + need_out > cap || need_out > sv->arena_bytes) return 2;
    if (charged + ring.live + need_arr + need_out > cap) return 1;
    if (kind == GGA_REQ_FLATTEN) {
      if (need_out == 0) *off = 0;
      else if (!ring.alloc(need_out, off)) return 1;
    }
    charged += need_arr;
    if (kind == GGA_REQ_APPEND) size[a] += tr->length[r];
    const uint64_t total = charged + ring.live;
    if (total > peak) peak = total;
    return 0;
  }

  void reject(uint32_t r) {
    const uint64_t t = now_ns(t0);
    status[r] = GGA_ENOMEM;
    t_issue[r] = t_done[r] = t;
    ++rejected;
    ++done;
  }

  // Flatten reservations go back by offset; one of zero bytes holds no span.
  std::vector<uint64_t> flat_bytes;

  void finish(uint32_t r, uint64_t t) {
    t_done[r] = t;
    if (tr->kind[r] == GGA_REQ_FLATTEN && flat_bytes[r] != 0) ring.release(out_offset[r]);
    ++done;
  }
};

int read_sizes(gga_server* sv, std::vector<uint64_t>& size) {
  hipStream_t s = sv->lanes[0].s;
  if (hipDeviceSynchronize() != hipSuccess) return GGA_EHIP;
  for (size_t i = 0; i < sv->arrays.size(); ++i) {
    ggarray* a = sv->arrays[i];
    const int rc = launch_scan(a, s);
    if (rc) return rc;
    if (hipMemcpyAsync(sv->h_sizes + i, a->ref.prefix + a->V, sizeof(uint64_t), hipMemcpyDeviceToHost, s) !=
        hipSuccess)
      return GGA_EHIP;
  }
  if (hipStreamSynchronize(s) != hipSuccess) return GGA_EHIP;
  for (size_t i = 0; i < sv->arrays.size(); ++i) size[i] = sv->h_sizes[i];
  return GGA_OK;
}

int drain(gga_server* sv) {
  int rc = GGA_OK;
  for (Lane& l : sv->lanes)
    if (hipStreamSynchronize(l.s) != hipSuccess) rc = GGA_EHIP;
  return rc;
}

// ------------------------------------------------------- continuous batching --
int run_batched(RunState& R) {
  gga_server* sv = R.sv;
  const gga_trace* tr = R.tr;
  const uint32_t A = (uint32_t)sv->arrays.size();
  const uint32_t te_log2 = sv->elem_bytes == 4 ? 12u : 11u;
  std::vector<std::deque<uint32_t>> q(A);
  std::vector<uint8_t> busy(A, 0);
  typedef std::pair<uint64_t, uint32_t> Head;  // (arrival of the array's oldest request, array)
  std::priority_queue<Head, std::vector<Head>, std::greater<Head>> ready;
  std::vector<BatchArr> items;
  std::vector<uint64_t> begins;
  std::vector<ServeItem> sitems;
  std::vector<uint32_t> reqs, a_reqs;
  struct Picked {
    uint32_t r;
    uint64_t off, s_before;  // flatten: its arena offset; the array's size before the request
  };
  std::vector<Picked> picked;
  uint64_t next = 0;
  const uint64_t n = tr->n;

  auto requeue = [&](uint32_t a) {
    if (!busy[a] && !q[a].empty()) ready.push(Head{tr->arrival_ns[q[a].front()], a});
  };

  while (R.done < n) {
    const uint64_t t = now_ns(R.t0);
    while (next < n && tr->arrival_ns[next] <= t) {
      const uint32_t a = tr->target[next];
      q[a].push_back((uint32_t)next);
      if (q[a].size() == 1) requeue(a);
      ++next;
    }
    for (Lane& l : sv->lanes) {
      if (!l.busy) continue;
      if (!l.a_done) {  // appends finish before the step's streaming launch
        const hipError_t e = hipEventQuery(l.ev_a);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return GGA_EHIP;
        const uint64_t tc = now_ns(R.t0);
        for (uint32_t r : l.a_reqs) {
          R.finish(r, tc);
          const uint32_t a = tr->target[r];
          busy[a] = 0;
          requeue(a);
        }
        l.a_reqs.clear();
        l.a_done = true;
      }
      const hipError_t e = hipEventQuery(l.ev);
      if (e == hipErrorNotReady) continue;
      if (e != hipSuccess) return GGA_EHIP;
      const uint64_t tc = now_ns(R.t0);
      for (uint32_t r : l.reqs) {
        R.finish(r, tc);
        const uint32_t a = tr->target[r];
        busy[a] = 0;
        requeue(a);
      }
      l.reqs.clear();
      l.busy = false;
    }
    // Ready requests are spread over the idle lanes: each takes its share, so at
    // low load requests go out at once as single-request steps on lanes of their
    // own (running side by side), and steps grow only when requests outnumber the
    // idle lanes.
    uint32_t idle = 0;
    for (const Lane& l : sv->lanes) idle += l.busy ? 0u : 1u;
    for (Lane& l : sv->lanes) {
      if (l.busy || ready.empty()) continue;
      const size_t share = (ready.size() + idle - 1) / idle;
      const size_t cap = share < sv->cfg.max_step ? (share ? share : 1) : sv->cfg.max_step;
      --idle;
      items.clear();
      begins.clear();
      sitems.clear();
      reqs.clear();
      a_reqs.clear();
      uint64_t blocks = 0, grid = 0;
      picked.clear();
      while (picked.size() < cap && !ready.empty()) {
        const Head h = ready.top();
        const uint32_t a = h.second;
        if (busy[a] || q[a].empty() || tr->arrival_ns[q[a].front()] != h.first) {
          ready.pop();  // stale entry
          continue;
        }
        const uint32_t r = q[a].front();
        ggarray* arr = sv->arrays[a];
        uint64_t ntiles = 0;
        if (tr->kind[r] == GGA_REQ_APPEND) {
          const uint64_t len = tr->length[r];
          const uint64_t chunk = (len + arr->V - 1) / arr->V;
          ntiles = (chunk + kInsertTile - 1) / kInsertTile * arr->V;
          if (blocks && blocks + ntiles > 0x7FFFFFFFull - sv->cfg.max_step) break;  // the step is full
          blocks += ntiles;
        }
        uint64_t off = kNone;
        const uint64_t s_before = R.size[a];
        const int ad = R.admit(r, &off);
        if (ad == 1) {
          ++R.waits;
          break;  // oldest first: wait for memory before taking younger requests
        }
        ready.pop();
        q[a].pop_front();
        if (ad == 2) {
          if (tr->kind[r] == GGA_REQ_APPEND) blocks -= ntiles;
          R.reject(r);
          requeue(a);
          continue;
        }
        busy[a] = 1;
        picked.push_back(Picked{r, off, s_before});
      }
      if (picked.empty()) continue;
      if (picked.size() == 1) {
        // A step of one request (light load) skips the step table: the request runs
        // with the single-array launches on the lane's stream, as it would alone.
        const Picked& p1 = picked[0];
        const uint32_t r = p1.r;
        ggarray* arr = sv->arrays[tr->target[r]];
        int rc = GGA_OK;
        if (tr->kind[r] == GGA_REQ_APPEND) {
          InsertDesc d{};
          d.mode = kModeKeyed;
          d.n_threads = tr->length[r];
          d.seed = sv->cfg.seed;
          d.round = sv->cfg.append_round;
          d.tag_shift = sv->cfg.append_shift;
          d.tag = r;
          d.max_count = 1;
          rc = launch_insert(arr, d, l.s);
        } else {
          rc = launch_scan(arr, l.s);
          if (!rc && tr->kind[r] == GGA_REQ_RW) rc = launch_rw(arr, sv->cfg.rw_op, l.s);
          if (!rc && tr->kind[r] == GGA_REQ_FLATTEN) {
            R.out_offset[r] = p1.off;
            R.flat_bytes[r] = p1.s_before * sv->elem_bytes;
            rc = launch_flatten(arr, sv->arena + p1.off, p1.s_before, l.s);
            if (!rc && R.dev_out_len &&
                hipMemcpyAsync(R.dev_out_len + r, arr->ref.prefix + arr->V, sizeof(uint64_t),
                               hipMemcpyDeviceToDevice, l.s) != hipSuccess)
              rc = GGA_EHIP;
          }
        }
        if (rc) return rc;
        // One event for the whole step: with a single request there is nothing to
        // release before the step ends (one event record and query fewer than
        // the table steps take).
        l.reqs.assign(1, r);
        if (hipEventRecord(l.ev, l.s) != hipSuccess) return GGA_EHIP;
        R.t_issue[r] = now_ns(R.t0);
        l.busy = true;
        l.a_done = true;
        ++R.steps;
        ++R.issued;
        if (R.largest < 1) R.largest = 1;
        continue;
      }
      blocks = 0;
      for (const Picked& pk : picked) {
        const uint32_t r = pk.r;
        ggarray* arr = sv->arrays[tr->target[r]];
        const uint8_t kind = tr->kind[r];
        (kind == GGA_REQ_APPEND ? a_reqs : reqs).push_back(r);
        if (kind == GGA_REQ_APPEND) {
          BatchArr it;
          uint64_t ntiles = 0;
          const int rc = prepare_round_item(arr, tr->length[r], r, (uint32_t)items.size(), &it, &ntiles, l.s, true);
          if (rc) return rc;
          items.push_back(it);
          begins.push_back(blocks);
          blocks += ntiles;
          sizes_changed(arr, l.s);
          grow_bound(arr, tr->length[r]);
        } else {
          const bool flat = kind == GGA_REQ_FLATTEN;
          if (flat) {
            R.out_offset[r] = pk.off;
            R.flat_bytes[r] = pk.s_before * sv->elem_bytes;
          }
          sitems.push_back(ServeItem{arr->ref, flat ? (void*)(sv->arena + pk.off) : nullptr, pk.s_before,
                                     flat && R.dev_out_len ? R.dev_out_len + r : nullptr,
                                     flat ? kOpFlatten : sv->cfg.rw_op, arr->elem_log2});
          grid += (pk.s_before >> te_log2) + 2ull * arr->V;
          arr->prefix_valid = true;
          arr->scan_tag = 0;  // the server runs eagerly
        }
      }
      if (reqs.empty() && a_reqs.empty()) continue;
      begins.push_back(blocks);
      const uint32_t n_a = (uint32_t)items.size(), n_s = (uint32_t)sitems.size();
      const TableLayout L = layout(n_a, n_s);
      if (n_a) {
        std::memcpy(l.h_stage, items.data(), n_a * sizeof(BatchArr));
        std::memcpy(l.h_stage + L.begins, begins.data(), (n_a + 1) * sizeof(uint64_t));
      }
      if (n_s) std::memcpy(l.h_stage + L.sitems, sitems.data(), n_s * sizeof(ServeItem));
      uint8_t* d = l.d_block;
      uint64_t* d_tile = reinterpret_cast<uint64_t*>(d + sv->table_bytes);
      uint64_t* d_elem = d_tile + sv->cfg.max_step + 1;
      uint32_t* d_err = reinterpret_cast<uint32_t*>(d_elem + sv->cfg.max_step + 1);
      if (hipMemcpyAsync(d, l.h_stage, L.used, hipMemcpyHostToDevice, l.s) != hipSuccess) return GGA_EHIP;
      const ServeItem* d_sitems = reinterpret_cast<const ServeItem*>(d + L.sitems);
      int rc = launch_serve_front(reinterpret_cast<const BatchArr*>(d), reinterpret_cast<const uint64_t*>(d + L.begins),
                                  n_a, blocks, d_sitems, n_s, sv->elem_bytes, sv->cfg.seed, sv->cfg.append_round,
                                  sv->cfg.append_shift, l.s);
      if (rc) return rc;
      if (hipEventRecord(l.ev_a, l.s) != hipSuccess) return GGA_EHIP;
      rc = launch_serve_stream(d_sitems, n_s, d_tile, d_elem, d_err, sv->elem_bytes,
                               (uint32_t)std::min<uint64_t>(grid, 1u << 20), l.s);
      if (rc) return rc;
      if (hipEventRecord(l.ev, l.s) != hipSuccess) return GGA_EHIP;
      const uint64_t ti = now_ns(R.t0);
      for (uint32_t r : reqs) R.t_issue[r] = ti;
      for (uint32_t r : a_reqs) R.t_issue[r] = ti;
      const uint64_t in_step = reqs.size() + a_reqs.size();
      l.reqs.swap(reqs);
      l.a_reqs.swap(a_reqs);
      l.busy = true;
      l.a_done = false;
      ++R.steps;
      R.issued += in_step;
      if (in_step > R.largest) R.largest = in_step;
    }
  }
  return GGA_OK;
}

// ------------------------------------------------------ one launch per request --
int run_per_request(RunState& R) {
  gga_server* sv = R.sv;
  const gga_trace* tr = R.tr;
  hipStream_t s = sv->lanes[0].s;
  const uint32_t depth = sv->cfg.depth;
  std::deque<uint32_t> arrived;
  std::deque<std::pair<uint32_t, uint32_t>> inflight;  // (request, event slot)
  uint64_t next = 0, slot = 0;
  const uint64_t n = tr->n;
  while (R.done < n) {
    const uint64_t t = now_ns(R.t0);
    while (next < n && tr->arrival_ns[next] <= t) arrived.push_back((uint32_t)next++);
    while (!inflight.empty()) {
      const hipError_t e = hipEventQuery(sv->rq_events[inflight.front().second]);
      if (e == hipErrorNotReady) break;
      if (e != hipSuccess) return GGA_EHIP;
      R.finish(inflight.front().first, now_ns(R.t0));
      inflight.pop_front();
    }
    while (!arrived.empty() && inflight.size() < depth) {
      const uint32_t r = arrived.front();
      const uint32_t a = tr->target[r];
      ggarray* arr = sv->arrays[a];
      uint64_t off = kNone;
      const uint64_t s_before = R.size[a];
      const int ad = R.admit(r, &off);
      if (ad == 1) {
        ++R.waits;
        break;
      }
      arrived.pop_front();
      if (ad == 2) {
        R.reject(r);
        continue;
      }
      int rc = GGA_OK;
      const uint8_t kind = tr->kind[r];
      if (kind == GGA_REQ_APPEND) {
        InsertDesc d{};
        d.mode = kModeKeyed;
        d.n_threads = tr->length[r];
        d.seed = sv->cfg.seed;
        d.round = sv->cfg.append_round;
        d.tag_shift = sv->cfg.append_shift;
        d.tag = r;
        d.max_count = 1;
        rc = launch_insert(arr, d, s);
      } else {
        rc = launch_scan(arr, s);
        if (!rc && kind == GGA_REQ_RW) rc = launch_rw(arr, sv->cfg.rw_op, s);
        if (!rc && kind == GGA_REQ_FLATTEN) {
          R.out_offset[r] = off;
          R.flat_bytes[r] = s_before * sv->elem_bytes;
          rc = launch_flatten(arr, sv->arena + off, s_before, s);
          if (!rc && R.dev_out_len &&
              hipMemcpyAsync(R.dev_out_len + r, arr->ref.prefix + arr->V, sizeof(uint64_t),
                             hipMemcpyDeviceToDevice, s) != hipSuccess)
            rc = GGA_EHIP;
        }
      }
      if (rc) return rc;
      const uint32_t k = (uint32_t)(slot++ % depth);
      if (hipEventRecord(sv->rq_events[k], s) != hipSuccess) return GGA_EHIP;
      R.t_issue[r] = now_ns(R.t0);
      inflight.push_back(std::make_pair(r, k));
      ++R.steps;
      ++R.issued;
      R.largest = 1;
    }
  }
  return GGA_OK;
}

bool valid_config(const gga_server_config* c) {
  if (!c || c->mode > GGA_SERVE_PER_REQUEST || c->seed >= 256 || c->append_round >= 256) return false;
  if (c->append_shift < 1 || c->append_shift > 47 || c->rw_op > GGA_ADD1_X30) return false;
  if (c->lanes < 1 || c->lanes > 8 || c->max_step < 1 || c->max_step > 65536) return false;
  if (c->depth < 1 || c->depth > 65536) return false;
  return true;
}

}  // namespace

extern "C" {

int gga_server_create(gga_server** out, ggarray* const* arrays, uint32_t n, void* arena, uint64_t arena_bytes,
                      const gga_server_config* cfg) {
  if (!out || !arrays || n == 0 || !valid_config(cfg) || (arena_bytes && !arena)) return GGA_EINVAL;
  *out = nullptr;
  for (uint32_t i = 0; i < n; ++i) {
    if (!arrays[i] || arrays[i]->elem_bytes != arrays[0]->elem_bytes) return GGA_EINVAL;
    for (uint32_t j = 0; j < i; ++j)
      if (arrays[j] == arrays[i]) return GGA_EINVAL;
  }
  gga_server* sv = new (std::nothrow) gga_server;
  if (!sv) return GGA_EHIP;
  sv->arrays.assign(arrays, arrays + n);
  sv->elem_bytes = arrays[0]->elem_bytes;
  sv->arena = static_cast<uint8_t*>(arena);
  sv->arena_bytes = arena_bytes / kAlign * kAlign;
  sv->cfg = *cfg;
  const uint32_t m = cfg->mode == GGA_SERVE_BATCHED ? cfg->max_step : 1;
  const uint32_t nl = cfg->mode == GGA_SERVE_BATCHED ? cfg->lanes : 1;
  const TableLayout L = layout(m, m);
  sv->table_bytes = align_up(L.used, kAlign);
  const uint64_t block = sv->table_bytes + 2ull * (m + 1) * sizeof(uint64_t) + kAlign;
  bool ok = hipHostMalloc(reinterpret_cast<void**>(&sv->h_sizes), sizeof(uint64_t) * n, hipHostMallocDefault) ==
            hipSuccess;
  sv->lanes.resize(nl);
  for (Lane& l : sv->lanes) {
    if (!ok) break;
    ok = hipStreamCreateWithFlags(&l.s, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&l.ev, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&l.ev_a, hipEventDisableTiming) == hipSuccess &&
         hipHostMalloc(reinterpret_cast<void**>(&l.h_stage), sv->table_bytes, hipHostMallocDefault) == hipSuccess &&
         hipMalloc(reinterpret_cast<void**>(&l.d_block), block) == hipSuccess &&
         hipMemset(l.d_block, 0, block) == hipSuccess;
  }
  if (ok && cfg->mode == GGA_SERVE_PER_REQUEST) {
    sv->rq_events.resize(cfg->depth, nullptr);
    for (hipEvent_t& e : sv->rq_events)
      if (ok) ok = hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    destroy_server(sv);
    return GGA_EHIP;
  }
  *out = sv;
  return GGA_OK;
}

int gga_server_destroy(gga_server* sv) {
  if (!sv) return GGA_EINVAL;
  destroy_server(sv);
  return GGA_OK;
}

int gga_server_run(gga_server* sv, const gga_trace* tr, uint64_t* t_issue_ns, uint64_t* t_done_ns, int32_t* status,
                   uint64_t* out_offset, uint64_t* dev_out_len, uint64_t* stats) {
  if (!sv || !tr || !t_issue_ns || !t_done_ns || !status || !out_offset) return GGA_EINVAL;
  const uint64_t n = tr->n;
  if (n && (!tr->arrival_ns || !tr->kind || !tr->target || !tr->length)) return GGA_EINVAL;
  if (n >= (1ull << 32) || (n && ((n - 1) >> (48 - sv->cfg.append_shift)) != 0)) return GGA_EINVAL;
  for (uint64_t r = 0; r < n; ++r) {
    if (tr->kind[r] > GGA_REQ_FLATTEN || tr->target[r] >= sv->arrays.size()) return GGA_EINVAL;
    if (r && tr->arrival_ns[r] < tr->arrival_ns[r - 1]) return GGA_EINVAL;
    if (tr->kind[r] == GGA_REQ_APPEND &&
        (tr->length[r] == 0 || (uint64_t)tr->length[r] > (1ull << sv->cfg.append_shift)))
      return GGA_EINVAL;
  }
  RunState R;
  R.sv = sv;
  R.tr = tr;
  R.t_issue = t_issue_ns;
  R.t_done = t_done_ns;
  R.status = status;
  R.out_offset = out_offset;
  R.dev_out_len = dev_out_len;
  R.ring.size = sv->arena_bytes;
  R.size.assign(sv->arrays.size(), 0);
  R.flat_bytes.assign(n, 0);
  for (uint64_t r = 0; r < n; ++r) {
    t_issue_ns[r] = t_done_ns[r] = 0;
    status[r] = GGA_OK;
    out_offset[r] = kNone;
  }
  int rc = read_sizes(sv, R.size);
  if (rc) return rc;
  for (uint32_t a = 0; a < sv->arrays.size(); ++a) R.charged += (2 * R.size[a] + R.vf(a)) * sv->elem_bytes;
  R.peak = R.charged;
  R.t0 = std::chrono::steady_clock::now();
  rc = sv->cfg.mode == GGA_SERVE_BATCHED ? run_batched(R) : run_per_request(R);
  const uint64_t elapsed = now_ns(R.t0);
  const int drc = drain(sv);
  if (!rc) rc = drc;
  if (!rc && sv->cfg.mode == GGA_SERVE_BATCHED) {
    for (Lane& l : sv->lanes) {
      uint32_t err = 0;
      const uint64_t* d_tile = reinterpret_cast<const uint64_t*>(l.d_block + sv->table_bytes);
      const uint32_t* d_err = reinterpret_cast<const uint32_t*>(d_tile + 2ull * (sv->cfg.max_step + 1));
      if (hipMemcpy(&err, d_err, sizeof(err), hipMemcpyDeviceToHost) != hipSuccess) rc = GGA_EHIP;
      else if (err == kErrRange && !rc) rc = GGA_ERANGE;
    }
  }
  if (stats) {
    stats[0] = R.steps;
    stats[1] = R.largest;
    stats[2] = R.issued;
    stats[3] = R.rejected;
    stats[4] = R.waits;
    stats[5] = R.peak;
    stats[6] = elapsed;
    stats[7] = R.ring.wraps;
  }
  return rc;
}

}  // extern "C"
