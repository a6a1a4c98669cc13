// Query server with continuous batching over resident scenes (include/ar.h, "Query
// server").  Host code: one worker thread per slot, each with its own HIP stream and
// workspace; a queue taken in order with admission by the device-memory budget; a query
// starts beside running ones only when a backlog has built up, and then takes the later
// queued queries that can share its launches with it (one batch of cells over their
// scenes).
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "ar_host.h"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Query {
  int64_t ticket = 0;
  int32_t scene = 0;
  ar_pose_box box{};
  ar_options opts{};
  ar::Params prm{};
  int P = 0;
  bool rotates = false;
  size_t est = 0;              // estimated workspace bytes
  size_t ws_bytes = 0;         // workspace bytes held by its slot when it finished
  float *lo = nullptr, *hi = nullptr;
  Clock::time_point t_submit, t_start, t_end;
  int status = AR_PENDING;
  int slot = -1;
  int batched = 1;             // queries of the launch that rendered it
  ar_stats stats{};
  std::string error;
};

struct Slot {
  hipStream_t stream = nullptr;
  ar::Workspace ws;
  bool busy = false;
  size_t charge = 0;           // bytes counted against the budget (held, or the estimate while running)
  std::thread worker;
};

}  // namespace

struct ar_server {
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Query>> queue;
  std::map<int64_t, std::shared_ptr<Query>> records;
  std::vector<const ar_scene *> scenes;
  std::vector<ar::Density> density;   // per scene, from its last query (rotating and not)
  std::vector<ar::Density> density_rot;
  std::vector<double> density_pix, density_rot_pix;   // image pixels of those queries
  std::vector<std::unique_ptr<Slot>> slots;
  std::vector<double> latencies;
  int device = 0;
  uint64_t budget = 0, peak_bytes = 0;
  int64_t next_ticket = 1, submitted = 0, completed = 0, failed = 0, pairs = 0, releases = 0;
  int64_t shared_launches = 0, shared_queries = 0;
  int inflight = 0, peak_inflight = 0;
  int overlap_queue = 4;       // queries waiting from which one starts beside running ones
  int batch_max = 1;           // most queries in one shared launch (1: none shared)
  double busy_s = 0.0;
  Clock::time_point busy_since;
  bool stop = false;

  // b can share a with launches: the same image, options and pose variables, results
  // that do not depend on the launch's size (rotation boxes: fixed segment length;
  // translation boxes: only with options.chunk), and plain scenes or one scene
  bool shareable(const Query &a, const Query &b) const {
    if (a.P != b.P || a.rotates != b.rotates) return false;
    if (!a.rotates && a.opts.chunk <= 0) return false;
    if (memcmp(&a.opts, &b.opts, sizeof(ar_options)) != 0) return false;
    if (a.prm.width != b.prm.width || a.prm.height != b.prm.height || a.prm.fx != b.prm.fx ||
        a.prm.fy != b.prm.fy || a.prm.cx != b.prm.cx || a.prm.cy != b.prm.cy)
      return false;
    return a.scene == b.scene || (scenes[a.scene]->dev.nvar == 0 && scenes[b.scene]->dev.nvar == 0);
  }

  size_t charged_except(const Slot *me) const {
    size_t b = 0;
    for (auto &s : slots)
      if (s.get() != me) b += s->charge;
    return b;
  }

  void work(int k) {
    (void)hipSetDevice(device);
    Slot &slot = *slots[k];
    for (;;) {
      std::vector<std::shared_ptr<Query>> group;   // the head query, then those sharing its launches
      {
        std::unique_lock<std::mutex> lk(mu);
        for (;;) {
          // the next query in order starts when no query runs, or beside running ones
          // once overlap_queue queries wait (kernels of concurrent queries interleave
          // without preemption, so a query beside a long one stretches: worth it only
          // to drain a backlog), and when its workspace fits the budget
          if (!queue.empty()) {
            const auto h = queue.front();
            const size_t need = std::max(slot.ws.bytes, h->est);
            const bool backlog = (int)queue.size() >= overlap_queue;
            if (inflight == 0 || (backlog && charged_except(&slot) + need <= budget)) {
              group.push_back(h);
              queue.pop_front();
              size_t total = h->est;
              // under the backlog, later queries that can share the head's launches, while
              // their estimates fit the budget together
              if (backlog && batch_max > 1) {
                for (auto it = queue.begin(); it != queue.end() && (int)group.size() < batch_max;) {
                  if (shareable(*h, **it) && charged_except(&slot) + total + (*it)->est <= budget) {
                    total += (*it)->est;
                    group.push_back(*it);
                    it = queue.erase(it);
                  } else {
                    ++it;
                  }
                }
              }
              slot.charge = std::max(slot.ws.bytes, total);
              break;
            }
          } else if (stop) {
            return;
          }
          cv_work.wait(lk);
        }
        slot.busy = true;
        if (inflight++ == 0) busy_since = Clock::now();
        peak_inflight = std::max(peak_inflight, inflight);
        for (auto &g : group) {
          g->t_start = Clock::now();
          g->slot = k;
        }
      }
      const Query &q = *group[0];
      const int m = (int)group.size();
      std::vector<ar_stats> st(m);
      std::vector<int> rcs(m, AR_OK);
      std::vector<std::string> errs(m);
      int rc = AR_OK;
      if (m > 1) {
        // one batch of cells over the queries' scenes into the slot's staging images, then
        // copied to each query's outputs
        std::vector<ar_pose_box> boxes(m);
        std::vector<const ar_scene *> cs(m);
        for (int i = 0; i < m; ++i) {
          boxes[i] = group[i]->box;
          cs[i] = scenes[group[i]->scene];
        }
        const size_t img = (size_t)q.prm.width * q.prm.height * 3;
        rc = ar::ensure_out_stage(slot.ws, (size_t)m * img);
        ar_stats bst{};
        if (rc == AR_OK)
          rc = ar::render_cells(cs[0], slot.ws, q.prm, boxes.data(), m, q.P, q.rotates, slot.ws.out_stage,
                                slot.ws.out_stage + (size_t)m * img, slot.stream, &bst, cs.data());
        for (int i = 0; i < m && rc == AR_OK; ++i) {
          const float *slo = slot.ws.out_stage + (size_t)i * img, *shi = slot.ws.out_stage + (size_t)(m + i) * img;
          if (hipMemcpyAsync(group[i]->lo, slo, img * sizeof(float), hipMemcpyDeviceToDevice, slot.stream) !=
                  hipSuccess ||
              hipMemcpyAsync(group[i]->hi, shi, img * sizeof(float), hipMemcpyDeviceToDevice, slot.stream) !=
                  hipSuccess)
            rc = ar::fail(AR_E_DEVICE, "copy of a shared launch's images failed");
        }
        if (rc == AR_OK && hipStreamSynchronize(slot.stream) != hipSuccess)
          rc = ar::fail(AR_E_DEVICE, "shared launch failed on the device");
        for (int i = 0; i < m; ++i) st[i] = bst;
      }
      if (m == 1 || rc != AR_OK) {
        // alone (or each query again on its own when the shared launch failed)
        for (int i = 0; i < m; ++i) {
          const Query &g = *group[i];
          st[i] = ar_stats{};
          rcs[i] = ar::render_cells(scenes[g.scene], slot.ws, g.prm, &g.box, 1, g.P, g.rotates, g.lo, g.hi, slot.stream,
                                    &st[i]);
          if (rcs[i]) errs[i] = ar::g_error;
        }
      }
      const bool shared = m > 1 && rc == AR_OK;
      {
        std::lock_guard<std::mutex> lk(mu);
        const Clock::time_point now = Clock::now();
        if (--inflight == 0) busy_s += std::chrono::duration<double>(now - busy_since).count();
        if (shared) {
          ++shared_launches;
          shared_queries += m;
          pairs += st[0].pairs;
        }
        for (int i = 0; i < m; ++i) {
          Query &g = *group[i];
          g.t_end = now;
          g.status = rcs[i];
          g.stats = st[i];
          g.error = errs[i];
          g.batched = shared ? m : 1;
          if (rcs[i] == AR_OK) {
            ++completed;
            latencies.push_back(ms_between(g.t_submit, now));
            if (!shared) pairs += st[i].pairs;
            if (m == 1) {
              // the scene's density, from a launch of that scene alone
              (g.rotates ? density_rot : density)[g.scene] = slot.ws.density;
              (g.rotates ? density_rot_pix : density_pix)[g.scene] = (double)g.prm.width * g.prm.height;
            }
          } else {
            ++failed;
          }
          g.ws_bytes = slot.ws.bytes;
        }
        slot.busy = false;
        slot.charge = slot.ws.bytes;
        peak_bytes = std::max<uint64_t>(peak_bytes, charged_except(nullptr));
        // hand memory back when the held workspaces exceed the budget
        if (charged_except(nullptr) > budget) {
          ar::release_workspace(slot.ws);
          slot.charge = 0;
          ++releases;
        }
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

int ar_server_create(const ar_server_config *cfg, ar_server **out) {
  if (!out) return ar::fail(AR_E_INVALID, "out is NULL");
  *out = nullptr;
  ar_server_config c{};
  if (cfg) c = *cfg;
  if (c.slots < 0 || c.slots > 16) return ar::fail(AR_E_INVALID, "slots %d outside [0, 16]", c.slots);
  if (c.overlap_queue < 0) return ar::fail(AR_E_INVALID, "overlap_queue %d is negative", c.overlap_queue);
  if (c.batch_max < 0 || c.batch_max > 256) return ar::fail(AR_E_INVALID, "batch_max %d outside [0, 256]", c.batch_max);
  if (c.reserved != 0) return ar::fail(AR_E_INVALID, "reserved must be 0");
  std::unique_ptr<ar_server> srv(new ar_server());
  HIP_TRY(hipGetDevice(&srv->device));
  if (c.hbm_budget == 0) {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    c.hbm_budget = free_b / 2;
  }
  srv->budget = c.hbm_budget;
  const int nslots = c.slots ? c.slots : 4;
  srv->overlap_queue = c.overlap_queue ? c.overlap_queue : nslots;
  srv->batch_max = c.batch_max ? c.batch_max : 1;
  for (int k = 0; k < nslots; ++k) {
    std::unique_ptr<Slot> s(new Slot());
    HIP_TRY(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
    srv->slots.push_back(std::move(s));
  }
  for (int k = 0; k < nslots; ++k) {
    ar_server *p = srv.get();
    srv->slots[k]->worker = std::thread([p, k] { p->work(k); });
  }
  *out = srv.release();
  return AR_OK;
}

void ar_server_destroy(ar_server *srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto &s : srv->slots)
    if (s->worker.joinable()) s->worker.join();
  for (auto &s : srv->slots) {
    ar::release_workspace(s->ws);
    if (s->stream) (void)hipStreamDestroy(s->stream);
  }
  delete srv;
}

int ar_server_add_scene(ar_server *srv, const ar_scene *scene, int32_t *scene_id) {
  if (!srv || !scene || !scene_id) return ar::fail(AR_E_INVALID, "server, scene or scene_id is NULL");
  std::lock_guard<std::mutex> lk(srv->mu);
  *scene_id = (int32_t)srv->scenes.size();
  srv->scenes.push_back(scene);
  srv->density.push_back(ar::Density{});
  srv->density_rot.push_back(ar::Density{});
  srv->density_pix.push_back(0.0);
  srv->density_rot_pix.push_back(0.0);
  return AR_OK;
}

int ar_server_submit(ar_server *srv, int32_t scene_id, const ar_intrinsics *intr, const ar_pose_box *box,
                     const ar_options *opts, float *lo_rgb, float *hi_rgb, int64_t *ticket) {
  if (!srv || !ticket) return ar::fail(AR_E_INVALID, "server or ticket is NULL");
  const ar_scene *scene = nullptr;
  ar::Density dens, dens_rot;
  double pix = 0.0, pix_rot = 0.0;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (scene_id < 0 || scene_id >= (int32_t)srv->scenes.size())
      return ar::fail(AR_E_INVALID, "unknown scene id %d", scene_id);
    scene = srv->scenes[scene_id];
    dens = srv->density[scene_id];
    dens_rot = srv->density_rot[scene_id];
    pix = srv->density_pix[scene_id];
    pix_rot = srv->density_rot_pix[scene_id];
  }
  int rc = ar::validate_box(box);
  if (rc) return rc;
  auto q = std::make_shared<Query>();
  rc = ar::make_params(scene, intr, opts, q->prm);
  if (rc) return rc;
  if (opts) q->opts = *opts;
  rc = ar::check_outputs(lo_rgb, hi_rgb);
  if (rc) return rc;
  rc = ar::render_vars(scene, box, &q->rotates, &q->P);
  if (rc) return rc;
  if (!q->rotates && q->P > 3) return ar::fail(AR_E_INVALID, "more than 3 translation variables");
  q->scene = scene_id;
  q->box = *box;
  q->lo = lo_rgb;
  q->hi = hi_rgb;
  // the scene's last density, its pairs per Gaussian scaled to this image (a Gaussian
  // covers a number of pixels proportional to the image's at a fixed field of view)
  ar::Density d = q->rotates ? dens_rot : dens;
  const double dpix = q->rotates ? pix_rot : pix;
  if (dpix > 0.0) d.pairs_per_item *= (double)q->prm.width * q->prm.height / dpix;
  q->est = ar::query_bytes(scene, q->prm, q->P, q->rotates, 1, d);
  q->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return ar::fail(AR_E_INVALID, "server is shutting down");
    q->ticket = srv->next_ticket++;
    srv->records[q->ticket] = q;
    srv->queue.push_back(q);
    ++srv->submitted;
    *ticket = q->ticket;
  }
  srv->cv_work.notify_all();
  return AR_OK;
}

int ar_server_wait(ar_server *srv, int64_t ticket, int32_t block, ar_query_result *out) {
  if (!srv || !out) return ar::fail(AR_E_INVALID, "server or out is NULL");
  memset(out, 0, sizeof(*out));
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->records.find(ticket);
  if (it == srv->records.end()) return ar::fail(AR_E_INVALID, "unknown or already collected ticket %lld", (long long)ticket);
  std::shared_ptr<Query> q = it->second;
  if (q->status == AR_PENDING) {
    if (!block) {
      out->status = AR_PENDING;
      return AR_PENDING;
    }
    srv->cv_done.wait(lk, [&] { return q->status != AR_PENDING; });
  }
  out->status = q->status;
  out->slot = q->slot;
  out->queue_ms = ms_between(q->t_submit, q->t_start);
  out->latency_ms = ms_between(q->t_submit, q->t_end);
  out->stats = q->stats;
  out->est_bytes = q->est;
  out->ws_bytes = q->ws_bytes;
  out->batched = q->batched;
  strncpy(out->error, q->error.c_str(), sizeof(out->error) - 1);
  srv->records.erase(ticket);
  if (q->status != AR_OK) return ar::fail(q->status, "%s", q->error.c_str());
  return AR_OK;
}

int ar_server_report(ar_server *srv, ar_server_stats *out) {
  if (!srv || !out) return ar::fail(AR_E_INVALID, "server or out is NULL");
  memset(out, 0, sizeof(*out));
  std::lock_guard<std::mutex> lk(srv->mu);
  out->submitted = srv->submitted;
  out->completed = srv->completed;
  out->failed = srv->failed;
  out->slots = (int32_t)srv->slots.size();
  out->peak_inflight = srv->peak_inflight;
  std::vector<double> v = srv->latencies;
  if (!v.empty()) {
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
      const double r = p * (double)(v.size() - 1);
      const size_t i = (size_t)r;
      const double f = r - (double)i;
      return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
    };
    out->p50_ms = pct(0.50);
    out->p99_ms = pct(0.99);
    double s = 0.0;
    for (double x : v) s += x;
    out->mean_ms = s / (double)v.size();
  }
  out->busy_s = srv->busy_s + (srv->inflight > 0 ? std::chrono::duration<double>(Clock::now() - srv->busy_since).count()
                                                 : 0.0);
  out->hbm_budget = srv->budget;
  out->peak_bytes = srv->peak_bytes;
  out->pairs = srv->pairs;
  out->releases = srv->releases;
  out->shared_launches = srv->shared_launches;
  out->shared_queries = srv->shared_queries;
  return AR_OK;
}

}  // extern "C"
