// Serving loop: continuous batching of periodic structures onto one device.
//
// Requests (one periodic structure each) enter a FIFO queue.  Each of n worker
// threads owns a HIP stream and an evaluation context that shares the model.  A
// free worker takes requests from the head of the queue while they fit its
// admission limits -- an atom cap derived from its slice of the HBM budget and the
// observed device bytes per atom, and a cap on structures per batch -- packs them
// into one graph (structures never exchange edges), evaluates E, F and virial, and
// completes every request of the batch.  Requests that arrive while other batches
// are on the device join the next batch of whichever worker frees up first, so
// batches of different workers overlap on the device.  A batch that still runs out
// of its budget is split in half and retried; a single structure that cannot fit
// completes with SN_ENOMEM.  A request is validated at submit (known species, finite
// positions and cell, nonzero cell volume); a batch that fails on what only the device
// finds (two atoms at one position, an unsupported geometry) is re-run one structure at
// a time, so only the offending request fails and every other result is the one it
// would get alone.
#include <cmath>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "sn.h"

namespace {

struct Request {
  uint64_t ticket = 0;
  int64_t n = 0;
  std::vector<double> pos;
  std::vector<int32_t> Z;
  double cell[9];
  double* atom_energy = nullptr;
  double* forces = nullptr;
  double t_submit = 0;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct sn_server {
  const sn_model_t* model = nullptr;
  int device = 0;
  int precision = SN_FP32;
  size_t slice = 0;  // HBM bytes per worker (0 = no cap)
  int64_t max_batch_atoms = 0;
  int max_batch_structures = 0;
  bool known_z[128] = {};  // atomic numbers of the model's species table
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::unique_ptr<Request>> queue;
  std::deque<sn_result_t> done;
  bool stop = false;
  uint64_t next_ticket = 1;
  int live_workers = 0;
  int64_t in_flight = 0;  // requests taken by workers and not yet completed
  // warm-up: every worker evaluates warm_req once per generation (results dropped)
  uint64_t warm_gen = 0;
  std::vector<uint64_t> warm_seen;
  std::unique_ptr<Request> warm_req;
  int warm_left = 0;
  int warm_status = SN_OK;
  std::vector<std::thread> threads;
  std::string err;

  double now() const { return std::chrono::duration<double>(Clock::now() - t0).count(); }
  void worker(int w);
  void warm_done(int w, int status);  // called with mu held
};

void sn_server::warm_done(int w, int status) {
  if (warm_seen[w] == warm_gen) return;
  warm_seen[w] = warm_gen;
  if (status != SN_OK && warm_status == SN_OK) warm_status = status;
  if (--warm_left == 0) cv_done.notify_all();
}

namespace {

// Device bytes per atom for admission before any batch has been measured: an
// upper estimate for dense condensed-phase cells under a five-block l <= 2 model.
constexpr double kInitialBytesPerAtom = 96.0 * 1024.0;

// results of batch[first .. first + count) (e and w indexed from 0 for that range)
void complete(sn_server* s, std::vector<std::unique_ptr<Request>>& batch, size_t first,
              size_t count, int status, const std::vector<double>& e,
              const std::vector<double>& w, double t_start, double t_end, int64_t atoms) {
  std::lock_guard<std::mutex> lk(s->mu);
  for (size_t k = 0; k < count; ++k) {
    const Request& q = *batch[first + k];
    sn_result_t r;
    std::memset(&r, 0, sizeof(r));
    r.ticket = q.ticket;
    r.status = status;
    if (status == SN_OK) {
      r.energy = e[k];
      for (int a = 0; a < 9; ++a) r.virial[a] = w[9 * k + a];
    }
    r.t_submit = q.t_submit;
    r.t_start = t_start;
    r.t_done = t_end;
    r.batch_structures = (int)count;
    r.batch_atoms = atoms;
    s->done.push_back(r);
  }
  s->in_flight -= (int64_t)count;
  s->cv_done.notify_all();
}

// host-side checks of one request (what a batch mate must not be able to fail)
bool valid_request(const sn_server* s, const sn_request_t* q) {
  for (int64_t i = 0; i < q->n; ++i) {
    const int z = q->Z[i];
    if (z < 0 || z >= 128 || !s->known_z[z]) return false;
  }
  for (int64_t i = 0; i < 3 * q->n; ++i)
    if (!std::isfinite(q->pos[i])) return false;
  for (int k = 0; k < 9; ++k)
    if (!std::isfinite(q->cell[k])) return false;
  const double* H = q->cell;
  const double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                     H[2] * (H[3] * H[7] - H[4] * H[6]);
  return std::isfinite(det) && std::fabs(det) > 1e-6;
}

}  // namespace

void sn_server::worker(int w) {
  hipStream_t stream = nullptr;
  sn_ctx_t* ctx = nullptr;
  bool ok = hipSetDevice(device) == hipSuccess &&
            hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
            sn_ctx_create(model, device, stream, slice, precision, 0.0, nullptr, &ctx) == SN_OK;
  size_t base = 0;
  if (ok) sn_ctx_memory(ctx, &base);
  size_t high_water = base;
  double bytes_per_atom = kInitialBytesPerAtom;
  int64_t atom_cap = max_batch_atoms;  // lowered after a batch ran out of memory
  std::vector<std::unique_ptr<Request>> batch;
  std::vector<int64_t> off;
  std::vector<double> pos, cells, e, vir, ae, f;
  std::vector<int32_t> Z;
  while (ok) {
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_work.wait(lk, [&] { return stop || !queue.empty() || warm_seen[w] != warm_gen; });
      if (stop) break;
      if (warm_seen[w] != warm_gen) {
        // warm-up: allocate this worker's workspace and load its kernels for a request of
        // this size before traffic arrives
        const Request* r = warm_req.get();
        lk.unlock();
        const int64_t o1[2] = {0, r->n};
        std::vector<double> e1(1), w1(9), ae1((size_t)r->n), f1(3 * (size_t)r->n);
        const int st = sn_compute_batch(ctx, 1, o1, r->pos.data(), r->Z.data(), r->cell, e1.data(),
                                        ae1.data(), f1.data(), w1.data());
        if (st == SN_OK) {
          size_t used = 0;
          sn_ctx_memory(ctx, &used);
          if (used > high_water) {
            high_water = used;
            bytes_per_atom = std::max(1024.0, (double)(used - base) / (double)r->n);
          }
        }
        lk.lock();
        warm_done(w, st);
        if (st == SN_EHIP) break;
        continue;
      }
      int64_t cap = atom_cap;
      if (slice) {
        const double room = (double)(slice > base ? slice - base : 0) / bytes_per_atom;
        cap = std::min<int64_t>(cap, std::max<int64_t>(1, (int64_t)room));
      }
      int64_t atoms = 0;
      batch.clear();
      while (!queue.empty() && (int)batch.size() < max_batch_structures &&
             (batch.empty() || atoms + queue.front()->n <= cap)) {
        atoms += queue.front()->n;
        batch.push_back(std::move(queue.front()));
        queue.pop_front();
      }
      in_flight += (int64_t)batch.size();
    }
    const int B = (int)batch.size();
    off.assign(B + 1, 0);
    for (int b = 0; b < B; ++b) off[b + 1] = off[b] + batch[b]->n;
    const int64_t n = off[B];
    pos.resize(3 * n);
    Z.resize(n);
    cells.resize(9 * (size_t)B);
    for (int b = 0; b < B; ++b) {
      std::memcpy(&pos[3 * off[b]], batch[b]->pos.data(), sizeof(double) * 3 * batch[b]->n);
      std::memcpy(&Z[off[b]], batch[b]->Z.data(), sizeof(int32_t) * batch[b]->n);
      std::memcpy(&cells[9 * (size_t)b], batch[b]->cell, sizeof(double) * 9);
    }
    e.assign(B, 0.0);
    vir.assign(9 * (size_t)B, 0.0);
    ae.resize(n);
    f.resize(3 * n);
    const double t_start = now();
    const int st = sn_compute_batch(ctx, B, off.data(), pos.data(), Z.data(), cells.data(),
                                    e.data(), ae.data(), f.data(), vir.data());
    const double t_end = now();
    if (st == SN_ENOMEM && B > 1) {
      // return the batch to the head of the queue, in order, and take its first half next
      std::lock_guard<std::mutex> lk(mu);
      for (int b = B - 1; b >= 0; --b) queue.push_front(std::move(batch[b]));
      in_flight -= (int64_t)B;
      atom_cap = off[B / 2];
      cv_work.notify_all();
      continue;
    }
    atom_cap = max_batch_atoms;
    if ((st == SN_EINVAL || st == SN_EUNSUPPORTED) && B > 1) {
      // a structure the device rejected: evaluate each alone, so only that one fails
      bool dead = false;
      for (int b = 0; b < B && !dead; ++b) {
        Request& r = *batch[b];
        const int64_t o1[2] = {0, r.n};
        std::vector<double> e1(1, 0.0), w1(9, 0.0);
        const double t1 = now();
        const int s1 = sn_compute_batch(ctx, 1, o1, r.pos.data(), r.Z.data(), r.cell, e1.data(),
                                        ae.data(), f.data(), w1.data());
        if (s1 == SN_OK) {
          if (r.atom_energy) std::memcpy(r.atom_energy, ae.data(), sizeof(double) * r.n);
          if (r.forces) std::memcpy(r.forces, f.data(), sizeof(double) * 3 * r.n);
        }
        complete(this, batch, (size_t)b, 1, s1, e1, w1, t1, now(), r.n);
        if (s1 == SN_EHIP) {
          // the context is gone: what is left of the batch cannot run here
          std::vector<double> none;
          if (b + 1 < B) complete(this, batch, (size_t)b + 1, (size_t)(B - b - 1), SN_EHIP, none,
                                  none, t1, now(), 0);
          dead = true;
        }
      }
      if (dead) break;
      continue;
    }
    if (st == SN_OK) {
      for (int b = 0; b < B; ++b) {
        Request& r = *batch[b];
        if (r.atom_energy) std::memcpy(r.atom_energy, &ae[off[b]], sizeof(double) * r.n);
        if (r.forces) std::memcpy(r.forces, &f[3 * off[b]], sizeof(double) * 3 * r.n);
      }
      // the workspace only grows when a batch needs more than any before it: then its
      // size over this batch's atoms measures the bytes per atom of such batches
      size_t used = 0;
      sn_ctx_memory(ctx, &used);
      if (used > high_water) {
        high_water = used;
        bytes_per_atom = std::max(1024.0, (double)(used - base) / (double)n);
      }
    }
    complete(this, batch, 0, (size_t)B, st, e, vir, t_start, t_end, n);
    if (st == SN_EHIP) break;  // the context is no longer usable
  }
  if (ctx) sn_ctx_free(ctx);
  if (stream) (void)hipStreamDestroy(stream);
  std::lock_guard<std::mutex> lk(mu);
  --live_workers;
  if (warm_left > 0) warm_done(w, SN_EHIP);
  if (live_workers == 0) {
    // nothing can run the remaining requests: complete them with an error
    while (!queue.empty()) {
      std::vector<std::unique_ptr<Request>> one;
      one.push_back(std::move(queue.front()));
      queue.pop_front();
      sn_result_t r;
      std::memset(&r, 0, sizeof(r));
      r.ticket = one[0]->ticket;
      r.status = SN_EHIP;
      r.t_submit = one[0]->t_submit;
      done.push_back(r);
    }
    cv_done.notify_all();
  }
}

extern "C" {

int sn_server_create(const sn_model_t* model, int device, int n_streams, int precision,
                     size_t hbm_budget, int64_t max_batch_atoms, int max_batch_structures,
                     sn_server_t** out) {
  if (!model || !out || n_streams < 1 || n_streams > 16 || max_batch_atoms < 1 ||
      max_batch_structures < 1)
    return SN_EINVAL;
  if (precision != SN_FP64 && precision != SN_FP32 && precision != SN_BF16) return SN_EINVAL;
  auto s = std::make_unique<sn_server>();
  s->model = model;
  s->device = device;
  s->precision = precision;
  s->slice = hbm_budget / (size_t)n_streams;
  s->max_batch_atoms = max_batch_atoms;
  s->max_batch_structures = max_batch_structures;
  sn_model_info_t info;
  if (sn_model_info(model, &info) != SN_OK) return SN_EINVAL;
  for (int k = 0; k < info.n_species; ++k)
    if (info.species_z[k] >= 0 && info.species_z[k] < 128) s->known_z[info.species_z[k]] = true;
  s->t0 = Clock::now();
  s->live_workers = n_streams;
  s->warm_seen.assign((size_t)n_streams, 0);
  try {
    for (int w = 0; w < n_streams; ++w) s->threads.emplace_back([p = s.get(), w] { p->worker(w); });
  } catch (const std::exception&) {
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    for (auto& t : s->threads) t.join();
    return SN_EINVAL;
  }
  *out = s.release();
  return SN_OK;
}

int sn_server_submit(sn_server_t* s, const sn_request_t* req, uint64_t* ticket) {
  if (!s || !req || !ticket || req->n <= 0 || !req->pos || !req->Z || !req->cell) return SN_EINVAL;
  if (!valid_request(s, req)) return SN_EINVAL;
  auto r = std::make_unique<Request>();
  r->n = req->n;
  try {
    r->pos.assign(req->pos, req->pos + 3 * req->n);
    r->Z.assign(req->Z, req->Z + req->n);
  } catch (const std::exception&) {
    return SN_ENOMEM;
  }
  std::memcpy(r->cell, req->cell, sizeof(double) * 9);
  r->atom_energy = req->atom_energy;
  r->forces = req->forces;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->live_workers == 0) return SN_EHIP;
    if (s->stop) return SN_EBUSY;
    r->ticket = s->next_ticket++;
    r->t_submit = s->now();
    *ticket = r->ticket;
    s->queue.push_back(std::move(r));
  }
  s->cv_work.notify_one();
  return SN_OK;
}

int sn_server_warmup(sn_server_t* s, const sn_request_t* req) {
  if (!s || !req || req->n <= 0 || !req->pos || !req->Z || !req->cell) return SN_EINVAL;
  if (!valid_request(s, req)) return SN_EINVAL;
  auto r = std::make_unique<Request>();
  r->n = req->n;
  try {
    r->pos.assign(req->pos, req->pos + 3 * req->n);
    r->Z.assign(req->Z, req->Z + req->n);
  } catch (const std::exception&) {
    return SN_ENOMEM;
  }
  std::memcpy(r->cell, req->cell, sizeof(double) * 9);
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->live_workers == 0) return SN_EHIP;
  if (s->stop || s->warm_left > 0) return SN_EBUSY;
  s->warm_req = std::move(r);
  s->warm_status = SN_OK;
  ++s->warm_gen;
  // workers that already exited never see this generation
  s->warm_left = s->live_workers;
  s->cv_work.notify_all();
  s->cv_done.wait(lk, [&] { return s->warm_left <= 0; });
  s->warm_req.reset();
  return s->warm_status;
}

int sn_server_poll(sn_server_t* s, sn_result_t* out, int max, int timeout_ms, int* n_out) {
  if (!s || !out || max < 1 || !n_out) return SN_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->done.empty() && timeout_ms != 0) {
    auto pred = [&] { return !s->done.empty(); };
    if (timeout_ms < 0) s->cv_done.wait(lk, pred);
    else s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
  }
  int k = 0;
  while (k < max && !s->done.empty()) {
    out[k++] = s->done.front();
    s->done.pop_front();
  }
  *n_out = k;
  return SN_OK;
}

int sn_server_pending(sn_server_t* s, int64_t* queued, int64_t* running) {
  if (!s) return SN_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  if (queued) *queued = (int64_t)s->queue.size();
  if (running) *running = s->in_flight;
  return SN_OK;
}

void sn_server_free(sn_server_t* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& t : s->threads) t.join();
  delete s;
}

}  // extern "C"
