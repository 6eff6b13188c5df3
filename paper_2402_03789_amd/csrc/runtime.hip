// libsn host runtime: weights file, contexts, device workspace, and the
// orchestration of one energy/force/virial evaluation on one subdomain with
// a ghost shell (paper sections 2-3), plus the C ABI of include/sn.h.
//
// Evaluation order (paper Fig 3a):
//   graph build (wrap, bins, ghost shell, receiver CSR, sender CSR)
//   edge basis (Y, rho)
//   for t = 1..T:  Lin1 (+ ghost refresh for t >= 2), Linsc, radial MLP,
//                  tensor-product convolution, Lin2, gate
//   readout, energy sum (eq 1)
//   for t = T..1:  gate adjoint, Lin2^T, tensor-product adjoint (dw, per-edge
//                  dx, dY), MLP adjoint (drho); for t >= 2: sender sums,
//                  ghost fold, Lin1^T + Linsc^T (eq 8)
//   edge gradients g_e (eq 5 summed over blocks), forces (eq 6) with the
//   ghost force fold, virial W = -sum_e d_e (x) g_e.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "kernels.h"
#include "json.h"
#include "cg_tables.h"
#include "sn.h"

namespace {

using namespace sn;

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct ArgError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct MemError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct UnsupportedError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
// the static scratch of sn_compute_noalloc is too small for the request
struct ScratchError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      throw HipError(std::string(#expr) + ": " + hipGetErrorString(e_));               \
  } while (0)

thread_local std::string g_load_error;

struct LayerDesc {
  bool last = false;
  std::vector<int> ins, outs;
  std::vector<std::array<int, 3>> paths;
  int P = 0;
  int gmul[kNumL] = {};
  int mid[kNumL] = {};
  IrrepLayout hin{}, yl{}, ml{}, hout{};
  TPLayer tp{};
  int64_t w_lin1[kNumL] = {-1, -1, -1, -1}, w_linsc[kNumL] = {-1, -1, -1, -1},
          w_lin2[kNumL] = {-1, -1, -1, -1};
  int64_t w_mlp[3] = {-1, -1, -1};
};

// channels per degree (kNumL entries, zero where absent)
IrrepLayout make_layout(const int* mul) {
  IrrepLayout L{};
  int off = 0;
  for (int l = 0; l < kNumL; ++l) {
    L.mul[l] = mul[l];
    L.off[l] = off;
    off += (2 * l + 1) * L.mul[l];
  }
  L.width = off;
  return L;
}
IrrepLayout scalar_layout(int c) {
  const int mul[kNumL] = {c, 0, 0, 0};
  return make_layout(mul);
}

RowMap rows_of(const IrrepLayout& L, int l) {
  return RowMap{2 * l + 1, L.mul[l], (int64_t)L.width, (int64_t)L.off[l]};
}

}  // namespace

struct sn_model {
  int T = 0, lmax = 0, lsh = 0, nb = 8, hidden = 64, p = 6;
  int muls[kNumL] = {};
  double rc = 0, kavg = 1, sigma = 1, act = 1;
  std::vector<int> species;
  std::vector<double> shift;
  std::vector<double> flat;
  std::map<std::string, std::pair<int64_t, std::vector<int>>> tensors;
  std::vector<LayerDesc> layers;
  std::vector<double> readout_v;
  int lut[128];
  int64_t n_params = 0;

  int64_t off(const std::string& name, std::vector<int> shape) const {
    auto it = tensors.find(name);
    if (it == tensors.end()) throw ArgError("weights file lacks tensor " + name);
    if (it->second.second != shape) {
      std::ostringstream o;
      o << "tensor " << name << " has the wrong shape";
      throw ArgError(o.str());
    }
    return it->second.first;
  }
};

namespace {

void build_layers(sn_model& m) {
  const int C0 = m.muls[0];
  const IrrepLayout feat = make_layout(m.muls);
  for (int t = 0; t < m.T; ++t) {
    LayerDesc L;
    L.last = (t == m.T - 1);
    if (t == 0) L.ins = {0};
    else for (int l = 0; l <= m.lmax; ++l) if (m.muls[l] > 0) L.ins.push_back(l);
    if (L.last) L.outs = {0};
    else for (int l = 0; l <= m.lmax; ++l) if (m.muls[l] > 0) L.outs.push_back(l);
    for (int l1 : L.ins)
      for (int l2 = 0; l2 <= m.lsh; ++l2)
        for (int l3 = std::abs(l1 - l2); l3 <= std::min(l1 + l2, m.lmax); ++l3)
          if (std::find(L.outs.begin(), L.outs.end(), l3) != L.outs.end())
            L.paths.push_back({l1, l2, l3});
    for (auto& pth : L.paths) L.P += m.muls[pth[0]];
    for (int l : L.outs) {
      if (L.last) L.gmul[l] = C0;
      else L.gmul[l] = (l == 0) ? (m.muls[0] + m.muls[1] + m.muls[2] + m.muls[3]) : m.muls[l];
    }
    for (auto& pth : L.paths) L.mid[pth[2]] += m.muls[pth[0]];
    L.hin = (t == 0) ? scalar_layout(C0) : feat;
    L.yl = make_layout(L.gmul);
    L.ml = make_layout(L.mid);
    L.hout = L.last ? scalar_layout(C0) : feat;
    // weights
    for (int l : L.ins) {
      const int mu = m.muls[l];
      L.w_lin1[l] = m.off("l" + std::to_string(t) + ".lin1." + std::to_string(l), {mu, mu});
      if (L.gmul[l] > 0)
        L.w_linsc[l] = m.off("l" + std::to_string(t) + ".linsc." + std::to_string(l), {mu, L.gmul[l]});
    }
    L.w_mlp[0] = m.off("l" + std::to_string(t) + ".mlp.0", {m.nb, m.hidden});
    L.w_mlp[1] = m.off("l" + std::to_string(t) + ".mlp.1", {m.hidden, m.hidden});
    L.w_mlp[2] = m.off("l" + std::to_string(t) + ".mlp.2", {m.hidden, L.P});
    for (int l : L.outs)
      L.w_lin2[l] = m.off("l" + std::to_string(t) + ".lin2." + std::to_string(l), {L.mid[l], L.gmul[l]});
    // tensor-product description
    TPLayer& tp = L.tp;
    tp.lmax = m.lmax;
    tp.lsh = m.lsh;
    tp.scalar_only = L.last;
    tp.xin = L.hin;
    tp.P = L.P;
    tp.Dm = L.ml.width;
    tp.NY = (m.lsh + 1) * (m.lsh + 1);
    int woff = 0;
    int kfill[kNumL] = {};
    for (int l1 = 0; l1 < kNumL; ++l1) {
      tp.woff[l1] = woff;
      int pi = 0;
      for (auto& pth : L.paths) {
        if (pth[0] != l1) continue;
        const int l3 = pth[2];
        tp.mo[l1][pi] = L.ml.off[l3] + kfill[l3];
        tp.mw[l1][pi] = L.mid[l3];
        kfill[l3] += m.muls[l1];
        woff += m.muls[l1];
        ++pi;
      }
    }
    tp.n_tasks = 0;
    for (int l1 : L.ins) {
      const int mu = m.muls[l1];
      int cpt = 1;
      while (cpt < mu && cpt < 64) cpt <<= 1;
      for (int u0 = 0; u0 < mu; u0 += cpt) {
        if (tp.n_tasks >= 16) throw ArgError("too many channel tasks");
        tp.tasks[tp.n_tasks++] = TPTask{l1, u0, cpt};
      }
    }
    m.layers.push_back(L);
  }
}

std::unique_ptr<sn_model> load_model(const char* path) {
  std::ifstream f(path, std::ios::binary);
  if (!f) throw ArgError(std::string("cannot open ") + path);
  char magic[8];
  f.read(magic, 8);
  if (!f || std::memcmp(magic, "SNW1\0\0\0\0", 8) != 0) throw ArgError("not an SNW1 weights file");
  uint64_t hlen = 0;
  f.read(reinterpret_cast<char*>(&hlen), 8);
  if (!f || hlen > (1u << 26)) throw ArgError("bad header length");
  std::string hdr(hlen, ' ');
  f.read(&hdr[0], (std::streamsize)hlen);
  if (!f) throw ArgError("truncated header");
  Json j = JsonParser(hdr).parse();
  auto m = std::make_unique<sn_model>();
  const Json& c = j.at("config");
  m->T = c.at("n_layers").integer();
  const auto& muls = c.at("muls").array();
  if (muls.empty() || muls.size() > (size_t)kNumL) throw UnsupportedError("l_max must be 0..3");
  for (size_t l = 0; l < muls.size(); ++l) m->muls[l] = muls[l].integer();
  m->lmax = (int)muls.size() - 1;
  m->lsh = c.at("l_sh").integer();
  m->rc = c.at("r_cut").number();
  m->nb = c.at("n_basis").integer();
  m->hidden = c.at("hidden").integer();
  m->p = c.at("envelope_p").integer();
  m->kavg = c.at("k_avg").number();
  m->sigma = c.at("sigma").number();
  m->act = c.at("act_scale").number();
  if (c.has("gate") && c.at("gate").string() != "silu") throw UnsupportedError("only SiLU gates");
  for (auto& z : c.at("species").array()) m->species.push_back(z.integer());
  for (auto& v : c.at("shift").array()) m->shift.push_back(v.number());
  if (m->T < 1 || m->rc <= 0 || m->species.empty() || m->species.size() > 128 ||
      m->shift.size() != m->species.size())
    throw ArgError("invalid model configuration");
  if (m->nb != 8 || m->hidden != 64) throw UnsupportedError("radial MLP must be 8 -> 64 -> 64");
  if (!((m->lmax == 1 && m->lsh == 1) || (m->lmax == 2 && m->lsh == 2) ||
        (m->lmax == 3 && m->lsh == 3)))
    throw UnsupportedError("supported (l_max, l_sh): (1, 1), (2, 2) and (3, 3)");
  for (int l = 0; l < kNumL; ++l) {
    if (m->muls[l] % 4 != 0) throw UnsupportedError("channel counts must be multiples of 4");
    if (m->muls[l] < 0 || m->muls[l] > 128) throw UnsupportedError("at most 128 channels per degree");
  }
  std::fill(m->lut, m->lut + 128, -1);
  for (size_t s = 0; s < m->species.size(); ++s) {
    int z = m->species[s];
    if (z < 0 || z >= 128) throw ArgError("species out of range");
    m->lut[z] = (int)s;
  }
  int64_t total = 0;
  for (auto& t : j.at("tensors").array()) {
    std::vector<int> shape;
    int64_t cnt = 1;
    for (auto& d : t.at("shape").array()) { shape.push_back(d.integer()); cnt *= d.integer(); }
    int64_t off = (int64_t)t.at("offset").number();
    if (off % 8 != 0) throw ArgError("misaligned tensor");
    m->tensors[t.at("name").string()] = {off / 8, shape};
    total = std::max(total, off / 8 + cnt);
    m->n_params += cnt;
  }
  m->flat.resize((size_t)total);
  f.read(reinterpret_cast<char*>(m->flat.data()), (std::streamsize)(total * 8));
  if (!f) throw ArgError("truncated weights data");
  const int C0 = m->muls[0];
  m->off("embed", {(int)m->species.size(), C0});
  int64_t r0 = m->off("readout.0", {C0, C0 / 2});
  int64_t r1 = m->off("readout.1", {C0 / 2, 1});
  m->readout_v.assign(C0, 0.0);
  for (int a = 0; a < C0; ++a)
    for (int k = 0; k < C0 / 2; ++k) m->readout_v[a] += m->flat[r0 + a * (C0 / 2) + k] * m->flat[r1 + k];
  build_layers(*m);
  return m;
}

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
};

}  // namespace

struct sn_ctx {
  const sn_model* m = nullptr;
  int device = 0;
  hipStream_t stream = nullptr;
  // device allocations come from the caller's allocator when one was given at creation
  sn_allocator_t alloc{nullptr, nullptr, nullptr};
  std::map<void*, size_t> weight_blocks;  // weight buffers and their sizes (for free)
  size_t budget = 0;
  int precision = SN_FP32;
  double skin = 0;
  std::string err;
  std::map<std::string, Buf> bufs;
  size_t used = 0;
  bool dead = false;
  // device weights (float64 copy and float32 copy)
  void* d_w = nullptr;
  void* d_w32 = nullptr;
  // per block: the radial MLP's output weights as 64-column panels (wc_panels)
  void* d_wpan = nullptr;
  std::vector<const bf16_t*> wc_pan16, wc_panT16, wc_panT3, wc_pan3;
  size_t weight_bytes = 0;
  double* d_v = nullptr;
  double* d_shift = nullptr;
  // graph state
  int N = 0, G = 0;
  int64_t E = 0, NP = 0;  // directed edges, undirected pairs
  // structures of the packed graph, each split into domains[0] x domains[1] x domains[2]
  // spatial subdomains (regions, R = B x subdomains), each with its own ghost shell
  int B = 0;
  int R = 0;
  int domains[3] = {1, 1, 1};
  std::vector<int64_t> atom_off;   // B + 1 atom offsets (input order = packed local order)
  std::vector<int64_t> edge_off;   // B + 1 edge offsets (edges are receiver-contiguous)
  std::vector<StructParams> sp;    // per-structure geometry (host copy)
  int nbins = 0;
  int n_echunk = 0, n_vchunk = 0;
  // A list built out to r_c + skin is evaluated over its pairs inside r_c only: after every
  // position refresh the built list (kept as full_*) is compacted into the arrays the
  // evaluation reads (see launch_compact_active).
  bool compact = true;           // enabled (sn_ctx_set_edge_compaction)
  bool compacted = false;        // the current graph is a compaction of the built list
  int64_t E_built = 0, NP_built = 0;
  std::vector<int> vchunk_host, vfirst_host;  // host copies of the virial chunk table
  bool pending = false;
  bool train = false;       // forwards keep every block's inputs and messages (weight gradients)
  bool fwd_train = false;   // the pending forward kept them
  bool reuse = false;       // keep the graph of the previous call when n and the cell match
  bool have_graph = false;
  // hipGraph replay of the reused-graph evaluation (see sn_ctx_set_capture)
  bool capture = false;
  bool capturing = false;        // launches are being recorded: no timing events
  uint64_t graph_version = 0;    // bumped at every neighbour-list build
  int reuse_runs = 0;            // eager forward calls on the current graph
  bool last_fwd_reused = false;
  hipStream_t cap_stream = nullptr;  // private stream for capture when the context's is null
  struct Replay {
    hipGraphExec_t exec = nullptr;
    uint64_t version = ~0ull;
    const void* key[3] = {nullptr, nullptr, nullptr};
  } rp_fwd, rp_bwd;
  std::vector<double> graph_cells;
  // second stream for the radial MLPs, which depend only on the edge basis (forward) or
  // on their own block's dE/dw (adjoint), so they overlap with the node-feature chain
  hipStream_t aux = nullptr;
  std::vector<hipEvent_t> sync_pool;  // dependency events between the two streams
  size_t sync_next = 0;
  // timing
  std::vector<std::pair<std::string, hipEvent_t>> marks;
  std::vector<std::pair<std::string, std::pair<hipEvent_t, hipEvent_t>>> aux_marks;
  std::vector<std::pair<std::string, double>> timings;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;

  // device memory from the caller's allocator, or hipMalloc; nullptr on failure
  void* dev_alloc(size_t bytes) {
    if (alloc.alloc) return alloc.alloc(alloc.user, bytes, device, stream);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    return p;
  }
  // the caller guarantees that no queued work still uses p
  bool dev_free(void* p, size_t bytes) {
    if (!p) return true;
    if (alloc.free) {
      alloc.free(alloc.user, p, bytes, device, stream);
      return true;
    }
    return hipFree(p) == hipSuccess;
  }
  // a weight buffer (released only by sn_ctx_free)
  void* weight_alloc(size_t bytes) {
    void* p = dev_alloc(bytes);
    if (!p) throw MemError("device allocation failed for the model weights");
    weight_blocks[p] = bytes;
    return p;
  }
  // Fixed-arena mode (sn_compute_noalloc): every buffer is a slice of caller-provided device
  // memory, handed out in request order; growing a buffer moves it to a new slice (its
  // contents are dropped, as when a pool buffer grows).  Nothing is allocated or freed.
  char* arena = nullptr;
  size_t arena_cap = 0, arena_top = 0;
  std::map<std::string, std::pair<size_t, size_t>> arena_slots;  // name -> (offset, bytes)
  void* arena_raw(const std::string& name, size_t bytes) {
    bytes = (std::max<size_t>(bytes, 1) + 255) & ~(size_t)255;
    auto it = arena_slots.find(name);
    if (it != arena_slots.end()) {
      if (bytes <= it->second.second) return arena + it->second.first;
      if (it->second.first + it->second.second == arena_top &&
          it->second.first + bytes <= arena_cap) {  // the newest slice grows in place
        arena_top = it->second.first + bytes;
        it->second.second = bytes;
        return arena + it->second.first;
      }
    }
    if (arena_top + bytes > arena_cap)
      throw ScratchError("the request needs more than the " + std::to_string(arena_cap >> 20) +
                         " MiB static scratch (buffer " + name + " of " +
                         std::to_string(bytes) + " bytes at offset " +
                         std::to_string(arena_top) + ")");
    arena_slots[name] = {arena_top, bytes};
    void* p = arena + arena_top;
    arena_top += bytes;
    return p;
  }
  void* raw(const std::string& name, size_t bytes) {
    if (arena) return arena_raw(name, bytes);
    Buf& b = bufs[name];
    if (bytes <= b.cap) return b.p;
    size_t want = std::max(bytes + bytes / 4, (size_t)256);
    if (budget && used - b.cap + want > budget)
      throw MemError("HBM budget exceeded allocating " + name);
    if (b.p) {
      HIPCHK(hipStreamSynchronize(stream));
      if (aux) HIPCHK(hipStreamSynchronize(aux));
      if (!dev_free(b.p, b.cap)) throw HipError("device free failed for " + name);
      used -= b.cap;
      b.p = nullptr;
      b.cap = 0;
    }
    b.p = dev_alloc(want);
    if (!b.p) throw MemError("device allocation failed for " + name);
    b.cap = want;
    used += want;
    return b.p;
  }
  template <typename T>
  T* get(const std::string& name, int64_t count) {
    return static_cast<T*>(raw(name, (size_t)std::max<int64_t>(count, 1) * sizeof(T)));
  }
  hipEvent_t sync_event() {
    if (sync_next >= sync_pool.size()) {
      hipEvent_t ev;
      HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      sync_pool.push_back(ev);
    }
    return sync_pool[sync_next++];
  }
  // record on `producer`, make `waiter` wait for it; returns the event
  hipEvent_t join(hipStream_t waiter, hipStream_t producer) {
    hipEvent_t ev = sync_event();
    HIPCHK(hipEventRecord(ev, producer));
    HIPCHK(hipStreamWaitEvent(waiter, ev, 0));
    return ev;
  }
  hipEvent_t timing_event() {
    if (event_next >= event_pool.size()) {
      hipEvent_t ev;
      HIPCHK(hipEventCreate(&ev));
      event_pool.push_back(ev);
    }
    return event_pool[event_next++];
  }
  // time one launch sequence on the aux stream (with a single stream, a phase of the
  // stream's own sequence that the next mark ends)
  void aux_begin(const std::string& name) {
    if (capturing) return;
    if (aux == stream) {
      mark(name);
      return;
    }
    hipEvent_t a = timing_event();
    HIPCHK(hipEventRecord(a, aux));
    aux_marks.push_back({name, {a, nullptr}});
  }
  void aux_end() {
    if (capturing || aux == stream) return;
    hipEvent_t b = timing_event();
    HIPCHK(hipEventRecord(b, aux));
    aux_marks.back().second.second = b;
  }
  void mark(const std::string& name) {
    if (capturing) return;
    if (event_next >= event_pool.size()) {
      hipEvent_t ev;
      HIPCHK(hipEventCreate(&ev));
      event_pool.push_back(ev);
    }
    hipEvent_t ev = event_pool[event_next++];
    HIPCHK(hipEventRecord(ev, stream));
    marks.push_back({name, ev});
  }
};

namespace {

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void zero(void* p, size_t bytes, hipStream_t s) {
  int64_t n = (int64_t)(bytes / 4);
  if (n > 0) k_fill_u32<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(static_cast<uint32_t*>(p), n, 0u);
}

template <typename T>
const T* W(const sn_ctx* c, int64_t off);
template <>
const double* W<double>(const sn_ctx* c, int64_t off) {
  return static_cast<const double*>(c->d_w) + off;
}
template <>
const float* W<float>(const sn_ctx* c, int64_t off) {
  return static_cast<const float*>(c->d_w32) + off;
}

// The radial MLP's output weights Wc [hidden x P] of every block, rearranged for the fused
// matrix-core kernels into 64-column panels of 64 x 64 contiguous values, zero past column
// P: bfloat16 [panel][j][c] and [panel][c][j] (BF16 form), and the three bfloat16 parts of
// every value (FP32 form) as [panel][part][c][j] and [panel][part][j][c].
void wc_panels(sn_ctx* c, const std::vector<float>& w32) {
  const sn_model* m = c->m;
  constexpr int H = 64, K = H * H;  // the model's hidden width (checked at load)
  std::vector<size_t> off;
  size_t total = 0;
  for (const LayerDesc& L : m->layers) {
    off.push_back(total);
    total += (size_t)((L.P + H - 1) / H) * K;
  }
  std::vector<bf16_t> h(total), ht(total), h3(3 * total), h3n(3 * total);
  auto widen = [](bf16_t b) { return __builtin_bit_cast(float, (uint32_t)b.u << 16); };
  for (size_t t = 0; t < m->layers.size(); ++t) {
    const LayerDesc& L = m->layers[t];
    const float* wc = w32.data() + L.w_mlp[2];
    for (int pan = 0; pan * H < L.P; ++pan)
      for (int j = 0; j < H; ++j)
        for (int q = 0; q < H; ++q) {
          const int col = pan * H + q;
          const float v = col < L.P ? wc[(size_t)j * L.P + col] : 0.f;
          const size_t b = off[t] + (size_t)pan * K;
          h[b + j * H + q] = sstore<bf16_t>(v);
          ht[b + q * H + j] = sstore<bf16_t>(v);
          // three bfloat16 parts of v (each remainder is exact in float32), [c][j] and [j][c]
          const bf16_t x0 = sstore<bf16_t>(v);
          const float r1 = v - widen(x0);
          const bf16_t x1 = sstore<bf16_t>(r1);
          const bf16_t x2 = sstore<bf16_t>(r1 - widen(x1));
          const size_t b3 = 3 * off[t] + (size_t)pan * 3 * K + q * H + j;
          h3[b3] = x0;
          h3[b3 + K] = x1;
          h3[b3 + 2 * K] = x2;
          const size_t b3n = 3 * off[t] + (size_t)pan * 3 * K + j * H + q;
          h3n[b3n] = x0;
          h3n[b3n + K] = x1;
          h3n[b3n + 2 * K] = x2;
        }
  }
  const size_t bytes = total * 8 * sizeof(bf16_t);
  c->d_wpan = c->weight_alloc(bytes);
  bf16_t* dh = static_cast<bf16_t*>(c->d_wpan);
  bf16_t* dht = dh + total;
  bf16_t* dh3 = dht + total;
  bf16_t* dh3n = dh3 + 3 * total;
  HIPCHK(hipMemcpy(dh, h.data(), total * sizeof(bf16_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dht, ht.data(), total * sizeof(bf16_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dh3, h3.data(), 3 * total * sizeof(bf16_t), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(dh3n, h3n.data(), 3 * total * sizeof(bf16_t), hipMemcpyHostToDevice));
  for (size_t t = 0; t < m->layers.size(); ++t) {
    c->wc_pan16.push_back(dh + off[t]);
    c->wc_panT16.push_back(dht + off[t]);
    c->wc_panT3.push_back(dh3 + 3 * off[t]);
    c->wc_pan3.push_back(dh3n + 3 * off[t]);
  }
  c->weight_bytes += bytes;
}

void upload_weights(sn_ctx* c) {
  const sn_model* m = c->m;
  // SN_SERIAL in the environment keeps every launch on the context's stream (clean
  // per-kernel timings for profiling); otherwise the radial MLPs get a second stream
  const char* serial = std::getenv("SN_SERIAL");
  if (serial && serial[0] && serial[0] != '0') c->aux = c->stream;
  else HIPCHK(hipStreamCreateWithFlags(&c->aux, hipStreamNonBlocking));
  std::vector<float> w32(m->flat.size());
  for (size_t i = 0; i < w32.size(); ++i) w32[i] = (float)m->flat[i];
  c->d_w = c->weight_alloc(m->flat.size() * sizeof(double));
  HIPCHK(hipMemcpy(c->d_w, m->flat.data(), m->flat.size() * sizeof(double), hipMemcpyHostToDevice));
  c->d_w32 = c->weight_alloc(w32.size() * sizeof(float));
  HIPCHK(hipMemcpy(c->d_w32, w32.data(), w32.size() * sizeof(float), hipMemcpyHostToDevice));
  c->d_v = static_cast<double*>(c->weight_alloc(m->readout_v.size() * sizeof(double)));
  HIPCHK(hipMemcpy(c->d_v, m->readout_v.data(), m->readout_v.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  c->d_shift = static_cast<double*>(c->weight_alloc(m->shift.size() * sizeof(double)));
  HIPCHK(hipMemcpy(c->d_shift, m->shift.data(), m->shift.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  c->weight_bytes = m->flat.size() * (sizeof(double) + sizeof(float)) +
                    (m->readout_v.size() + m->shift.size()) * sizeof(double);
  wc_panels(c, w32);
}

// ------------------------------------------------------------------ graph build
void inv3(const double* H, double* Hi, double* det_out) {
  double det = H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
               H[2] * (H[3] * H[7] - H[4] * H[6]);
  *det_out = det;
  double id = 1.0 / det;
  Hi[0] = (H[4] * H[8] - H[5] * H[7]) * id;
  Hi[1] = (H[2] * H[7] - H[1] * H[8]) * id;
  Hi[2] = (H[1] * H[5] - H[2] * H[4]) * id;
  Hi[3] = (H[5] * H[6] - H[3] * H[8]) * id;
  Hi[4] = (H[0] * H[8] - H[2] * H[6]) * id;
  Hi[5] = (H[2] * H[3] - H[0] * H[5]) * id;
  Hi[6] = (H[3] * H[7] - H[4] * H[6]) * id;
  Hi[7] = (H[1] * H[6] - H[0] * H[7]) * id;
  Hi[8] = (H[0] * H[4] - H[1] * H[3]) * id;
}

// Chunks of a per-structure segmented sum: (structure, begin, end), at most `len` items each,
// plus the first chunk of every structure (B + 1 entries).
struct SegChunks {
  std::vector<int> chunk;  // 3 ints per chunk
  std::vector<int> first;  // B + 1
};
SegChunks make_chunks(const std::vector<int64_t>& off, int64_t len) {
  SegChunks sc;
  const int B = (int)off.size() - 1;
  for (int b = 0; b < B; ++b) {
    sc.first.push_back((int)(sc.chunk.size() / 3));
    int64_t a = off[b];
    do {
      const int64_t e = std::min(off[b + 1], a + len);
      sc.chunk.push_back(b);
      sc.chunk.push_back((int)a);
      sc.chunk.push_back((int)e);
      a = e;
    } while (a < off[b + 1]);
  }
  sc.first.push_back((int)(sc.chunk.size() / 3));
  return sc;
}

// One region: the fractional box [lo, hi) of a cell, its shell half-width and bin grid.
StructParams make_struct(const double* cell, double reach, const double* lo, const double* hi) {
  StructParams P{};
  for (int i = 0; i < 9; ++i) {
    if (!std::isfinite(cell[i])) throw ArgError("cell has non-finite entries");
    P.H[i] = cell[i];
  }
  double det;
  inv3(P.H, P.Hinv, &det);
  const double* a = P.H;
  double cr[3][3];
  for (int k = 0; k < 3; ++k) {
    const double* u = a + 3 * ((k + 1) % 3);
    const double* v = a + 3 * ((k + 2) % 3);
    cr[k][0] = u[1] * v[2] - u[2] * v[1];
    cr[k][1] = u[2] * v[0] - u[0] * v[2];
    cr[k][2] = u[0] * v[1] - u[1] * v[0];
  }
  const double vol = std::fabs(det);
  if (!(vol > 1e-6)) throw ArgError("singular cell");
  BinGrid& g = P.g;
  for (int k = 0; k < 3; ++k) {
    double w = vol / std::sqrt(cr[k][0] * cr[k][0] + cr[k][1] * cr[k][1] + cr[k][2] * cr[k][2]);
    g.delta[k] = reach / w;
    g.lo[k] = lo[k];
    g.hi[k] = hi[k];
    double span = (hi[k] - lo[k]) + 2.0 * g.delta[k];
    g.bw[k] = std::max(g.delta[k], span / 256.0);
    g.nb[k] = std::max(1, (int)std::ceil(span / g.bw[k] - 1e-12));
    g.nimg[k] = (int)std::ceil(g.delta[k]) + 1;
  }
  return P;
}

// Geometry of B structures: cells[b*9 .. b*9+8]; offsets[b] .. offsets[b+1] are the atoms
// of structure b.  Uploads the per-structure table and the structure id of every atom.
void setup_cells(sn_ctx* c, int B, const int64_t* offsets, const double* cells) {
  if (B < 1) throw ArgError("no structures");
  c->B = B;
  c->atom_off.assign(offsets, offsets + B + 1);
  const int* nd = c->domains;
  const int D = nd[0] * nd[1] * nd[2];
  c->R = B * D;
  c->sp.resize(c->R);
  int64_t bins = 0;
  const double reach = c->m->rc + c->skin;
  for (int b = 0; b < B; ++b) {
    if (offsets[b + 1] <= offsets[b]) throw ArgError("empty structure in batch");
    for (int dx = 0; dx < nd[0]; ++dx)
      for (int dy = 0; dy < nd[1]; ++dy)
        for (int dz = 0; dz < nd[2]; ++dz) {
          const int r = b * D + (dx * nd[1] + dy) * nd[2] + dz;
          const double lo[3] = {(double)dx / nd[0], (double)dy / nd[1], (double)dz / nd[2]};
          const double hi[3] = {(double)(dx + 1) / nd[0], (double)(dy + 1) / nd[1],
                                (double)(dz + 1) / nd[2]};
          StructParams& P = c->sp[r];
          P = make_struct(cells + 9 * b, reach, lo, hi);
          P.bin_base = (int)bins;
          P.first_region = b * D;
          for (int a = 0; a < 3; ++a) P.ndom[a] = nd[a];
          bins += (int64_t)P.g.nb[0] * P.g.nb[1] * P.g.nb[2];
          if (bins > (1 << 26)) throw UnsupportedError("bin grid too large");
        }
  }
  c->nbins = (int)bins;
  const int64_t N = offsets[B];
  StructParams* dsp = c->get<StructParams>("struct_params", c->R);
  HIPCHK(hipMemcpyAsync(dsp, c->sp.data(), sizeof(StructParams) * c->R, hipMemcpyHostToDevice,
                        c->stream));
  // every atom starts with its structure's first region; the wrap kernel picks its own
  std::vector<int> sid((size_t)N);
  for (int b = 0; b < B; ++b)
    for (int64_t i = offsets[b]; i < offsets[b + 1]; ++i) sid[i] = b * D;
  int* dsid = c->get<int>("sid_orig", N);
  HIPCHK(hipMemcpyAsync(dsid, sid.data(), sizeof(int) * N, hipMemcpyHostToDevice, c->stream));
  std::vector<int> offs(offsets, offsets + B + 1);
  int* doff = c->get<int>("struct_atom_off", B + 1);
  HIPCHK(hipMemcpyAsync(doff, offs.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, c->stream));
  SegChunks ec = make_chunks(c->atom_off, 2048);
  c->n_echunk = (int)(ec.chunk.size() / 3);
  int* dch = c->get<int>("echunks", 3 * c->n_echunk);
  int* dfi = c->get<int>("efirst", B + 1);
  HIPCHK(hipMemcpyAsync(dch, ec.chunk.data(), sizeof(int) * ec.chunk.size(), hipMemcpyHostToDevice,
                        c->stream));
  HIPCHK(hipMemcpyAsync(dfi, ec.first.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, c->stream));
  // the pageable sources above must stay valid until the copies ran
  HIPCHK(hipStreamSynchronize(c->stream));
}

__global__ void k_gather_offsets(int B, const int* __restrict__ row_ptr, const int* __restrict__ aoff,
                                 int* __restrict__ eoff) {
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= B) eoff[b] = row_ptr[aoff[b]];
}

// The built list's arrays, kept under full_* while compacted copies are evaluated.
const char* const kListArrays[] = {"row_ptr", "src", "recv", "pidx", "pair_e1", "pair_e2",
                                   "send_ptr", "send_idx", "struct_edge_off"};
int64_t list_array_len(const sn_ctx* c, int k) {
  const int64_t N = c->N, NE = c->N + c->G;
  switch (k) {
    case 0: return N + 1;
    case 4: case 5: return c->NP;
    case 6: return NE + 1;
    case 8: return c->B + 1;
    default: return c->E;
  }
}
void keep_built_list(sn_ctx* c) {
  for (int k = 0; k < 9; ++k) {
    const int64_t n = list_array_len(c, k);
    const std::string name = kListArrays[k];
    int* dst = c->get<int>("full_" + name, n);
    const int* src = c->get<int>(name, n);
    if (n > 0)
      HIPCHK(hipMemcpyAsync(dst, src, sizeof(int) * n, hipMemcpyDeviceToDevice, c->stream));
  }
  c->E_built = c->E;
  c->NP_built = c->NP;
}

// Compact the built list to the pairs inside r_c at the current positions (pos_ext) and
// make the compacted list the one the evaluation reads.
void compact_list(sn_ctx* c) {
  hipStream_t s = c->stream;
  const int N = c->N, NE = N + c->G, B = c->B;
  const int64_t E = c->E_built, NPr = c->NP_built;
  auto full = [&](const char* name, int64_t n) { return c->get<int>(std::string("full_") + name, n); };
  CompactIn a{E, NPr, N, NE, B,
              full("row_ptr", N + 1), full("src", E), full("recv", E), full("pidx", E),
              full("pair_e1", NPr), full("pair_e2", NPr), full("send_ptr", NE + 1),
              full("send_idx", E), full("struct_edge_off", B + 1),
              c->get<double>("pos_ext", 3 * (int64_t)NE), c->m->rc};
  CompactOut o{c->get<int>("row_ptr", N + 1), c->get<int>("src", E), c->get<int>("recv", E),
               c->get<int>("pidx", E), c->get<int>("pair_e1", E), c->get<int>("pair_e2", E),
               c->get<int>("send_ptr", NE + 1), c->get<int>("send_idx", E),
               c->get<int>("struct_edge_off", B + 1)};
  CompactScratch t{c->get<int>("cmp_active", NPr + 1), c->get<int>("cmp_pscan", NPr + 1),
                   c->get<int>("cmp_keep", E + 1), c->get<int>("cmp_escan", E + 1),
                   c->get<int>("cmp_keep_s", E + 1), c->get<int>("cmp_sscan", E + 1),
                   c->get<int>("cmp_tmp", (int64_t)scan_tmp_ints(std::max(E, NPr) + 1))};
  launch_compact_active(a, o, t, s);
  std::vector<int> h((size_t)B + 3);
  HIPCHK(hipMemcpyAsync(h.data(), o.edge_off, sizeof(int) * (B + 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&h[B + 1], t.escan + E, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&h[B + 2], t.pscan + NPr, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  c->E = h[B + 1];
  c->NP = h[B + 2];
  c->edge_off.assign(h.begin(), h.begin() + B + 1);
  SegChunks vc = make_chunks(c->edge_off, 16384);
  c->vchunk_host.swap(vc.chunk);
  c->vfirst_host.swap(vc.first);
  c->n_vchunk = (int)(c->vchunk_host.size() / 3);
  // from host vectors that live in the context until the next compaction, which waits for
  // this copy before it writes them
  HIPCHK(hipMemcpyAsync(c->get<int>("vchunks", 3 * c->n_vchunk), c->vchunk_host.data(),
                        sizeof(int) * c->vchunk_host.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(c->get<int>("vfirst", B + 1), c->vfirst_host.data(), sizeof(int) * (B + 1),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipGetLastError());
  c->compacted = true;
}

template <typename T>
void build_graph(sn_ctx* c, int N, const double* d_pos, const int* d_spec) {
  hipStream_t s = c->stream;
  const int nbins = c->nbins;
  const StructParams* sp = c->get<StructParams>("struct_params", c->R);
  const int* sid_orig = c->get<int>("sid_orig", N);
  int* rid = c->get<int>("region_orig", N);
  c->N = N;
  int* err = c->get<int>("err", 4);
  zero(err, 16, s);
  double* posw = c->get<double>("posw", 3 * N);
  double* fracw = c->get<double>("fracw", 3 * N);
  int* key = c->get<int>("key", N);
  launch_wrap_bin(N, d_pos, sid_orig, sp, posw, fracw, key, rid, err, s);
  // order local atoms by bin (cell order within each structure) for gather locality
  int* cnt = c->get<int>("bin_count", nbins + 1);
  int* start = c->get<int>("bin_start", nbins + 1);
  int* cursor = c->get<int>("bin_cursor", nbins + 1);
  int64_t scan_max = std::max<int64_t>(nbins, 4 * (int64_t)N + 1024);
  int* tmp = c->get<int>("scan_tmp", (int64_t)scan_tmp_ints(scan_max + 1));
  int* order = c->get<int>("order", N);
  zero(cnt, sizeof(int) * nbins, s);
  zero(cursor, sizeof(int) * nbins, s);
  launch_count_keys(N, key, cnt, s);
  scan_exclusive(cnt, start, nbins, tmp, s);
  launch_scatter_keys(N, key, start, cursor, order, s);
  launch_sort_segments(nbins, start, order, s);
  // local rows
  int* gcount = c->get<int>("ghost_count", N + 1);
  int* gptr = c->get<int>("ghost_ptr", N + 1);
  double* fr_loc = c->get<double>("frac_local", 3 * N);
  double* pos_loc = c->get<double>("pos_local", 3 * N);
  int* spec_loc = c->get<int>("spec_local", N);
  int* sid_loc = c->get<int>("sid_local", N);
  launch_gather_local(N, order, posw, fracw, d_spec, rid, pos_loc, fr_loc, spec_loc, sid_loc, s);
  launch_ghost_count(N, fr_loc, sid_loc, sp, gcount, s);
  scan_exclusive(gcount, gptr, N, tmp, s);
  int hG[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(&hG[0], gptr + N, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&hG[1], err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hG[1] & 1) throw ArgError("non-finite positions");
  const int G = hG[0];
  c->G = G;
  const int NE = N + G;
  double* pos_ext = c->get<double>("pos_ext", 3 * (int64_t)NE);
  double* frac_ext = c->get<double>("frac_ext", 3 * (int64_t)NE);
  int* spec_ext = c->get<int>("spec_ext", NE);
  int* sid_ext = c->get<int>("sid_ext", NE);
  int* owner = c->get<int>("ghost_owner", G);
  int* shift = c->get<int>("ghost_shift", 3 * (int64_t)G);
  HIPCHK(hipMemcpyAsync(pos_ext, pos_loc, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(frac_ext, fr_loc, sizeof(double) * 3 * N, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(spec_ext, spec_loc, sizeof(int) * N, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipMemcpyAsync(sid_ext, sid_loc, sizeof(int) * N, hipMemcpyDeviceToDevice, s));
  launch_ghost_fill(N, fr_loc, pos_loc, spec_loc, sid_ext, sp, gptr, owner, shift, pos_ext,
                    frac_ext, spec_ext, s);
  // bin every extended point
  int* ekey = c->get<int>("ext_key", NE);
  int* cell_items = c->get<int>("cell_items", NE);
  launch_bin_keys(NE, frac_ext, sid_ext, sp, ekey, s);
  zero(cnt, sizeof(int) * nbins, s);
  zero(cursor, sizeof(int) * nbins, s);
  launch_count_keys(NE, ekey, cnt, s);
  scan_exclusive(cnt, start, nbins, tmp, s);
  launch_scatter_keys(NE, ekey, start, cursor, cell_items, s);
  launch_sort_segments(nbins, start, cell_items, s);
  // receiver CSR
  // edges out to r_c + skin, so the list stays complete while atoms move < skin / 2
  const double rc2 = (c->m->rc + c->skin) * (c->m->rc + c->skin);
  int* ecount = c->get<int>("edge_count", N + 1);
  int* row_ptr = c->get<int>("row_ptr", N + 1);
  launch_edge_count(N, pos_ext, frac_ext, sid_ext, sp, start, cell_items, rc2, ecount, err, s);
  scan_exclusive(ecount, row_ptr, N, tmp, s);
  // per-structure edge offsets (receivers of a structure are contiguous)
  const int B = c->B;
  int* eoff = c->get<int>("struct_edge_off", B + 1);
  k_gather_offsets<<<(unsigned)((B + 1 + 255) / 256), 256, 0, s>>>(
      B, row_ptr, c->get<int>("struct_atom_off", B + 1), eoff);
  std::vector<int> hE((size_t)B + 2);
  HIPCHK(hipMemcpyAsync(hE.data(), eoff, sizeof(int) * (B + 1), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&hE[B + 1], err, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hE[B + 1] & 2) throw ArgError("two atoms at the same position (r = 0 pair)");
  c->edge_off.assign(hE.begin(), hE.begin() + B + 1);
  const int64_t E = hE[B];
  c->E = E;
  int* src = c->get<int>("src", E);
  int* recv = c->get<int>("recv", E);
  launch_edge_fill(N, pos_ext, frac_ext, sid_ext, sp, start, cell_items, rc2, row_ptr, src, recv, s);
  // sender CSR over extended rows (local and ghost senders)
  int* scount = c->get<int>("send_count", NE + 1);
  int* sptr = c->get<int>("send_ptr", NE + 1);
  int* scur = c->get<int>("send_cursor", NE + 1);
  int* sidx = c->get<int>("send_idx", E);
  zero(scount, sizeof(int) * NE, s);
  zero(scur, sizeof(int) * NE, s);
  launch_count_keys((int)E, src, scount, s);
  scan_exclusive(scount, sptr, NE, tmp, s);
  launch_scatter_keys((int)E, src, sptr, scur, sidx, s);
  launch_sort_segments(NE, sptr, sidx, s);
  // reverse edges and undirected pairs (the radial MLP runs once per pair)
  int* rev = c->get<int>("rev", E);
  int* flag = c->get<int>("pair_flag", E);
  int* fscan = c->get<int>("pair_scan", E + 1);
  int* tmp_e = c->get<int>("scan_tmp_e", (int64_t)scan_tmp_ints(E + 1));
  int* pidx = c->get<int>("pidx", E);
  int* pe1 = c->get<int>("pair_e1", E);
  int* pe2 = c->get<int>("pair_e2", E);
  launch_pairs(E, N, recv, src, row_ptr, owner, shift, rev, flag, fscan, tmp_e, pidx, pe1, pe2, s);
  SegChunks vc = make_chunks(c->edge_off, 16384);
  c->n_vchunk = (int)(vc.chunk.size() / 3);
  int* dvc = c->get<int>("vchunks", 3 * c->n_vchunk);
  int* dvf = c->get<int>("vfirst", B + 1);
  HIPCHK(hipMemcpyAsync(dvc, vc.chunk.data(), sizeof(int) * vc.chunk.size(), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(dvf, vc.first.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, s));
  int hP = 0;
  HIPCHK(hipMemcpyAsync(&hP, fscan + E, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  HIPCHK(hipGetLastError());
  c->NP = hP;
}

// ------------------------------------------------------------------ forward / backward
// T is the per-edge arithmetic type (float64 in the FP64 form, float32 otherwise).  The
// node-state chain -- features h, self-connection and gate input y, the gate, the
// readout input and the backward node gradients -- is NodeT: float64 in the FP64 and
// FP32 forms (the self-connection carries most of each atom's energy through all blocks
// and is the one place where float32 rounding reaches the per-atom energy at the 1e-6
// level), float32 in the BF16 form, whose bfloat16 operands dominate its error.
// S is the storage type of the sender features x that feed the tensor product, the radial
// weights w, the messages M and their gradients dE/dM, dE/dw and the per-edge sender
// gradient rows: T, or bfloat16 in the BF16 form (arithmetic stays in T).
// Energies, edge gradients, forces, the virial and their reductions stay float64.
template <typename T, typename S>
struct Pipe {
  using NodeT = typename std::conditional<std::is_same<S, bf16_t>::value, float, double>::type;
  // node gradients of the adjoint (dE/dh, dE/dy, the per-sender sums): type T.  They reach
  // only forces, the virial and weight gradients, whose float32 bounds they meet; the
  // energies come from the forward chain alone.
  using GradT = T;
  sn_ctx* c;
  const sn_model* m;
  hipStream_t s;
  bool bf16;
  explicit Pipe(sn_ctx* ctx)
      : c(ctx), m(ctx->m), s(ctx->stream), bf16(ctx->precision == SN_BF16) {}
  // launches inside the scope go to another stream
  struct OnStream {
    Pipe* p;
    hipStream_t old;
    OnStream(Pipe* pp, hipStream_t ns) : p(pp), old(pp->s) { p->s = ns; }
    ~OnStream() { p->s = old; }
  };

  // float32-accumulated contractions (and every contraction of the BF16 form) run on the
  // matrix cores; float64-accumulated ones on the vector units.
  template <typename TA, typename TB, typename TC, typename TACC>
  void gemm(int64_t rows, int N, int K, const TA* A, RowMap am, int64_t woff, int ldb, bool bt,
            TC* C, RowMap cm, TACC alpha, bool acc) {
    if constexpr (std::is_same<TC, bf16_t>::value) {
      launch_gemm_mfma<TA, TB, TC>(rows, N, K, A, am, W<TB>(c, woff), ldb, bt, C, cm, (float)alpha,
                                   acc, bf16, s);
    } else {
      if (bf16 || std::is_same<TACC, float>::value)
        launch_gemm_mfma<TA, TB, TC>(rows, N, K, A, am, W<TB>(c, woff), ldb, bt, C, cm,
                                     (float)alpha, acc, bf16, s);
      else
        launch_gemm<TA, TB, TC, TACC>(rows, N, K, A, am, W<TB>(c, woff), ldb, bt, C, cm, alpha, acc,
                                      false, s);
    }
  }

  // the per-degree contractions of one channel-mixing layer as one grouped launch (same
  // dispatch rule as gemm())
  template <typename TA, typename TB, typename TC>
  GemmDesc<TA, TB, TC> gd(int64_t rows, int N, int K, const TA* A, RowMap am, int64_t woff, int ldb,
                          TC* C, RowMap cm, double alpha, bool acc) {
    return GemmDesc<TA, TB, TC>{rows, N, K, A, am, W<TB>(c, woff), ldb, C, cm, alpha, acc ? 1 : 0};
  }
  template <typename TA, typename TB, typename TC, typename TACC>
  void gemm_group(const std::vector<GemmDesc<TA, TB, TC>>& d, bool bt) {
    if (d.empty()) return;
    const int n = (int)d.size();
    if (std::is_same<TC, bf16_t>::value || bf16 || std::is_same<TACC, float>::value)
      launch_gemm_mfma_group<TA, TB, TC>(n, d.data(), bt, bf16, s);
    else
      launch_gemm_group<TA, TB, TC, TACC>(n, d.data(), bt, false, s);
  }

  // bfloat16 panels of block L's output weights for the fused kernels: [c][j] for the
  // forward, [j][c] for the adjoint
  const bf16_t* wc_panel(const LayerDesc& L, bool fwd) const {
    const size_t t = (size_t)(&L - m->layers.data());
    return fwd ? c->wc_panT16[t] : c->wc_pan16[t];
  }

  // radial MLP over undirected pairs: fused matrix-core kernels for float32 storage,
  // vector-unit path for float64
  void mlp_forward(const LayerDesc& L, const T* rho, S* w) {
    const int64_t NPr = c->NP;
    const int* pe1 = c->get<int>("pair_e1", c->E);
    if constexpr (std::is_same<T, float>::value) {
      if (L.P % 8) throw UnsupportedError("radial weight count not a multiple of 8");
      if constexpr (std::is_same<S, float>::value)  // FP32 form: split-bfloat16 output layer
        launch_mlp_fused_fwd_split(NPr, pe1, rho, W<float>(c, L.w_mlp[0]), W<float>(c, L.w_mlp[1]),
                                   c->wc_panT3[(size_t)(&L - m->layers.data())], L.P,
                                   (float)m->act, w, s);
      else
        launch_mlp_fused_fwd(NPr, pe1, rho, W<float>(c, L.w_mlp[0]), W<float>(c, L.w_mlp[1]),
                             wc_panel(L, true), L.P, (float)m->act, w, s);
    } else {
      T* z2 = c->get<T>("z2", NPr * m->hidden);
      launch_mlp_hidden_fwd<T>(NPr, pe1, rho, m->nb, m->hidden, W<T>(c, L.w_mlp[0]),
                               W<T>(c, L.w_mlp[1]), (T)m->act, z2, s);
      gemm<T, T, T, T>(NPr, L.P, m->hidden, z2, plain_rows(m->hidden), L.w_mlp[2], L.P, false, w,
                       plain_rows(L.P), T(1), false);
    }
  }
  void mlp_backward(const LayerDesc& L, const T* rho, const S* dw, T* dz2, T* drho) {
    const int64_t NPr = c->NP;
    const int* pe1 = c->get<int>("pair_e1", c->E);
    const int* pe2 = c->get<int>("pair_e2", c->E);
    if constexpr (std::is_same<T, float>::value) {
      (void)dz2;
      if constexpr (std::is_same<S, float>::value)  // FP32 form: split-bfloat16 dw Wc^T
        launch_mlp_fused_bwd_split(NPr, pe1, pe2, rho, W<float>(c, L.w_mlp[0]),
                                   W<float>(c, L.w_mlp[1]),
                                   c->wc_pan3[(size_t)(&L - m->layers.data())], L.P,
                                   (float)m->act, dw, drho, true, s);
      else
        launch_mlp_fused_bwd(NPr, pe1, pe2, rho, W<float>(c, L.w_mlp[0]), W<float>(c, L.w_mlp[1]),
                             wc_panel(L, false), L.P, (float)m->act, dw, drho, true, s);
    } else {
      T* dws = c->get<T>("dw_pair", NPr * L.P);
      launch_pair_sum<T>(NPr, pe1, pe2, dw, L.P, dws, s);
      gemm<T, T, T, T>(NPr, m->hidden, L.P, dws, plain_rows(L.P), L.w_mlp[2], L.P, true, dz2,
                       plain_rows(m->hidden), T(1), false);
      launch_mlp_hidden_bwd<T>(NPr, pe1, rho, m->nb, m->hidden, W<T>(c, L.w_mlp[0]),
                               W<T>(c, L.w_mlp[1]), (T)m->act, dz2, drho, true, s);
    }
  }

  // Training: the radial-MLP adjoint unfused (pair sums of dE/dw, dz2 = dE/dw Wc^T, the
  // hidden layers' adjoint) with the MLP's weight gradients, pairs as rows:
  //   dWc = z2^T dE/dw,  dWb = z1^T da2,  dWa = rho^T da1
  void mlp_backward_train(const LayerDesc& L, const T* rho, const S* dw, T* drho, double* gw) {
    const int64_t NPr = c->NP;
    const int* pe1 = c->get<int>("pair_e1", c->E);
    const int* pe2 = c->get<int>("pair_e2", c->E);
    const int H = m->hidden, NB = m->nb;
    T* dws = c->get<T>("dw_pair", NPr * L.P);
    launch_pair_sum<S, T>(NPr, pe1, pe2, dw, L.P, dws, s);
    T* dz2 = c->get<T>("dz2", NPr * H);
    gemm<T, T, T, T>(NPr, H, L.P, dws, plain_rows(L.P), L.w_mlp[2], L.P, true, dz2, plain_rows(H),
                     T(1), false);
    T* z1 = c->get<T>("tr_z1", NPr * H);
    T* z2 = c->get<T>("tr_z2", NPr * H);
    T* da1 = c->get<T>("tr_da1", NPr * H);
    T* da2 = c->get<T>("tr_da2", NPr * H);
    launch_mlp_hidden_bwd<T>(NPr, pe1, rho, NB, H, W<T>(c, L.w_mlp[0]), W<T>(c, L.w_mlp[1]),
                             (T)m->act, dz2, drho, true, s, z1, da1, da2);
    launch_mlp_hidden_fwd<T>(NPr, pe1, rho, NB, H, W<T>(c, L.w_mlp[0]), W<T>(c, L.w_mlp[1]),
                             (T)m->act, z2, s);
    double* part = c->get<double>("wg_part_aux", wgrad_chunks(NPr) * (int64_t)H * std::max(L.P, H));
    launch_wgrad<T, T>(NPr, H, L.P, z2, plain_rows(H), nullptr, nullptr, dws, plain_rows(L.P), 1.0,
                       part, gw + L.w_mlp[2], s);
    launch_wgrad<T, T>(NPr, H, H, z1, plain_rows(H), nullptr, nullptr, da2, plain_rows(H), 1.0, part,
                       gw + L.w_mlp[1], s);
    launch_wgrad<T, T>(NPr, NB, H, rho, plain_rows(NB), pe1, nullptr, da1, plain_rows(H), 1.0, part,
                       gw + L.w_mlp[0], s);
  }

  // weight gradient of a channel mixing over `rows` rows into the tensor at offset woff
  template <typename TA, typename TB>
  void wgrad(int64_t rows, int K, int N, const TA* A, RowMap am, const TB* B, RowMap bm,
             int64_t woff, double* gw) {
    double* part = c->get<double>("wg_part", wgrad_chunks(rows) * (int64_t)K * N);
    launch_wgrad<TA, TB>(rows, K, N, A, am, nullptr, nullptr, B, bm, 1.0, part, gw + woff, s);
  }

  void forward(double* d_energy, double* d_atom_energy_orig) {
    const int N = c->N, G = c->G, NE = N + G;
    const int64_t E = c->E;
    const int* row_ptr = c->get<int>("row_ptr", N + 1);
    const int* src = c->get<int>("src", E);
    const int* recv = c->get<int>("recv", E);
    const double* pos_ext = c->get<double>("pos_ext", 3 * (int64_t)NE);
    const int* spec_ext = c->get<int>("spec_ext", NE);
    const int* owner = c->get<int>("ghost_owner", G);
    const int* pidx = c->get<int>("pidx", E);
    const int NY = (m->lsh + 1) * (m->lsh + 1);
    T* Y = c->get<T>("Y", E * NY);
    T* rho = c->get<T>("rho", E * m->nb);
    c->mark("edge_basis");
    launch_edge_basis<T>(E, recv, src, pos_ext, m->rc, m->nb, m->p, m->lsh, Y, rho, s);
    // radial weights of every block on the aux stream: they need only rho
    std::vector<hipEvent_t> w_ready(m->T);
    c->join(c->aux, s);
    for (int t = 0; t < m->T; ++t) {
      const LayerDesc& L = m->layers[t];
      const std::string ts = std::to_string(t);
      S* w = c->get<S>("w" + ts, c->NP * L.P);
      c->aux_begin("layer" + ts + ".mlp");
      {
        OnStream os(this, c->aux);
        mlp_forward(L, rho, w);
      }
      c->aux_end();
      w_ready[t] = c->sync_event();
      HIPCHK(hipEventRecord(w_ready[t], c->aux));
    }
    const T act = (T)m->act;
    const int C0 = m->muls[0];
    // h^(1): embedding rows for locals and ghosts (a ghost's first features come from its species)
    c->mark("embed");
    NodeT* h = c->get<NodeT>("h_cur", (int64_t)NE * C0);
    launch_embed<NodeT>(NE, spec_ext, W<NodeT>(c, m->off("embed", {(int)m->species.size(), C0})),
                         C0, h, C0, s);
    for (int t = 0; t < m->T; ++t) {
      const LayerDesc& L = m->layers[t];
      const std::string ts = std::to_string(t);
      c->mark("layer" + ts + ".linear_in");
      S* x = c->get<S>("x" + ts, (int64_t)NE * L.hin.width);
      NodeT* y = c->get<NodeT>("y" + ts, (int64_t)N * L.yl.width);
      const int xrows = (t == 0) ? NE : N;  // block 1: ghosts from their own species
      // Lin1 accumulates in the edge type: x only feeds the tensor product, which runs in it
      {
        std::vector<GemmDesc<NodeT, T, S>> g;
        for (int l : L.ins)
          g.push_back(gd<NodeT, T, S>((int64_t)xrows * (2 * l + 1), L.hin.mul[l], L.hin.mul[l], h,
                                       rows_of(L.hin, l), L.w_lin1[l], L.hin.mul[l], x,
                                       rows_of(L.hin, l), 1.0, false));
        gemm_group<NodeT, T, S, T>(g, false);
      }
      if (t > 0) {
        c->mark("layer" + ts + ".ghost_refresh");
        launch_ghost_refresh<S>(N, G, owner, x, L.hin.width, s);
      }
      c->mark("layer" + ts + ".linsc");
      {
        std::vector<GemmDesc<NodeT, NodeT, NodeT>> g;
        for (int l : L.ins)
          if (L.gmul[l] > 0)
            g.push_back(gd<NodeT, NodeT, NodeT>((int64_t)N * (2 * l + 1), L.gmul[l],
                                                   L.hin.mul[l], h, rows_of(L.hin, l),
                                                   L.w_linsc[l], L.gmul[l], y, rows_of(L.yl, l),
                                                   1.0, false));
        gemm_group<NodeT, NodeT, NodeT, NodeT>(g, false);
      }
      S* w = c->get<S>("w" + ts, c->NP * L.P);
      c->mark("layer" + ts + ".tp");
      HIPCHK(hipStreamWaitEvent(s, w_ready[t], 0));
      S* M = c->get<S>(c->fwd_train ? "M" + ts : std::string("M"), (int64_t)N * L.ml.width);
      launch_tp_fwd<T, S>(L.tp, N, row_ptr, src, pidx, Y, x, w, M, (T)(1.0 / m->kavg), s);
      c->mark("layer" + ts + ".linear_out");
      {
        std::vector<GemmDesc<S, T, NodeT>> g;
        for (int l : L.outs) {
          const bool has_sc =
              std::find(L.ins.begin(), L.ins.end(), l) != L.ins.end() && L.gmul[l] > 0;
          g.push_back(gd<S, T, NodeT>((int64_t)N * (2 * l + 1), L.gmul[l], L.mid[l], M,
                                       rows_of(L.ml, l), L.w_lin2[l], L.gmul[l], y,
                                       rows_of(L.yl, l), 1.0, has_sc));
        }
        gemm_group<S, T, NodeT, T>(g, false);
      }
      // block outputs alternate between two buffers, or stay per block for weight gradients
      NodeT* hn = c->get<NodeT>(c->fwd_train ? "h_out" + ts : std::string(t % 2 ? "h_a" : "h_b"),
                                  (int64_t)N * L.hout.width);
      launch_gate_fwd<NodeT>(N, L.last, L.yl, L.hout, y, hn, (NodeT)m->act, s);
      h = hn;
    }
    c->mark("readout");
    double* ae = c->get<double>("atom_e", N);
    const int* spec_loc = c->get<int>("spec_local", N);
    launch_readout<NodeT>(N, h, m->layers.back().hout.width, c->d_v, C0, m->sigma, c->d_shift,
                           spec_loc, ae, s);
    // per-structure energies (eq 1): fixed-order segmented sums
    double* part = c->get<double>("partial_e", c->n_echunk);
    launch_seg_energy(c->n_echunk, c->get<int>("echunks", 3 * c->n_echunk), ae, part, s);
    launch_seg_finalize(c->B, c->get<int>("efirst", c->B + 1), part, 1, d_energy, nullptr, s);
    if (d_atom_energy_orig) {
      const int* order = c->get<int>("order", N);
      launch_unpermute(N, order, ae, 1, d_atom_energy_orig, nullptr, nullptr, 1, s);
    }
    // a launch refused by the runtime (resources, configuration) leaves its outputs unwritten
    HIPCHK(hipGetLastError());
  }

  // d_grad: dL/dE_b per structure in device memory (null: 1), applied to the outputs (the
  // adjoint is linear in the seed and structures share no edges).  With gw (training; the
  // forward kept every block's inputs and messages) the seed itself carries each atom's
  // dL/dE_b and gw receives dL/dW of every weight, laid out as the weights file.
  void backward(const double* d_grad, double* d_forces_orig, double* d_virial,
                double* gw = nullptr) {
    const int N = c->N, G = c->G, NE = N + G;
    const bool train = gw != nullptr;
    (void)G;
    const int64_t E = c->E;
    const int* row_ptr = c->get<int>("row_ptr", N + 1);
    const int* src = c->get<int>("src", E);
    const int* recv = c->get<int>("recv", E);
    const int* sptr = c->get<int>("send_ptr", NE + 1);
    const int* sidx = c->get<int>("send_idx", E);
    const int* gptr = c->get<int>("ghost_ptr", N + 1);
    const int* pidx = c->get<int>("pidx", E);
    const double* pos_ext = c->get<double>("pos_ext", 3 * (int64_t)NE);
    const int NY = (m->lsh + 1) * (m->lsh + 1);
    const T* Y = c->get<T>("Y", E * NY);
    const T* rho = c->get<T>("rho", E * m->nb);
    const T act = (T)m->act;
    const int C0 = m->muls[0];
    int max_w = 0, max_P = 0, max_tasks = 0, max_m = 0, max_y = 0;
    for (auto& L : m->layers) {
      max_w = std::max(max_w, L.hin.width);
      max_P = std::max(max_P, L.P);
      max_tasks = std::max(max_tasks, L.tp.n_tasks);
      max_m = std::max(max_m, L.ml.width);
      max_y = std::max(max_y, L.yl.width);
    }
    GradT* dh = c->get<GradT>("dh_a", (int64_t)N * max_w);
    GradT* dh_other = c->get<GradT>("dh_b", (int64_t)N * max_w);
    GradT* dy = c->get<GradT>("dy", (int64_t)N * max_y);
    S* Gm = c->get<S>("G", (int64_t)N * max_m);
    // dE/dw alternates between two buffers: the MLP adjoint of block t (aux stream) reads
    // one while the tensor-product adjoint of block t-1 writes the other
    S* dw_buf[2] = {c->get<S>("dw_a", 2 * c->NP * max_P), c->get<S>("dw_b", 2 * c->NP * max_P)};
    std::vector<hipEvent_t> mlp_done(m->T, nullptr);
    S* dxe = c->get<S>("dxe", E * max_w);
    GradT* dx_ext = c->get<GradT>("dx_ext", (int64_t)NE * max_w);
    GradT* dx = c->get<GradT>("dx", (int64_t)N * max_w);
    T* dz2 = c->get<T>("dz2", c->NP * m->hidden);
    T* dY = c->get<T>("dY", E * NY);
    T* drho = c->get<T>("drho", E * m->nb);
    zero(drho, sizeof(T) * E * m->nb, s);  // only the first edge of each pair receives drho
    c->mark("bwd.readout");
    const double* g_atom = nullptr;
    if (train) {
      zero(gw, sizeof(double) * m->flat.size(), s);
      double* ga = c->get<double>("g_atom", N);
      launch_atom_grad(N, c->get<int>("sid_local", N), c->R / c->B, d_grad, ga, s);
      g_atom = ga;
      // dE/dh^(T+1)_i = sigma g_i (Wr1 Wr2); readout weights from u = sum_i g_i h_i
      const int wlast = m->layers.back().hout.width;
      launch_seed_rows(N, c->d_v, C0, m->sigma, g_atom, dh, wlast, s);
      const NodeT* hT = c->get<NodeT>("h_out" + std::to_string(m->T - 1), (int64_t)N * wlast);
      double* u = c->get<double>("tr_u", C0);
      wgrad<NodeT, double>(N, C0, 1, hT, plain_rows(wlast), g_atom, plain_rows(1), 0, u);
      const int64_t r0 = m->tensors.at("readout.0").first, r1 = m->tensors.at("readout.1").first;
      launch_readout_wgrad(C0, u, W<double>(c, r0), W<double>(c, r1), m->sigma, gw + r0, gw + r1, s);
    } else {
      // dE/dh^(T+1) = sigma (Wr1 Wr2): the same vector for every atom
      launch_fill_rows<GradT>(N, c->d_v, C0, m->sigma, dh, m->layers.back().hout.width, s);
    }
    for (int t = m->T - 1; t >= 0; --t) {
      const LayerDesc& L = m->layers[t];
      const std::string ts = std::to_string(t);
      const S* x = c->get<S>("x" + ts, (int64_t)NE * L.hin.width);
      const NodeT* y = c->get<NodeT>("y" + ts, (int64_t)N * L.yl.width);
      const S* w = c->get<S>("w" + ts, c->NP * L.P);
      c->mark("bwd.layer" + ts + ".linear_out");
      launch_gate_bwd<NodeT, GradT>(N, L.last, L.yl, L.hout, y, dh, dy, (NodeT)m->act, s);
      // the block's input features (NE rows in block 1, whose ghosts carry their own species)
      const NodeT* h_in =
          train ? c->get<NodeT>(t == 0 ? std::string("h_cur") : "h_out" + std::to_string(t - 1),
                                 (int64_t)(t == 0 ? NE : N) * L.hin.width)
                : nullptr;
      if (train) {
        // Lin2: dW = M^T dy;  Linsc: dW = h^T dy
        const S* Mt = c->get<S>("M" + ts, (int64_t)N * L.ml.width);
        for (int l : L.outs)
          wgrad<S, GradT>((int64_t)N * (2 * l + 1), L.mid[l], L.gmul[l], Mt, rows_of(L.ml, l), dy,
                           rows_of(L.yl, l), L.w_lin2[l], gw);
        for (int l : L.ins)
          if (L.gmul[l] > 0)
            wgrad<NodeT, GradT>((int64_t)N * (2 * l + 1), L.hin.mul[l], L.gmul[l], h_in,
                                  rows_of(L.hin, l), dy, rows_of(L.yl, l), L.w_linsc[l], gw);
      }
      {
        std::vector<GemmDesc<GradT, T, S>> g;
        for (int l : L.outs)
          g.push_back(gd<GradT, T, S>((int64_t)N * (2 * l + 1), L.mid[l], L.gmul[l], dy,
                                       rows_of(L.yl, l), L.w_lin2[l], L.gmul[l], Gm,
                                       rows_of(L.ml, l), 1.0 / m->kavg, false));
        gemm_group<GradT, T, S, T>(g, true);
      }
      S* dw = dw_buf[t % 2];
      if (t + 2 < m->T) {  // dw_buf[t % 2] is free once the MLP adjoint of block t + 2 is done
        c->mark("bwd.layer" + ts + ".mlp_wait");
        HIPCHK(hipStreamWaitEvent(s, mlp_done[t + 2], 0));
      }
      c->mark("bwd.layer" + ts + ".tp");
      launch_tp_bwd<T, S>(L.tp, N, row_ptr, src, pidx, Y, x, w, Gm, dw,
                          (t > 0 || train) ? dxe : nullptr, dY, t != m->T - 1, s);
      c->join(c->aux, s);
      c->aux_begin("bwd.layer" + ts + ".mlp");
      {
        OnStream os(this, c->aux);
        if (train) mlp_backward_train(L, rho, dw, drho, gw);
        else mlp_backward(L, rho, dw, dz2, drho);
      }
      c->aux_end();
      mlp_done[t] = c->sync_event();
      HIPCHK(hipEventRecord(mlp_done[t], c->aux));
      if (t == 0 && !train) break;
      c->mark("bwd.layer" + ts + ".sender_fold");
      // sender-side sums over every extended row
      launch_sender_reduce<S, GradT>(NE, sptr, sidx, dxe, L.hin.width, dx_ext, s);
      if (t == 0) {
        // block 1 (training): x = Lin1(h^(1)) on every extended row, each ghost from its own
        // species, so nothing folds: dW = h^T dx over all rows, then dE/dh^(1) on all rows
        // (plus the self-connection's share on local rows) feeds the embedding gradient
        wgrad<NodeT, GradT>(NE, C0, C0, h_in, rows_of(L.hin, 0), dx_ext, rows_of(L.hin, 0),
                              L.w_lin1[0], gw);
        GradT* dh1 = c->get<GradT>("tr_dh1", (int64_t)NE * C0);
        gemm<GradT, T, GradT, T>(NE, C0, C0, dx_ext, rows_of(L.hin, 0), L.w_lin1[0], C0, true, dh1,
                                   rows_of(L.hin, 0), T(1), false);
        if (L.gmul[0] > 0)
          gemm<GradT, T, GradT, T>(N, C0, L.gmul[0], dy, rows_of(L.yl, 0), L.w_linsc[0],
                                     L.gmul[0], true, dh1, rows_of(L.hin, 0), T(1), true);
        const int S_ = (int)m->species.size();
        double* part = c->get<double>("wg_part", wgrad_chunks(NE) * (int64_t)S_ * C0);
        launch_wgrad<NodeT, GradT>(NE, S_, C0, nullptr, plain_rows(0), nullptr,
                                     c->get<int>("spec_ext", NE), dh1, plain_rows(C0), 1.0, part,
                                     gw + m->tensors.at("embed").first, s);
        break;
      }
      // fold ghost rows onto owners
      launch_ghost_fold<GradT>(N, gptr, dx_ext, dx, L.hin.width, s);
      if (train)  // Lin1: dW = h^T dx
        for (int l : L.ins)
          wgrad<NodeT, GradT>((int64_t)N * (2 * l + 1), L.hin.mul[l], L.hin.mul[l], h_in,
                                rows_of(L.hin, l), dx, rows_of(L.hin, l), L.w_lin1[l], gw);
      c->mark("bwd.layer" + ts + ".linear_in");
      {
        // dh = dx Lin1^T (all degrees), then += dy Linsc^T (all degrees)
        std::vector<GemmDesc<GradT, T, GradT>> g1, g2;
        for (int l : L.ins) {
          g1.push_back(gd<GradT, T, GradT>((int64_t)N * (2 * l + 1), L.hin.mul[l], L.hin.mul[l],
                                             dx, rows_of(L.hin, l), L.w_lin1[l], L.hin.mul[l],
                                             dh_other, rows_of(L.hin, l), 1.0, false));
          if (L.gmul[l] > 0)
            g2.push_back(gd<GradT, T, GradT>((int64_t)N * (2 * l + 1), L.hin.mul[l], L.gmul[l],
                                               dy, rows_of(L.yl, l), L.w_linsc[l], L.gmul[l],
                                               dh_other, rows_of(L.hin, l), 1.0, true));
        }
        gemm_group<GradT, T, GradT, T>(g1, true);
        gemm_group<GradT, T, GradT, T>(g2, true);
      }
      std::swap(dh, dh_other);
    }
    c->mark("bwd.forces");
    double* gE = c->get<double>("g_edge", 3 * E);
    HIPCHK(hipStreamWaitEvent(s, mlp_done[0], 0));  // every block's dE/drho is in
    launch_edge_grad<T>(E, recv, src, pos_ext, m->rc, m->nb, m->p, m->lsh, dY, drho, gE, s);
    double* F = c->get<double>("F_local", 3 * (int64_t)N);
    launch_forces(N, row_ptr, sptr, sidx, gptr, gE, F, s);
    // (with training seeds the edge gradients already carry each structure's dL/dE_b)
    const double* out_scale = train ? nullptr : d_grad;
    if (d_forces_orig) {
      const int* order = c->get<int>("order", N);
      launch_unpermute(N, order, F, 3, d_forces_orig, out_scale, c->get<int>("sid_orig", N),
                       c->R / c->B, s);
    }
    if (d_virial) {
      double* part = c->get<double>("partial_w", 9 * (int64_t)c->n_vchunk);
      launch_seg_virial(c->n_vchunk, c->get<int>("vchunks", 3 * c->n_vchunk), recv, src, pos_ext,
                        gE, part, s);
      launch_seg_finalize(c->B, c->get<int>("vfirst", c->B + 1), part, 9, d_virial, out_scale, s);
    }
    HIPCHK(hipGetLastError());
    c->mark("end");
  }
};

void destroy_replays(sn_ctx* c);

// Free every workspace buffer (not the weights); the graph and any pending forward are
// dropped.  False when the device reported an error meanwhile (the context is then dead).
bool release_workspace(sn_ctx* c) {
  bool ok = hipStreamSynchronize(c->stream) == hipSuccess;
  destroy_replays(c);
  if (c->aux && hipStreamSynchronize(c->aux) != hipSuccess) ok = false;
  for (auto& kv : c->bufs)
    if (kv.second.p && !c->dev_free(kv.second.p, kv.second.cap)) ok = false;
  c->bufs.clear();
  c->used = 0;
  c->have_graph = false;
  c->pending = false;
  c->marks.clear();
  c->aux_marks.clear();
  if (!ok) c->dead = true;
  return ok;
}

void collect_timings(sn_ctx* c) {
  c->timings.clear();
  if (c->marks.size() < 2) return;
  HIPCHK(hipEventSynchronize(c->marks.back().second));
  std::map<std::string, double> acc;
  std::vector<std::string> orderv;
  for (size_t i = 0; i + 1 < c->marks.size(); ++i) {
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, c->marks[i].second, c->marks[i + 1].second));
    if (!acc.count(c->marks[i].first)) orderv.push_back(c->marks[i].first);
    acc[c->marks[i].first] += ms;
  }
  for (auto& am : c->aux_marks) {
    if (!am.second.second) continue;
    HIPCHK(hipEventSynchronize(am.second.second));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, am.second.first, am.second.second));
    if (!acc.count(am.first)) orderv.push_back(am.first);
    acc[am.first] += ms;
  }
  for (auto& k : orderv) c->timings.push_back({k, acc[k]});
}

template <typename F>
int guarded(sn_ctx* c, F&& f) {
  if (c && c->dead) {
    return SN_EHIP;
  }
  try {
    if (c) HIPCHK(hipSetDevice(c->device));
    f();
    return SN_OK;
  } catch (const ArgError& e) {
    if (c) c->err = e.what();
    return SN_EINVAL;
  } catch (const ScratchError& e) {
    if (c) {
      c->err = e.what();
      // kernels of the refused call may still run on either stream over the shared scratch:
      // let them finish before another call reuses it
      bool ok = hipStreamSynchronize(c->stream) == hipSuccess;
      if (c->aux && hipStreamSynchronize(c->aux) != hipSuccess) ok = false;
      if (!ok) {
        c->dead = true;
        return SN_EHIP;
      }
    }
    return SN_ENOMEM;
  } catch (const MemError& e) {
    if (c) {
      c->err = e.what();
      // a partly grown workspace would make every later, smaller request fail as well
      if (!release_workspace(c)) return SN_EHIP;
    }
    return SN_ENOMEM;
  } catch (const UnsupportedError& e) {
    if (c) c->err = e.what();
    return SN_EUNSUPPORTED;
  } catch (const HipError& e) {
    if (c) {
      c->err = e.what();
      c->dead = true;
    }
    return SN_EHIP;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return SN_EINVAL;
  }
}

// ------------------------------------------------------------------ hipGraph replay
// Records the launches of f() into a graph and instantiates it.  Everything is recorded on
// one stream (the aux stream is folded into it while recording) and without timing events;
// when the context's stream is the null stream, a private stream records and replays,
// ordered against the null stream by events.
hipStream_t replay_stream(sn_ctx* c) {
  if (c->stream) return c->stream;
  if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  return c->cap_stream;
}
void destroy_replays(sn_ctx* c) {
  for (sn_ctx::Replay* r : {&c->rp_fwd, &c->rp_bwd}) {
    if (r->exec) (void)hipGraphExecDestroy(r->exec);
    r->exec = nullptr;
    r->version = ~0ull;
  }
}
template <class F>
hipGraphExec_t record_graph(sn_ctx* c, F&& f) {
  hipStream_t cs = replay_stream(c);
  hipStream_t user = c->stream, aux = c->aux;
  c->stream = cs;
  c->aux = cs;
  c->capturing = true;
  auto restore = [&] {
    c->stream = user;
    c->aux = aux;
    c->capturing = false;
  };
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    f();
  } catch (...) {
    (void)hipStreamEndCapture(cs, &g);
    if (g) (void)hipGraphDestroy(g);
    restore();
    throw;
  }
  const hipError_t e = hipStreamEndCapture(cs, &g);
  restore();
  HIPCHK(e);
  hipGraphExec_t exec = nullptr;
  const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HIPCHK(ei);
  return exec;
}
void launch_replay(sn_ctx* c, hipGraphExec_t exec) {
  hipStream_t cs = replay_stream(c);
  if (cs != c->stream) c->join(cs, c->stream);
  HIPCHK(hipGraphLaunch(exec, cs));
  if (cs != c->stream) c->join(c->stream, cs);
}
bool replay_hit(const sn_ctx::Replay& r, uint64_t version, const void* k0, const void* k1,
                const void* k2) {
  return r.exec && r.version == version && r.key[0] == k0 && r.key[1] == k1 && r.key[2] == k2;
}

template <typename T, typename S>
void forward_impl(sn_ctx* c, int B, const int64_t* offsets, const double* d_pos, const int* d_spec,
                  const double* cells, double* d_energy, double* d_atom_energy) {
  const int64_t n = offsets[B];
  if (n <= 0 || n > (1 << 28)) throw ArgError("atom count out of range");
  c->fwd_train = c->train;
  c->marks.clear();
  c->aux_marks.clear();
  c->event_next = 0;
  c->sync_next = 0;
  c->mark("graph");
  const bool same = c->have_graph && c->B == B && c->N == n &&
                    std::equal(offsets, offsets + B + 1, c->atom_off.begin()) &&
                    std::memcmp(c->graph_cells.data(), cells, sizeof(double) * 9 * B) == 0;
  if (c->reuse && same) {
    // atoms moved less than skin/2 since the last build: refresh positions only
    auto body = [&] {
      launch_refresh_positions(c->N, c->G, c->get<int>("order", c->N), d_pos,
                               c->get<double>("wrap_off", 3 * (int64_t)c->N),
                               c->get<int>("ghost_owner", c->G),
                               c->get<int>("ghost_shift", 3 * (int64_t)c->G),
                               c->get<int>("sid_ext", c->N + c->G),
                               c->get<StructParams>("struct_params", c->R),
                               c->get<double>("pos_ext", 3 * (int64_t)(c->N + c->G)), c->stream);
      if (c->compacted) compact_list(c);
      Pipe<T, S> p(c);
      p.forward(d_energy, d_atom_energy);
    };
    c->last_fwd_reused = true;
    c->pending = true;
    sn_ctx::Replay& r = c->rp_fwd;
    // replay once an eager run on this graph has sized every buffer (not in training mode,
    // whose forwards keep other buffers)
    if (c->capture && !c->train && !c->compacted && c->reuse_runs >= 1) {
      if (!replay_hit(r, c->graph_version, d_pos, d_energy, d_atom_energy)) {
        if (r.exec) (void)hipGraphExecDestroy(r.exec);
        r.exec = nullptr;
        r.exec = record_graph(c, body);
        r.version = c->graph_version;
        r.key[0] = d_pos;
        r.key[1] = d_energy;
        r.key[2] = d_atom_energy;
      }
      launch_replay(c, r.exec);
      return;
    }
    body();
    ++c->reuse_runs;
    return;
  }
  c->have_graph = false;
  c->last_fwd_reused = false;
  c->reuse_runs = 0;
  ++c->graph_version;
  setup_cells(c, B, offsets, cells);
  build_graph<T>(c, (int)n, d_pos, d_spec);
  launch_wrap_offsets((int)n, c->get<int>("order", n), d_pos, c->get<double>("pos_ext", 3 * n),
                      c->get<double>("wrap_off", 3 * n), c->stream);
  // a list with a skin is evaluated over its pairs inside r_c (not with graph replay, whose
  // recorded launches need fixed sizes)
  c->compacted = false;
  if (c->compact && c->skin > 0 && !c->capture) {
    keep_built_list(c);
    compact_list(c);
  }
  c->graph_cells.assign(cells, cells + 9 * B);
  c->have_graph = true;
  Pipe<T, S> p(c);
  p.forward(d_energy, d_atom_energy);
  c->pending = true;
}

template <typename T, typename S>
void backward_impl(sn_ctx* c, const double* d_grad, double* d_forces, double* d_virial,
                   double* d_wgrad = nullptr) {
  if (!c->pending) throw std::logic_error("busy");
  auto body = [&] {
    Pipe<T, S> p(c);
    p.backward(d_grad, d_forces, d_virial, d_wgrad);
  };
  c->pending = false;
  sn_ctx::Replay& r = c->rp_bwd;
  if (!d_wgrad && c->capture && !c->compacted && c->last_fwd_reused && c->reuse_runs >= 1) {
    if (!replay_hit(r, c->graph_version, d_forces, d_virial, d_grad)) {
      if (r.exec) (void)hipGraphExecDestroy(r.exec);
      r.exec = nullptr;
      r.exec = record_graph(c, body);
      r.version = c->graph_version;
      r.key[0] = d_forces;
      r.key[1] = d_virial;
      r.key[2] = d_grad;
    }
    launch_replay(c, r.exec);
    return;
  }
  body();
}

void map_species(const sn_model* m, int64_t n, const int32_t* Z, std::vector<int>& out) {
  out.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) {
    int z = Z[i];
    if (z < 0 || z >= 128 || m->lut[z] < 0) throw ArgError("atomic number not in the model");
    out[i] = m->lut[z];
  }
}

// The host-buffer evaluation of B packed structures (sn_compute_batch, sn_compute and
// sn_compute_noalloc): inputs copied in, forward and adjoint, results copied out.
void compute_batch_host(sn_ctx_t* ctx, int B, const int64_t* offsets, const double* pos,
                     const int32_t* Z, const double* cells, double* energies,
                     double* atom_energies, double* forces, double* virials) {
  const int64_t n = offsets[B];
  {
    std::vector<int> spec;
    map_species(ctx->m, n, Z, spec);
    for (int64_t i = 0; i < 3 * n; ++i)
      if (!std::isfinite(pos[i])) throw ArgError("non-finite positions");
    hipStream_t s = ctx->stream;
    double* d_pos = ctx->get<double>("in_pos", 3 * n);
    int* d_spec = ctx->get<int>("spec_orig", n);
    // staging for the results: B energies, B virials, n atom energies, n x 3 forces
    double* d_out = ctx->get<double>("out_host_stage", 10 * (int64_t)B + 4 * n);
    HIPCHK(hipMemcpyAsync(d_pos, pos, sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_spec, spec.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    double* d_e = d_out;
    double* d_w = d_out + B;
    double* d_ae = d_out + 10 * (int64_t)B;
    double* d_f = d_ae + n;
    const bool need_bwd = forces || virials;
    if (ctx->precision == SN_FP64) {
      forward_impl<double, double>(ctx, B, offsets, d_pos, d_spec, cells, d_e, d_ae);
      if (need_bwd) backward_impl<double, double>(ctx, nullptr, d_f, d_w);
    } else if (ctx->precision == SN_BF16) {
      forward_impl<float, bf16_t>(ctx, B, offsets, d_pos, d_spec, cells, d_e, d_ae);
      if (need_bwd) backward_impl<float, bf16_t>(ctx, nullptr, d_f, d_w);
    } else {
      forward_impl<float, float>(ctx, B, offsets, d_pos, d_spec, cells, d_e, d_ae);
      if (need_bwd) backward_impl<float, float>(ctx, nullptr, d_f, d_w);
    }
    ctx->pending = false;
    std::vector<double> h((size_t)(10 * (int64_t)B + 4 * n));
    HIPCHK(hipMemcpyAsync(h.data(), d_out, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    collect_timings(ctx);
    std::memcpy(energies, &h[0], B * sizeof(double));
    if (virials) std::memcpy(virials, &h[B], 9 * (size_t)B * sizeof(double));
    if (atom_energies) std::memcpy(atom_energies, &h[10 * (size_t)B], n * sizeof(double));
    if (forces) std::memcpy(forces, &h[10 * (size_t)B + n], 3 * n * sizeof(double));
  }
}


// ------------------------------------------------------------------ static scratch
// Device memory of sn_compute_noalloc: one array per device, allocated with the code object
// and held until the process ends.  Host code never passes the symbol itself to a kernel:
// it uses the device address that hipGetSymbolAddress returns, looked up once per device
// with that device current.
}  // namespace

constexpr size_t kScratchBytes = (size_t)512 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, char*> g_scratch_ptr;  // device -> address of its scratch

char* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));  // the caller made device current
  if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) throw HipError("static scratch not aligned");
  g_scratch_ptr[device] = static_cast<char*>(p);
  return static_cast<char*>(p);
}

}  // namespace

namespace {

// The gradient of the whole training loss (sn_train_loss_grad).
template <typename T, typename S>
void train_loss_grad(sn_ctx* c, const sn_batch_t* bt, const double* refE, const double* refF,
                     const double* refS, double delta, double mu_f, double mu_s, double fd_step,
                     double* loss, double* gw) {
  const int B = bt->n_structures;
  const int64_t* off = bt->offsets;
  const int64_t n = off[B];
  hipStream_t s = c->stream;
  const int64_t np = c->m->n_params;
  std::vector<int> spec;
  {
    std::vector<int32_t> hz((size_t)n);
    HIPCHK(hipMemcpyAsync(hz.data(), bt->d_Z, sizeof(int32_t) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    map_species(c->m, n, hz.data(), spec);
  }
  int* d_spec = c->get<int>("spec_orig", n);
  HIPCHK(hipMemcpyAsync(d_spec, spec.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
  // (1) energies, forces and virials of the batch
  double* d_E = c->get<double>("tr_E", B);
  double* d_F = c->get<double>("tr_F", 3 * n);
  double* d_W = c->get<double>("tr_W", 9 * (int64_t)B);
  double* d_one = c->get<double>("tr_one", B);
  launch_fill_f64(B, 1.0, d_one, s);
  const bool was_train = c->train, was_reuse = c->reuse;
  c->train = false;
  c->reuse = false;  // every evaluation below builds its own graph
  forward_impl<T, S>(c, B, off, bt->d_pos, d_spec, bt->cells, d_E, nullptr);
  backward_impl<T, S>(c, d_one, d_F, d_W);
  std::vector<double> E(B), F(3 * n), Wv(9 * (size_t)B);
  HIPCHK(hipMemcpyAsync(E.data(), d_E, sizeof(double) * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(F.data(), d_F, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(Wv.data(), d_W, sizeof(double) * 9 * B, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  // (2) the loss and its derivatives with respect to E_b, F_i and the virials W_b
  auto hub = [&](double r) { const double a = std::fabs(r); return a < delta ? 0.5 * r * r : delta * (a - 0.5 * delta); };
  auto dhub = [&](double r) { return std::fabs(r) < delta ? r : (r > 0 ? delta : -delta); };
  constexpr double kGPa = 160.21766208;  // GPa per eV / A^3
  const double cf = mu_f / (3.0 * B * (double)n), cs = mu_s / (6.0 * B);
  double le = 0, lf = 0, ls = 0;
  std::vector<double> gE(B), v(3 * n, 0.0), U(9 * (size_t)B, 0.0);
  std::vector<int> atom_struct((size_t)n);
  for (int b = 0; b < B; ++b) {
    const double nb = (double)(off[b + 1] - off[b]);
    const double r = E[b] / nb - refE[b] / nb;
    le += hub(r);
    gE[b] = dhub(r) / (B * nb);
    for (int64_t i = off[b]; i < off[b + 1]; ++i) {
      atom_struct[i] = b;
      for (int k = 0; k < 3; ++k) {
        const double rf = F[3 * i + k] - refF[3 * i + k];
        lf += hub(rf);
        v[3 * i + k] = cf * dhub(rf);
      }
    }
    const double* H = bt->cells + 9 * b;
    const double V = std::fabs(H[0] * (H[4] * H[8] - H[5] * H[7]) - H[1] * (H[3] * H[8] - H[5] * H[6]) +
                               H[2] * (H[3] * H[7] - H[4] * H[6]));
    const double* w = &Wv[9 * b];
    // S = -sym(W) / V in GPa, components xx yy zz yz xz xy
    const int ia[6] = {0, 1, 2, 1, 0, 0}, ib[6] = {0, 1, 2, 2, 2, 1};
    for (int l = 0; l < 6; ++l) {
      const double Wab = 0.5 * (w[3 * ia[l] + ib[l]] + w[3 * ib[l] + ia[l]]);
      const double Sl = -Wab / V * kGPa;
      const double rs = Sl - refS[6 * b + l];
      ls += hub(rs);
      const double gS = cs * dhub(rs) * (-kGPa / V);  // dL/dW_ab (symmetric part)
      if (ia[l] == ib[l]) U[9 * b + 4 * ia[l]] += gS;
      else {
        U[9 * b + 3 * ia[l] + ib[l]] += 0.5 * gS;
        U[9 * b + 3 * ib[l] + ia[l]] += 0.5 * gS;
      }
    }
  }
  *loss = le / B + cf * lf + cs * ls;
  // (3) the energy term's weight gradient: the adjoint seeded with dL/dE_b
  double* d_gE = c->get<double>("tr_gE", B);
  HIPCHK(hipMemcpyAsync(d_gE, gE.data(), sizeof(double) * B, hipMemcpyHostToDevice, s));
  c->train = true;
  forward_impl<T, S>(c, B, off, bt->d_pos, d_spec, bt->cells, d_E, nullptr);
  backward_impl<T, S>(c, d_gE, nullptr, nullptr, gw);
  // (4) force and stress terms: sum_i v_i . dF_i/dW + sum_b U_b : dW_b/dW = -d/dW of the
  // directional derivative of E along (v, U); four-point central difference of exact weight
  // gradients along r + eps (v + U r), cells H (I + eps U)^T
  double m = 0;
  std::vector<double> pos(3 * n);
  HIPCHK(hipMemcpyAsync(pos.data(), bt->d_pos, sizeof(double) * 3 * n, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t i = 0; i < n; ++i) {
    const double* u = &U[9 * atom_struct[i]];
    for (int a = 0; a < 3; ++a) {
      const double d = v[3 * i + a] + u[3 * a] * pos[3 * i] + u[3 * a + 1] * pos[3 * i + 1] +
                       u[3 * a + 2] * pos[3 * i + 2];
      m = std::max(m, std::fabs(d));
    }
  }
  if (m > 0) {
    const double step = fd_step > 0 ? fd_step : (c->precision == SN_FP64 ? 1e-3 : 2e-2);
    const double h = step / m;
    double* d_v = c->get<double>("tr_v", 3 * n);
    double* d_U = c->get<double>("tr_U", 9 * (int64_t)B);
    int* d_as = c->get<int>("tr_as", n);
    double* d_pp = c->get<double>("tr_pos", 3 * n);
    double* d_G = c->get<double>("tr_G", np);
    HIPCHK(hipMemcpyAsync(d_v, v.data(), sizeof(double) * 3 * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_U, U.data(), sizeof(double) * 9 * B, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(d_as, atom_struct.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
    std::vector<double> cells(9 * (size_t)B);
    const double steps[4] = {1.0, -1.0, 2.0, -2.0};
    const double wts[4] = {8.0, -8.0, -1.0, 1.0};  // (8 (G+ - G-) - (G++ - G--)) / 12h
    for (int q = 0; q < 4; ++q) {
      const double eps = steps[q] * h;
      launch_perturb(n, bt->d_pos, d_v, d_U, d_as, eps, d_pp, s);
      for (int b = 0; b < B; ++b)
        for (int k = 0; k < 3; ++k)  // cell row k: a_k + eps U a_k
          for (int a = 0; a < 3; ++a) {
            double t = bt->cells[9 * b + 3 * k + a];
            for (int j = 0; j < 3; ++j) t += eps * U[9 * b + 3 * a + j] * bt->cells[9 * b + 3 * k + j];
            cells[9 * b + 3 * k + a] = t;
          }
      forward_impl<T, S>(c, B, off, d_pp, d_spec, cells.data(), d_E, nullptr);
      backward_impl<T, S>(c, d_one, nullptr, nullptr, d_G);
      launch_axpy(np, -wts[q] / (12.0 * h), d_G, gw, s);
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  c->train = was_train;
  c->reuse = was_reuse;
  c->pending = false;
  c->have_graph = false;  // the last graph is the perturbed one
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* sn_strerror(int status) {
  switch (status) {
    case SN_OK: return "ok";
    case SN_EINVAL: return "invalid argument";
    case SN_ENOMEM: return "out of device memory or HBM budget";
    case SN_EHIP: return "HIP runtime error";
    case SN_EUNSUPPORTED: return "unsupported";
    case SN_EBUSY: return "busy";
    default: return "unknown status";
  }
}

const char* sn_last_error(const sn_ctx_t* ctx) {
  if (!ctx) return g_load_error.c_str();
  return ctx->err.c_str();
}

int sn_model_load(const char* path, sn_model_t** out) {
  if (!path || !out) return SN_EINVAL;
  try {
    *out = load_model(path).release();
    return SN_OK;
  } catch (const UnsupportedError& e) {
    g_load_error = e.what();
    return SN_EUNSUPPORTED;
  } catch (const std::exception& e) {
    g_load_error = e.what();
    return SN_EINVAL;
  }
}

void sn_model_free(sn_model_t* model) { delete model; }

int sn_model_info(const sn_model_t* m, sn_model_info_t* info) {
  if (!m || !info) return SN_EINVAL;
  std::memset(info, 0, sizeof(*info));
  info->n_layers = m->T;
  info->l_max = m->lmax;
  info->l_sh = m->lsh;
  for (int l = 0; l < kNumL; ++l) info->muls[l] = m->muls[l];
  info->n_basis = m->nb;
  info->hidden = m->hidden;
  info->n_species = (int)m->species.size();
  for (size_t s = 0; s < m->species.size(); ++s) info->species_z[s] = m->species[s];
  info->r_cut = m->rc;
  info->k_avg = m->kavg;
  info->sigma = m->sigma;
  info->n_params = m->n_params;
  return SN_OK;
}

int sn_cg_table(int l1, int l2, int l3, double* out) {
  constexpr int L = sn::kCGMaxL;
  if (!out || l1 < 0 || l2 < 0 || l3 < 0 || l1 > L || l2 > L || l3 > L) return SN_EINVAL;
  if (l3 < std::abs(l1 - l2) || l3 > l1 + l2) return SN_EINVAL;
  int id = 0;
  for (int a = 0; a <= L; ++a)
    for (int b = 0; b <= L; ++b)
      for (int c = std::abs(a - b); c <= std::min(a + b, L); ++c) {
        if (a == l1 && b == l2 && c == l3) {
          const int n = (2 * l1 + 1) * (2 * l2 + 1) * (2 * l3 + 1);
          for (int i = 0; i < n; ++i) out[i] = sn::kCGDense[id][i];
          return SN_OK;
        }
        ++id;
      }
  return SN_EINVAL;
}

int sn_ctx_create(const sn_model_t* model, int device, void* hip_stream, size_t hbm_budget,
                  int precision, double skin, const sn_allocator_t* alloc, sn_ctx_t** out) {
  if (!model || !out || skin < 0 || !std::isfinite(skin)) return SN_EINVAL;
  if (precision != SN_FP64 && precision != SN_FP32 && precision != SN_BF16) return SN_EINVAL;
  if (alloc && (!alloc->alloc || !alloc->free)) return SN_EINVAL;
  auto c = std::make_unique<sn_ctx>();
  c->m = model;
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (alloc) c->alloc = *alloc;
  c->budget = hbm_budget;
  c->precision = precision;
  c->skin = skin;
  int st = guarded(c.get(), [&] { upload_weights(c.get()); });
  if (st != SN_OK) {
    g_load_error = c->err;
    sn_ctx_free(c.release());  // what upload_weights allocated before failing
    return st;
  }
  *out = c.release();
  return SN_OK;
}

void sn_ctx_free(sn_ctx_t* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->aux) (void)hipStreamSynchronize(ctx->aux);
  for (auto& kv : ctx->bufs)
    if (kv.second.p) (void)ctx->dev_free(kv.second.p, kv.second.cap);
  for (auto& kv : ctx->weight_blocks) (void)ctx->dev_free(kv.first, kv.second);
  ctx->weight_blocks.clear();
  destroy_replays(ctx);
  if (ctx->cap_stream) {
    (void)hipStreamSynchronize(ctx->cap_stream);
    (void)hipStreamDestroy(ctx->cap_stream);
  }
  for (auto ev : ctx->event_pool) (void)hipEventDestroy(ev);
  for (auto ev : ctx->sync_pool) (void)hipEventDestroy(ev);
  if (ctx->aux && ctx->aux != ctx->stream) {
    (void)hipStreamSynchronize(ctx->aux);
    (void)hipStreamDestroy(ctx->aux);
  }
  delete ctx;
}

int sn_forward_device(sn_ctx_t* ctx, const sn_batch_t* batch, double* d_energy,
                      double* d_atom_energy) {
  if (!ctx || !batch || !d_energy) return SN_EINVAL;
  const int B = batch->n_structures;
  const int64_t* off = batch->offsets;
  if (B < 1 || !off || !batch->cells || !batch->d_pos || !batch->d_Z || off[0] != 0) {
    ctx->err = "malformed batch";
    return SN_EINVAL;
  }
  for (int b = 0; b < B; ++b)
    if (off[b + 1] <= off[b]) {
      ctx->err = "empty structure in batch";
      return SN_EINVAL;
    }
  const int64_t n = off[B];
  return guarded(ctx, [&] {
    auto run = [&](const int* d_spec) {
      if (ctx->precision == SN_FP64)
        forward_impl<double, double>(ctx, B, off, batch->d_pos, d_spec, batch->cells, d_energy,
                                     d_atom_energy);
      else if (ctx->precision == SN_BF16)
        forward_impl<float, bf16_t>(ctx, B, off, batch->d_pos, d_spec, batch->cells, d_energy,
                                    d_atom_energy);
      else
        forward_impl<float, float>(ctx, B, off, batch->d_pos, d_spec, batch->cells, d_energy,
                                   d_atom_energy);
    };
    const bool reusable = ctx->reuse && ctx->have_graph && ctx->B == B && ctx->N == n &&
                          std::equal(off, off + B + 1, ctx->atom_off.begin()) &&
                          std::memcmp(ctx->graph_cells.data(), batch->cells,
                                      sizeof(double) * 9 * B) == 0;
    if (reusable) {  // the species of the kept graph stay (reuse contract): no host round trip
      run(ctx->get<int>("spec_orig", n));
      return;
    }
    // map atomic numbers to embedding rows on the host (validation before any launch)
    std::vector<int32_t> hz((size_t)n);
    HIPCHK(hipMemcpyAsync(hz.data(), batch->d_Z, sizeof(int32_t) * n, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    std::vector<int> spec;
    map_species(ctx->m, n, hz.data(), spec);
    int* d_spec = ctx->get<int>("spec_orig", n);
    HIPCHK(hipMemcpyAsync(d_spec, spec.data(), sizeof(int) * n, hipMemcpyHostToDevice, ctx->stream));
    run(d_spec);
  });
}

int sn_backward_device(sn_ctx_t* ctx, const double* d_grad_energy, double* d_forces,
                       double* d_virial) {
  if (!ctx || !d_grad_energy) return SN_EINVAL;
  if (!ctx->pending) {
    ctx->err = "backward without a pending forward";
    return SN_EBUSY;
  }
  return guarded(ctx, [&] {
    if (ctx->precision == SN_FP64)
      backward_impl<double, double>(ctx, d_grad_energy, d_forces, d_virial);
    else if (ctx->precision == SN_BF16)
      backward_impl<float, bf16_t>(ctx, d_grad_energy, d_forces, d_virial);
    else
      backward_impl<float, float>(ctx, d_grad_energy, d_forces, d_virial);
  });
}

int sn_ctx_set_training(sn_ctx_t* ctx, int on) {
  if (!ctx) return SN_EINVAL;
  ctx->train = on != 0;
  return SN_OK;
}

int sn_backward_train_device(sn_ctx_t* ctx, const double* d_grad_energy, double* d_forces,
                             double* d_virial, double* d_weight_grad) {
  if (!ctx || !d_grad_energy || !d_weight_grad) return SN_EINVAL;
  if (!ctx->pending || !ctx->fwd_train) {
    ctx->err = ctx->pending ? "the pending forward did not run in training mode"
                            : "backward without a pending forward";
    return SN_EBUSY;
  }
  if ((int64_t)ctx->m->flat.size() != ctx->m->n_params) {
    ctx->err = "weights file with gaps between tensors";
    return SN_EUNSUPPORTED;
  }
  return guarded(ctx, [&] {
    if (ctx->precision == SN_FP64)
      backward_impl<double, double>(ctx, d_grad_energy, d_forces, d_virial, d_weight_grad);
    else if (ctx->precision == SN_BF16)
      backward_impl<float, bf16_t>(ctx, d_grad_energy, d_forces, d_virial, d_weight_grad);
    else
      backward_impl<float, float>(ctx, d_grad_energy, d_forces, d_virial, d_weight_grad);
  });
}


int sn_train_loss_grad(sn_ctx_t* ctx, const sn_batch_t* batch, const double* ref_energy,
                       const double* ref_forces, const double* ref_stress, double delta,
                       double mu_f, double mu_s, double fd_step, double* loss,
                       double* d_weight_grad) {
  if (!ctx || !batch || !ref_energy || !ref_forces || !ref_stress || !loss || !d_weight_grad ||
      !(delta > 0) || mu_f < 0 || mu_s < 0 || fd_step < 0)
    return SN_EINVAL;
  const int B = batch->n_structures;
  const int64_t* off = batch->offsets;
  if (B < 1 || !off || !batch->cells || !batch->d_pos || !batch->d_Z || off[0] != 0) return SN_EINVAL;
  for (int b = 0; b < B; ++b)
    if (off[b + 1] <= off[b]) return SN_EINVAL;
  if ((int64_t)ctx->m->flat.size() != ctx->m->n_params) {
    ctx->err = "weights file with gaps between tensors";
    return SN_EUNSUPPORTED;
  }
  const bool was_train = ctx->train, was_reuse = ctx->reuse;
  const int st = guarded(ctx, [&] {
    if (ctx->precision == SN_FP64)
      train_loss_grad<double, double>(ctx, batch, ref_energy, ref_forces, ref_stress, delta, mu_f,
                                      mu_s, fd_step, loss, d_weight_grad);
    else if (ctx->precision == SN_BF16)
      train_loss_grad<float, bf16_t>(ctx, batch, ref_energy, ref_forces, ref_stress, delta, mu_f,
                                     mu_s, fd_step, loss, d_weight_grad);
    else
      train_loss_grad<float, float>(ctx, batch, ref_energy, ref_forces, ref_stress, delta, mu_f,
                                    mu_s, fd_step, loss, d_weight_grad);
  });
  ctx->train = was_train;
  ctx->reuse = was_reuse;
  return st;
}

int sn_model_tensor(const sn_model_t* model, int index, const char** name, int64_t* offset,
                    int64_t* count) {
  if (!model || index < 0 || index >= (int)model->tensors.size()) return SN_EINVAL;
  auto it = model->tensors.begin();
  std::advance(it, index);
  int64_t n = 1;
  for (int d : it->second.second) n *= d;
  if (name) *name = it->first.c_str();
  if (offset) *offset = it->second.first;
  if (count) *count = n;
  return SN_OK;
}

int sn_huber_energy_loss(int B, const double* energy, const double* ref, const int64_t* natoms,
                         double delta, double* loss, double* dloss_denergy) {
  if (B < 1 || !energy || !ref || !natoms || !loss || !(delta > 0)) return SN_EINVAL;
  double acc = 0.0;
  for (int b = 0; b < B; ++b) {
    if (natoms[b] < 1) return SN_EINVAL;
    const double nb = (double)natoms[b];
    const double r = energy[b] / nb - ref[b] / nb;
    const double a = std::fabs(r);
    acc += a < delta ? 0.5 * r * r : delta * (a - 0.5 * delta);
    if (dloss_denergy) dloss_denergy[b] = (a < delta ? r : (r > 0 ? delta : -delta)) / (B * nb);
  }
  *loss = acc / B;
  return SN_OK;
}

int sn_ctx_synchronize(sn_ctx_t* ctx) {
  if (!ctx) return SN_EINVAL;
  return guarded(ctx, [&] {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->aux));
    collect_timings(ctx);
  });
}

int sn_compute_batch(sn_ctx_t* ctx, int B, const int64_t* offsets, const double* pos,
                     const int32_t* Z, const double* cells, double* energies,
                     double* atom_energies, double* forces, double* virials) {
  if (!ctx || B < 1 || !offsets || !pos || !Z || !cells || !energies) return SN_EINVAL;
  if (offsets[0] != 0) return SN_EINVAL;
  for (int b = 0; b < B; ++b)
    if (offsets[b + 1] <= offsets[b]) return SN_EINVAL;
  return guarded(ctx, [&] {
    compute_batch_host(ctx, B, offsets, pos, Z, cells, energies, atom_energies, forces, virials);
  });
}

int sn_compute(sn_ctx_t* ctx, int64_t n, const double* pos, const int32_t* Z, const double* cell,
               const uint8_t* pbc, double* energy, double* atom_energy, double* forces,
               double* virial) {
  if (!ctx || !pos || !Z || !cell || !energy || n <= 0) return SN_EINVAL;
  if (pbc && !(pbc[0] && pbc[1] && pbc[2])) {
    ctx->err = "only fully periodic cells are supported";
    return SN_EUNSUPPORTED;
  }
  const int64_t off[2] = {0, n};
  return sn_compute_batch(ctx, 1, off, pos, Z, cell, energy, atom_energy, forces, virial);
}

int sn_compute_noalloc(sn_ctx_t* ctx, int64_t n, const double* pos, const int32_t* Z,
                       const double* cell, const uint8_t* pbc, double* energy,
                       double* atom_energy, double* forces, double* virial) {
  if (!ctx || !pos || !Z || !cell || !energy || n <= 0) return SN_EINVAL;
  if (pbc && !(pbc[0] && pbc[1] && pbc[2])) {
    ctx->err = "only fully periodic cells are supported";
    return SN_EUNSUPPORTED;
  }
  const int64_t off[2] = {0, n};
  return guarded(ctx, [&] {
    char* base = scratch_address(ctx->device);  // guarded() made the device current
    // every buffer of this call is a slice of the device's scratch; the call always builds
    // its own graph, and none of its state survives it
    struct ArenaScope {
      sn_ctx* c;
      ArenaScope(sn_ctx* cc, char* b) : c(cc) {
        c->arena = b;
        c->arena_cap = kScratchBytes;
        c->arena_top = 0;
        c->arena_slots.clear();
        c->have_graph = false;
        c->pending = false;
      }
      ~ArenaScope() {
        c->arena = nullptr;
        c->arena_slots.clear();
        c->have_graph = false;
        c->pending = false;
      }
    } scope(ctx, base);
    compute_batch_host(ctx, 1, off, pos, Z, cell, energy, atom_energy, forces, virial);
  });
}

int sn_ctx_graph_size(const sn_ctx_t* ctx, int64_t* n_local, int64_t* n_ghost, int64_t* n_edge) {
  if (!ctx) return SN_EINVAL;
  if (n_local) *n_local = ctx->N;
  if (n_ghost) *n_ghost = ctx->G;
  if (n_edge) *n_edge = ctx->compacted ? ctx->E_built : ctx->E;
  return SN_OK;
}

int sn_ctx_evaluated_edges(const sn_ctx_t* ctx, int64_t* n_edge, int64_t* n_pair) {
  if (!ctx) return SN_EINVAL;
  if (n_edge) *n_edge = ctx->E;
  if (n_pair) *n_pair = ctx->NP;
  return SN_OK;
}

int sn_ctx_set_edge_compaction(sn_ctx_t* ctx, int on) {
  if (!ctx) return SN_EINVAL;
  ctx->compact = on != 0;
  return SN_OK;
}

int sn_ctx_set_capture(sn_ctx_t* ctx, int on) {
  if (!ctx) return SN_EINVAL;
  ctx->capture = on != 0;
  return SN_OK;
}

int sn_ctx_set_domains(sn_ctx_t* ctx, int nx, int ny, int nz) {
  if (!ctx || nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz > 4096) return SN_EINVAL;
  ctx->domains[0] = nx;
  ctx->domains[1] = ny;
  ctx->domains[2] = nz;
  ctx->have_graph = false;  // the next call rebuilds
  return SN_OK;
}

int sn_ctx_set_graph_reuse(sn_ctx_t* ctx, int reuse) {
  if (!ctx) return SN_EINVAL;
  ctx->reuse = reuse != 0;
  return SN_OK;
}

int sn_md_verlet(sn_ctx_t* ctx, int64_t n, double* d_pos, double* d_vel, const double* d_forces,
                 const double* d_inv_mass, double dt, int stage) {
  if (!ctx || !d_pos || !d_vel || !d_forces || !d_inv_mass || n <= 0 || (stage != 0 && stage != 1))
    return SN_EINVAL;
  return guarded(ctx, [&] {
    launch_verlet((int)n, d_pos, d_vel, d_forces, d_inv_mass, dt, stage, ctx->stream);
  });
}

int sn_md_nh_half(sn_ctx_t* ctx, int64_t n, double* d_vel, const double* d_inv_mass, double dt,
                  double kT, double dof, double Q, double* d_state) {
  if (!ctx || !d_vel || !d_inv_mass || !d_state || n <= 0 || n > INT32_MAX / 3 || !(dt > 0) ||
      !(kT > 0) || !(dof > 0) || !(Q > 0) || !std::isfinite(dt) || !std::isfinite(Q))
    return SN_EINVAL;
  return guarded(ctx, [&] {
    double* part = ctx->get<double>("md_partials", md_partials((int)n));
    launch_nh_half((int)n, d_vel, d_inv_mass, dt, dof * kT, Q, d_state, part, ctx->stream);
  });
}

int sn_md_max_displacement(sn_ctx_t* ctx, int64_t n, const double* d_pos, const double* d_ref,
                           double* max_disp) {
  if (!ctx || !d_pos || !d_ref || !max_disp || n <= 0 || n > INT32_MAX / 3) return SN_EINVAL;
  return guarded(ctx, [&] {
    double* part = ctx->get<double>("md_partials", md_partials((int)n));
    double* out = ctx->get<double>("md_max", 1);
    launch_max_disp2((int)n, d_pos, d_ref, part, out, ctx->stream);
    double h = 0;
    HIPCHK(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *max_disp = std::sqrt(h);
  });
}

int sn_ctx_memory(const sn_ctx_t* ctx, size_t* bytes) {
  if (!ctx || !bytes) return SN_EINVAL;
  *bytes = ctx->used + ctx->weight_bytes;
  return SN_OK;
}

int sn_ctx_pair_count(const sn_ctx_t* ctx, int64_t* n_pairs) {
  if (!ctx || !n_pairs) return SN_EINVAL;
  *n_pairs = ctx->NP;
  return SN_OK;
}

int sn_ctx_graph(const sn_ctx_t* cctx, int32_t* recv, int32_t* send_owner, int32_t* shift,
                 int32_t* ghost_owner, int32_t* ghost_shift) {
  sn_ctx_t* ctx = const_cast<sn_ctx_t*>(cctx);
  if (!ctx) return SN_EINVAL;
  if (!ctx->have_graph) {  // none built, or released, or built in the static scratch
    ctx->err = "no graph is held by the context";
    return SN_EBUSY;
  }
  return guarded(ctx, [&] {
    const int N = ctx->N, G = ctx->G;
    // the built list (of which the evaluated one may be a compaction)
    const int64_t E = ctx->compacted ? ctx->E_built : ctx->E;
    const std::string pre = ctx->compacted ? "full_" : "";
    hipStream_t s = ctx->stream;
    std::vector<int> order(N), owner(G), gsh(3 * (size_t)G), src(E), rcv(E);
    HIPCHK(hipMemcpyAsync(order.data(), ctx->get<int>("order", N), sizeof(int) * N,
                          hipMemcpyDeviceToHost, s));
    if (G) {
      HIPCHK(hipMemcpyAsync(owner.data(), ctx->get<int>("ghost_owner", G), sizeof(int) * G,
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(gsh.data(), ctx->get<int>("ghost_shift", 3 * (int64_t)G),
                            sizeof(int) * 3 * G, hipMemcpyDeviceToHost, s));
    }
    if (E) {
      HIPCHK(hipMemcpyAsync(src.data(), ctx->get<int>(pre + "src", E), sizeof(int) * E,
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(rcv.data(), ctx->get<int>(pre + "recv", E), sizeof(int) * E,
                            hipMemcpyDeviceToHost, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    for (int64_t e = 0; e < E; ++e) {
      const int sd = src[e];
      const int own = sd < N ? sd : owner[sd - N];
      if (recv) recv[e] = order[rcv[e]];
      if (send_owner) send_owner[e] = order[own];
      if (shift)
        for (int a = 0; a < 3; ++a) shift[3 * e + a] = sd < N ? 0 : gsh[3 * (size_t)(sd - N) + a];
    }
    for (int g = 0; g < G; ++g) {
      if (ghost_owner) ghost_owner[g] = order[owner[g]];
      if (ghost_shift)
        for (int a = 0; a < 3; ++a) ghost_shift[3 * g + a] = gsh[3 * (size_t)g + a];
    }
  });
}

int sn_ctx_timings(const sn_ctx_t* ctx, const char** names, double* ms, int* count) {
  if (!ctx || !count) return SN_EINVAL;
  int n = std::min<int>(*count, (int)ctx->timings.size());
  for (int i = 0; i < n; ++i) {
    if (names) names[i] = ctx->timings[i].first.c_str();
    if (ms) ms[i] = ctx->timings[i].second;
  }
  *count = (int)ctx->timings.size();
  return SN_OK;
}

}  // extern "C"
