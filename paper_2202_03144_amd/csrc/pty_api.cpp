// C ABI of the ptymi library: context ownership, validation, and the
// per-iteration phase schedule of ePIE, DM and LSQML (Sec. 2.3 of the ptychopy
// paper; step API of Sec. 3.2 / Fig. 3 / Listing 1).
#include "ptymi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <sstream>
#include <new>
#include <string>
#include <vector>

#include "pty_common.hpp"
#include "pty_kernels.hpp"

using namespace pty;

// Work space of pty_nll_forward_noalloc: one array per GPU, part of the code
// object, so no call ever allocates it.  In host code this name is only a
// stand-in: kernels and copies take the per-device address that
// noalloc_scratch() obtains from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[PTY_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of `scratch` on each GPU, looked up once per device at
// context set-up with that device current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices)
    throw DeviceError("no-allocation scratch: device " + std::to_string(device) + " beyond the table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      (void)hipGetLastError();
      throw DeviceError(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    g_scratch_addr[device] = ptr;
  }
  return g_scratch_addr[device];
}

thread_local std::string g_tls_error;

struct InvalidArg : std::runtime_error {
  explicit InvalidArg(const std::string& m) : std::runtime_error(m) {}
};
struct StateError : std::runtime_error {
  explicit StateError(const std::string& m) : std::runtime_error(m) {}
};
struct Unsupported : std::runtime_error {
  explicit Unsupported(const std::string& m) : std::runtime_error(m) {}
};

// Object tiles with the list of patches (slots) that overlap each of them.
struct TileSet {
  TileEntry* tiles = nullptr;
  PatchRef* refs = nullptr;
  int ntiles = 0;
  int nrefs = 0;
  size_t tiles_cap = 0, refs_cap = 0;   // allocated entries (lists are rebuilt in place)
};

// A set of positions iterated together (DM: all; LSQML: one group).
struct Group {
  std::vector<int> jl;   // slot -> pattern index
  int* d_jl = nullptr;   // device copy
  TileSet tiles;
};

}  // namespace

struct pty_ctx {
  int N = 0, K = 0, J = 0, H = 0, W = 0, device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  std::vector<std::pair<void*, size_t>> allocs;
  size_t mem = 0, mem_limit = 0;

  // state
  float2* obj = nullptr;
  float2* probe = nullptr;
  float2* probe_alt = nullptr;
  float* amp = nullptr;
  unsigned char* mask = nullptr;   // detector mask, natural order, 1 = measured
  bool have_mask = false;
  PosInfo* pos = nullptr;
  float2* tw = nullptr;
  int* jl_identity = nullptr;
  std::vector<PosInfo> hpos;
  bool have_patterns = false, have_positions = false, have_object = false, have_probe = false;
  int iter = 0;

  // error history (device, one double per iteration)
  double* err_dev = nullptr;
  int err_cap = 0;

  // work buffers (allocated on first use, grown as needed)
  float2* zs = nullptr;            size_t zs_patterns = 0;
  float2* psi = nullptr;
  float2* contrib = nullptr;       size_t contrib_slots = 0;
  float2* chi = nullptr;           size_t chi_slots = 0;
  double* errp = nullptr;
  double* posgrad = nullptr;       size_t posgrad_slots = 0;
  float* den = nullptr;
  float2* dobj = nullptr;
  unsigned* scal = nullptr;        // [0] max den_O, [1] max den_P (float bits)
  float* pint = nullptr;
  float2* part_num = nullptr;      size_t part_slices = 0;
  float* part_den = nullptr;
  float2* num_p = nullptr;
  float2* num_p2 = nullptr;
  float* den_p = nullptr;
  float2* dprobe = nullptr;
  double* loss_dev = nullptr;
  float2* lsq_pq = nullptr;
  float* lsq_dint = nullptr;
  double* lsq_part = nullptr;      size_t lsq_part_n = 0;
  float2* alpha = nullptr;         size_t alpha_slots = 0;
  float2* alpha_by_j = nullptr;
  float2* shift = nullptr;         size_t shift_slots = 0;   // LSQML position shifts per slot
  double* poisp = nullptr;         size_t poisp_n = 0;       // Poisson step length per slot
  float* pinten_c = nullptr;       size_t pinten_c_n = 0;    // Poisson: chunk x N x N model intensity
  double2* mode_gram = nullptr;    // K x K Gram matrix of the probe modes
  float2* mode_mix = nullptr;      // K x K mixing matrix of the orthogonalisation
  int* epie_order = nullptr;       // device copy of a shuffled ePIE order
  unsigned* epie_max = nullptr;    // per position of an iteration: the two ePIE step normalisers
  float2* epie_patch = nullptr;    // N x N: the pre-update patch of the current ePIE position
  float* epw_max = nullptr;        // 512 x 512 ePIE: per row block the two step maxima
  double* epw_err = nullptr;       // 512 x 512 ePIE: per column block the two error sums
  // adjoint with positions supplied on the device: their PosInfo form and
  // device-built tile lists over all object tiles
  PosInfo* adj_pos = nullptr;
  int* adj_cnt = nullptr;
  TileEntry* adj_tiles = nullptr;
  PatchRef* adj_refs = nullptr;

  // device-side iteration counter (error / NRMSE history slot of the running
  // iteration), so that one captured iteration can be replayed
  int* iter_dev = nullptr;
  uint64_t gen = 0;                // bumped by every device (de)allocation
  // captured iterations: replayed while the key (algorithm, parameters, probe
  // update on/off, buffers, state flags) matches
  struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int algo = -1;
    bool pon = false, dm_valid = false, den_valid = false;
    bool dm_valid_after = false, den_valid_after = false;
    pty_iter_params p{};
    uint64_t gen = 0;
    const float2* probe = nullptr;
    bool have_truth = false;
  };
  std::vector<GraphEntry> graphs;
  int tuned_chunk = 0;             // from pty_autotune; 0 = the default rule
  int tuned_slice = 0;             // probe-sum patterns per slice from pty_autotune; 0 = the rule

  // evaluation against a known object: invariant NRMSE on a region of interest
  float2* truth = nullptr;
  unsigned char* roi = nullptr;
  double* nrmse_dev = nullptr;     // one per iteration (capacity err_cap)
  double* nrmse_part = nullptr;
  double* eval_dev = nullptr;      // scratch scalars
  bool have_truth = false;
  // learned seed
  float* seed_patches = nullptr;   size_t seed_patches_n = 0;
  float2* seed_obj = nullptr;
  // stitching work buffers (kept between calls)
  int2* st_t = nullptr;            size_t st_t_n = 0;
  int* st_beg = nullptr;           size_t st_beg_n = 0;
  int* st_idx = nullptr;           size_t st_idx_n = 0;
  float2* st_S = nullptr;          size_t st_S_n = 0;
  float2* st_ph = nullptr;         size_t st_ph_n = 0;

  bool dm_valid = false;           // psi / contrib consistent with object and probe
  bool den_valid = false;          // den holds sum_j S_j^T sum_k |P_k|^2 for all positions
  Group all;                       // DM: every position
  std::vector<Group> groups;       // LSQML groups
  int groups_batch = -1;

  // kernel timing (families as in the header)
  static constexpr int kFamilies = PTY_TIMING_FAMILIES;
  struct Pending {
    int fam;
    hipEvent_t a, b;
  };
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<Pending> pending;
  double fam_ms[kFamilies] = {};
  int64_t fam_n[kFamilies] = {};

  hipEvent_t get_event() {
    if (!ev_pool.empty()) {
      hipEvent_t e = ev_pool.back();
      ev_pool.pop_back();
      return e;
    }
    hipEvent_t e;
    PTY_HIP(hipEventCreate(&e));
    return e;
  }
  void drain_timing() {
    if (pending.empty()) return;
    PTY_HIP(hipStreamSynchronize(stream));
    for (auto& p : pending) {
      float ms = 0.f;
      PTY_HIP(hipEventElapsedTime(&ms, p.a, p.b));
      fam_ms[p.fam] += ms;
      fam_n[p.fam] += 1;
      ev_pool.push_back(p.a);
      ev_pool.push_back(p.b);
    }
    pending.clear();
  }

  void set_device() const { PTY_HIP(hipSetDevice(device)); }

  void* dalloc(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (mem_limit && mem + bytes > mem_limit)
      throw NoMemError("device memory limit (PTY_MEM_LIMIT) reached");
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw NoMemError(std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    }
    allocs.emplace_back(p, bytes);
    mem += bytes;
    ++gen;
    return p;
  }
  void dfree(void* p) {
    if (!p) return;
    for (size_t i = 0; i < allocs.size(); ++i) {
      if (allocs[i].first == p) {
        mem -= allocs[i].second;
        allocs.erase(allocs.begin() + i);
        (void)hipFree(p);
        ++gen;
        return;
      }
    }
  }
  template <typename T>
  T* alloc(size_t n) { return static_cast<T*>(dalloc(n * sizeof(T))); }

  // Replaces *slot by a new buffer of n elements if it holds fewer than n.
  template <typename T>
  void ensure(T*& buf, size_t& have, size_t n) {
    if (buf && have >= n) return;
    T* nb = alloc<T>(n);
    dfree(buf);
    buf = nb;
    have = n;
  }
  template <typename T>
  void ensure_once(T*& buf, size_t n) {
    if (!buf) buf = alloc<T>(n);
  }

  void drop_graphs() {
    for (auto& g : graphs) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    graphs.clear();
  }

  ~pty_ctx() {
    drop_graphs();
    for (auto& p : pending) {
      ev_pool.push_back(p.a);
      ev_pool.push_back(p.b);
    }
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    for (auto& a : allocs) (void)hipFree(a.first);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

pty_status fail(pty_ctx* ctx, pty_status st, const std::string& msg) {
  if (ctx) ctx->err = msg;
  g_tls_error = msg;
  if (std::getenv("PTY_LOG")) std::fprintf(stderr, "[ptymi] %s\n", msg.c_str());
  return st;
}

template <typename F>
pty_status guarded(pty_ctx* ctx, F&& f) {
  try {
    f();
    return PTY_OK;
  } catch (const InvalidArg& e) {
    return fail(ctx, PTY_E_INVALID, e.what());
  } catch (const StateError& e) {
    return fail(ctx, PTY_E_STATE, e.what());
  } catch (const Unsupported& e) {
    return fail(ctx, PTY_E_UNSUPPORTED, e.what());
  } catch (const NoMemError& e) {
    return fail(ctx, PTY_E_NOMEM, e.what());
  } catch (const DeviceError& e) {
    return fail(ctx, PTY_E_DEVICE, e.what());
  } catch (const std::bad_alloc&) {
    return fail(ctx, PTY_E_NOMEM, "host allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(ctx, PTY_E_INVALID, e.what());
  } catch (const std::exception& e) {
    return fail(ctx, PTY_E_DEVICE, e.what());
  } catch (...) {
    return fail(ctx, PTY_E_DEVICE, "unknown error");
  }
}

void require(bool ok, const char* msg) {
  if (!ok) throw InvalidArg(msg);
}

enum Fam { kRowsFwd = 0, kCols, kRowsInv, kObjGather, kProbeAcc, kProbeFin, kLsqSteps, kEpie, kOther };

// Runs a launch; when timing is on, brackets it with events on the stream.
template <typename F>
void timed(pty_ctx* c, int fam, F&& f) {
  if (!c->timing) {
    f();
    return;
  }
  hipEvent_t a = c->get_event(), b = c->get_event();
  PTY_HIP(hipEventRecord(a, c->stream));
  f();
  PTY_HIP(hipEventRecord(b, c->stream));
  c->pending.push_back({fam, a, b});
  if (c->pending.size() > 50000) c->drain_timing();
}

bool supported_n(int n) { return n == 32 || n == 64 || n == 128 || n == 256 || n == 512; }

void copy_in(pty_ctx* c, void* dst, const void* src, size_t bytes, int on_device) {
  PTY_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
  PTY_HIP(hipStreamSynchronize(c->stream));
}

void copy_out(pty_ctx* c, void* dst, const void* src, size_t bytes, int on_device) {
  PTY_HIP(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  PTY_HIP(hipStreamSynchronize(c->stream));
}

// Host-side tile lists: for every object tile the patches whose (N+1)^2
// footprint overlaps it, in slot order.
void build_tiles(pty_ctx* c, Group& g) {
  const int nty = (c->H + kTileH - 1) / kTileH, ntx = (c->W + kTileW - 1) / kTileW;
  const size_t nt = size_t(nty) * ntx;
  auto span = [&](const PosInfo& p, int& y0, int& y1, int& x0, int& x1) {
    y0 = p.iy / kTileH;
    y1 = std::min(nty - 1, (p.iy + c->N) / kTileH);
    x0 = p.ix / kTileW;
    x1 = std::min(ntx - 1, (p.ix + c->N) / kTileW);
  };
  // counting sort by tile: entries per tile, tile offsets, then the entries
  // in slot order within each tile
  std::vector<int> cnt(nt, 0);
  for (int s = 0; s < (int)g.jl.size(); ++s) {
    int y0, y1, x0, x1;
    span(c->hpos[g.jl[s]], y0, y1, x0, x1);
    for (int ty = y0; ty <= y1; ++ty)
      for (int tx = x0; tx <= x1; ++tx) ++cnt[size_t(ty) * ntx + tx];
  }
  std::vector<TileEntry> tiles;
  std::vector<int> next(nt, 0);
  int total = 0;
  for (int ty = 0; ty < nty; ++ty)
    for (int tx = 0; tx < ntx; ++tx) {
      const size_t t = size_t(ty) * ntx + tx;
      if (!cnt[t]) continue;
      tiles.push_back({ty * kTileH, tx * kTileW, total, total + cnt[t]});
      next[t] = total;
      total += cnt[t];
    }
  std::vector<PatchRef> refs(total);
  for (int s = 0; s < (int)g.jl.size(); ++s) {
    const int j = g.jl[s];
    const PosInfo& p = c->hpos[j];
    int y0, y1, x0, x1;
    span(p, y0, y1, x0, x1);
    for (int ty = y0; ty <= y1; ++ty)
      for (int tx = x0; tx <= x1; ++tx) refs[next[size_t(ty) * ntx + tx]++] = {s, j, p.iy, p.ix, p.fy, p.fx, 0, 0};
  }
  g.tiles.ntiles = (int)tiles.size();
  g.tiles.nrefs = (int)refs.size();
  // reuse the lists' buffers when they are large enough (position refinement
  // rebuilds them every iteration), with a quarter of headroom when growing
  if (!g.tiles.tiles || g.tiles.tiles_cap < tiles.size()) {
    const size_t cap = std::max<size_t>(1, tiles.size() + tiles.size() / 4);
    TileEntry* nb = c->alloc<TileEntry>(cap);
    c->dfree(g.tiles.tiles);
    g.tiles.tiles = nb;
    g.tiles.tiles_cap = cap;
  }
  if (!g.tiles.refs || g.tiles.refs_cap < refs.size()) {
    const size_t cap = std::max<size_t>(1, refs.size() + refs.size() / 4);
    PatchRef* nb = c->alloc<PatchRef>(cap);
    c->dfree(g.tiles.refs);
    g.tiles.refs = nb;
    g.tiles.refs_cap = cap;
  }
  PTY_HIP(hipMemcpy(g.tiles.tiles, tiles.data(), tiles.size() * sizeof(TileEntry), hipMemcpyHostToDevice));
  PTY_HIP(hipMemcpy(g.tiles.refs, refs.data(), refs.size() * sizeof(PatchRef), hipMemcpyHostToDevice));
}

void free_group(pty_ctx* c, Group& g) {
  c->dfree(g.d_jl);
  c->dfree(g.tiles.tiles);
  c->dfree(g.tiles.refs);
  g = Group{};
}

void make_group(pty_ctx* c, Group& g, std::vector<int> jl) {
  g.jl = std::move(jl);
  g.d_jl = c->alloc<int>(g.jl.size());
  PTY_HIP(hipMemcpy(g.d_jl, g.jl.data(), g.jl.size() * sizeof(int), hipMemcpyHostToDevice));
  build_tiles(c, g);
}

void ensure_all_group(pty_ctx* c) {
  if (c->all.d_jl) return;
  std::vector<int> jl(c->J);
  for (int j = 0; j < c->J; ++j) jl[j] = j;
  make_group(c, c->all, std::move(jl));
}

void ensure_lsq_groups(pty_ctx* c, int batch) {
  const int G = std::max(1, (c->J + batch - 1) / batch);
  if (c->groups_batch == batch && (int)c->groups.size() == G) return;
  for (auto& g : c->groups) free_group(c, g);
  c->groups.clear();
  c->groups.resize(G);
  for (int g = 0; g < G; ++g) {
    std::vector<int> jl;
    for (int j = g; j < c->J; j += G) jl.push_back(j);
    make_group(c, c->groups[g], std::move(jl));
  }
  c->groups_batch = batch;
}

// Patterns per Fourier-pass launch: as many as a 96 MB scratch budget holds
// (inside the 256 MB Infinity Cache), rounded down to a whole number of block
// waves over the 256 compute units (a ragged last wave of blocks left the
// passes ~15% slower at 256^2).  pty_autotune can replace it.
int chunk_patterns(const pty_ctx* c, const pty_iter_params& p) {
  if (p.chunk > 0) return p.chunk;
  if (c->tuned_chunk > 0) return c->tuned_chunk;
  const size_t per = size_t(c->K) * c->N * c->N * sizeof(float2);
  const size_t budget = size_t(96) << 20;
  const int fit = (int)std::max<size_t>(1, budget / per);
  const int wave = std::max(1, 256 / row_blocks(c->N));   // patterns per 256 blocks
  return fit >= wave ? fit / wave * wave : fit;
}


// Common work buffers of the Fourier passes.
void ensure_common(pty_ctx* c, int chunk, size_t slots) {
  const size_t nn = size_t(c->N) * c->N;
  c->ensure(c->zs, c->zs_patterns, size_t(chunk) * c->K * nn);
  c->ensure(c->contrib, c->contrib_slots, slots * nn);
  c->ensure_once(c->errp, size_t(c->J) * col_blocks(c->N, c->K) * 2);
  c->ensure_once(c->den, size_t(c->H) * c->W);
  c->ensure_once(c->scal, 16);
  c->ensure_once(c->pint, nn);
  c->ensure_once(c->num_p, size_t(c->K) * nn);
  c->ensure_once(c->num_p2, size_t(c->K) * nn);
  c->ensure_once(c->den_p, nn);
  c->ensure_once(c->dprobe, size_t(c->K) * nn);
}

void ensure_err_slot(pty_ctx* c, int n_iter) {
  if (!c->iter_dev) {
    c->iter_dev = c->alloc<int>(1);
    launch_set_i32(c->iter_dev, c->iter, c->stream);
  }
  if (c->err_dev && c->iter + n_iter <= c->err_cap) return;
  int cap = std::max(256, c->err_cap);
  while (cap < c->iter + n_iter) cap *= 2;
  double* nb = c->alloc<double>(cap);
  double* nr = c->alloc<double>(cap);
  if (c->err_dev && c->iter > 0) {
    PTY_HIP(hipMemcpyAsync(nb, c->err_dev, sizeof(double) * c->iter, hipMemcpyDeviceToDevice, c->stream));
    PTY_HIP(hipMemcpyAsync(nr, c->nrmse_dev, sizeof(double) * c->iter, hipMemcpyDeviceToDevice, c->stream));
  }
  PTY_HIP(hipStreamSynchronize(c->stream));
  c->dfree(c->err_dev);
  c->dfree(c->nrmse_dev);
  c->err_dev = nb;
  c->nrmse_dev = nr;
  c->err_cap = cap;
}

// Closes iteration t: records the NRMSE against the truth, if one is set.
// Records E of iteration t (and the NRMSE against the truth, if one is set) in
// the device histories at the device counter's slot, advances that counter,
// and closes the iteration.
void end_iteration(pty_ctx* c, int t) {
  (void)t;
  timed(c, kOther, [&] {
    launch_err_reduce(c->errp, c->J * col_blocks(c->N, c->K), c->err_dev, c->stream, c->iter_dev, !c->have_truth);
  });
  if (c->have_truth)
    timed(c, kOther, [&] {
      launch_nrmse(c->obj, c->truth, c->roi, size_t(c->H) * c->W, c->nrmse_part, c->nrmse_dev, c->stream,
                   c->iter_dev, true);
    });
  c->iter++;
}

FourierArgs fourier_args(pty_ctx* c, const Group& g) {
  FourierArgs a{};
  a.n = c->N;
  a.k = c->K;
  a.obj = c->obj;
  a.h = c->H;
  a.w = c->W;
  a.probe = c->probe;
  a.jlist = g.d_jl;
  a.pos = c->pos;
  a.amp = c->amp;
  a.psi = c->psi;
  a.chi = c->chi;
  a.contrib = c->contrib;
  a.zs = c->zs;
  a.errp = c->errp;
  a.posgrad = c->posgrad;
  a.tw = reinterpret_cast<const float*>(c->tw);
  a.nll_eps = 1e-6f;
  a.masked = c->have_mask ? 1 : 0;
  a.stream = c->stream;
  return a;
}

// Forward rows, columns with the modulus projection, inverse rows, over the
// slots [s0, s0 + count) of group g in chunks.
void fourier_pass(pty_ctx* c, const Group& g, int s0, int count, int chunk, RowIn in, ColOp op,
                  RowOut out, bool inverse = true) {
  FourierArgs a = fourier_args(c, g);
  for (int off = 0; off < count; off += chunk) {
    a.jl_off = s0 + off;
    a.slot_off = s0 + off;
    a.nc = std::min(chunk, count - off);
    timed(c, kRowsFwd, [&] { launch_rows_fwd(a, in); });
    a.poisp = op == ColOp::Poisson ? c->poisp : nullptr;
    a.pinten = op == ColOp::Poisson ? c->pinten_c : nullptr;
    timed(c, kCols, [&] { launch_cols(a, op); });
    if (op == ColOp::Poisson) timed(c, kCols, [&] { launch_poisson_alpha(a); });
    if (inverse && op != ColOp::Intensity) timed(c, kRowsInv, [&] { launch_rows_inv(a, out); });
  }
}

ObjGatherArgs obj_args(pty_ctx* c, const Group& g) {
  ObjGatherArgs o{};
  o.n = c->N;
  o.h = c->H;
  o.w = c->W;
  o.tiles = g.tiles.tiles;
  o.ntiles = g.tiles.ntiles;
  o.refs = g.tiles.refs;
  o.pos = c->pos;
  o.src = c->contrib;
  o.pint = c->pint;
  o.alpha = c->alpha;
  o.obj = c->obj;
  o.den = c->den;
  o.den_max = c->scal;
  o.stream = c->stream;
  return o;
}

// den_O = sum over the group of S_j^T sum_k |P_k|^2 and its maximum
void density(pty_ctx* c, const Group& g) {
  timed(c, kOther, [&] { launch_probe_intensity(c->probe, c->pint, c->N, c->K, c->stream, c->scal); });
  ObjGatherArgs o = obj_args(c, g);
  timed(c, kObjGather, [&] { launch_obj_gather(o, ObjOp::Density); });
}

// Probe sums over slots [0, count) of group g: part -> num_p / den_p
void probe_reduce(pty_ctx* c, const Group& g, const float2* src, int by_pattern, PrbOp op,
                  float2* num, bool with_den, const float2* obj = nullptr, const PosInfo* pos = nullptr) {
  const int count = (int)g.jl.size();
  const int per_slice = c->tuned_slice > 0 ? c->tuned_slice : probe_per_slice(c->N, count);
  const int slices = probe_slices(count, per_slice);
  ProbeAccArgs pa{};
  pa.n = c->N;
  pa.k = c->K;
  pa.obj = obj ? obj : c->obj;
  pa.h = c->H;
  pa.w = c->W;
  pa.jlist = g.d_jl;
  pa.pos = pos ? pos : c->pos;
  pa.src = src;
  pa.src_by_pattern = by_pattern;
  pa.alpha = c->alpha;
  pa.s0 = 0;
  pa.count = count;
  pa.per_slice = per_slice;
  pa.part_num = c->part_num;
  pa.part_den = c->part_den;
  pa.zero = with_den ? c->scal + 1 : nullptr;   // the finish's max of den_P
  pa.stream = c->stream;
  timed(c, kProbeAcc, [&] { launch_probe_acc(pa, op); });
  ProbeFinishArgs pf{};
  pf.n = c->N;
  pf.k = c->K;
  pf.slices = slices;
  pf.part_num = c->part_num;
  pf.part_den = with_den ? c->part_den : nullptr;
  pf.num = num;
  pf.den = with_den ? c->den_p : nullptr;
  pf.den_max = with_den ? c->scal + 1 : nullptr;
  pf.stream = c->stream;
  timed(c, kProbeFin, [&] { launch_probe_finish(pf); });
}

void ensure_probe_parts(pty_ctx* c, int count) {
  const int slices = std::max(probe_slices_max(c->N, count), c->tuned_slice > 0 ? probe_slices(count, c->tuned_slice) : 0);
  const size_t nn = size_t(c->N) * c->N;
  size_t have = c->part_slices;
  if (c->part_num && have >= size_t(slices) * c->K * nn && c->part_den) return;
  c->dfree(c->part_num);
  c->dfree(c->part_den);
  c->part_num = c->alloc<float2>(size_t(slices) * c->K * nn);
  c->part_den = c->alloc<float>(size_t(slices) * nn);
  c->part_slices = size_t(slices) * c->K * nn;
}

void probe_apply(pty_ctx* c, PrbApply op, const float2* num, float gamma, float beta) {
  ProbeApplyArgs ap{};
  ap.n = c->N;
  ap.k = c->K;
  ap.num = num;
  ap.den = c->den_p;
  ap.den_max = c->scal + 1;
  ap.gamma = gamma;
  ap.beta = beta;
  ap.probe = c->probe;
  ap.dir = c->dprobe;
  ap.stream = c->stream;
  timed(c, kProbeFin, [&] { launch_probe_apply(ap, op); });
}

void require_loaded(pty_ctx* c) {
  if (!c->have_patterns) throw StateError("patterns not loaded");
  if (!c->have_positions) throw StateError("positions not loaded");
  if (!c->have_object) throw StateError("object not set");
  if (!c->have_probe) throw StateError("probe not set");
}

bool probe_on(const pty_iter_params& p, int t) { return p.probe_update_start >= 0 && t >= p.probe_update_start; }

// Orthogonal probe modes after an iteration that updated the probe (and the
// DM exit waves alike), when the parameters ask for it.
// Its two K x K scratch matrices are allocated with the other work buffers,
// before any iteration (a captured iteration must not allocate).
void ensure_mode_scratch(pty_ctx* c, const pty_iter_params& p) {
  if (!(p.flags & PTY_ITER_ORTHO_MODES) || c->K <= 1) return;
  c->ensure_once(c->mode_gram, size_t(c->K) * c->K);
  c->ensure_once(c->mode_mix, size_t(c->K) * c->K);
}

void maybe_orthogonalise(pty_ctx* c, const pty_iter_params& p, bool pon, float2* psi) {
  if (!(p.flags & PTY_ITER_ORTHO_MODES) || !pon || c->K <= 1) return;
  timed(c, kOther, [&] {
    launch_orthogonalise_modes(c->probe, psi, c->N, c->K, c->J, c->mode_gram, c->mode_mix, c->stream);
  });
  c->den_valid = false;
}

// ---------------------------------------------------------------------------
// DM
// ---------------------------------------------------------------------------
void run_dm(pty_ctx* c, int n_iter, const pty_iter_params& p) {
  const float g_obj = p.gamma_obj < 0 ? 1e-6f : p.gamma_obj;
  const float g_prb = p.gamma_probe < 0 ? 1e-6f : p.gamma_probe;
  const int chunk = chunk_patterns(c, p);
  const size_t nn = size_t(c->N) * c->N;
  ensure_all_group(c);
  ensure_common(c, std::min(chunk, c->J), c->J);
  c->ensure_once(c->psi, size_t(c->J) * c->K * nn);
  ensure_probe_parts(c, c->J);
  ensure_err_slot(c, n_iter);
  ensure_mode_scratch(c, p);
  const Group& g = c->all;
  if (!c->dm_valid) {
    DmInitArgs di{};
    di.n = c->N;
    di.k = c->K;
    di.obj = c->obj;
    di.h = c->H;
    di.w = c->W;
    di.probe = c->probe;
    di.pos = c->pos;
    di.j = c->J;
    di.psi = c->psi;
    di.contrib = c->contrib;
    di.stream = c->stream;
    timed(c, kOther, [&] { launch_dm_init(di); });
    c->dm_valid = true;
    c->den_valid = false;
  }
  for (int it = 0; it < n_iter; ++it) {
    const int t = c->iter;
    if (!c->den_valid) {
      density(c, g);
      c->den_valid = true;
    }
    ObjGatherArgs o = obj_args(c, g);
    o.gamma = g_obj;
    timed(c, kObjGather, [&] { launch_obj_gather(o, ObjOp::DmObject); });
    if (probe_on(p, t)) {
      probe_reduce(c, g, c->psi, 1, PrbOp::Plain, c->num_p, true);
      probe_apply(c, PrbApply::Dm, c->num_p, g_prb, 1.f);
      c->den_valid = false;
    }
    fourier_pass(c, g, 0, c->J, chunk, RowIn::DmReflect, ColOp::Project, RowOut::DmUpdate);
    maybe_orthogonalise(c, p, probe_on(p, t), c->psi);
    end_iteration(c, t);
  }
}

// ---------------------------------------------------------------------------
// LSQML
// ---------------------------------------------------------------------------
// After positions moved on the device: the host copy, and every patch list
// built from it (LSQML groups now; the all-positions group on its next use).
void refresh_positions(pty_ctx* c) {
  PTY_HIP(hipMemcpyAsync(c->hpos.data(), c->pos, sizeof(PosInfo) * c->J, hipMemcpyDeviceToHost, c->stream));
  PTY_HIP(hipStreamSynchronize(c->stream));
  for (auto& g : c->groups) build_tiles(c, g);
  free_group(c, c->all);
  c->den_valid = false;
}

void run_lsqml(pty_ctx* c, int n_iter, const pty_iter_params& p) {
  const float g_obj = p.gamma_obj < 0 ? 1e-3f : p.gamma_obj;
  const float g_prb = p.gamma_probe < 0 ? 1e-3f : p.gamma_probe;
  const int batch = p.lsqml_batch > 0 ? p.lsqml_batch : 512;
  const int chunk = chunk_patterns(c, p);
  const size_t nn = size_t(c->N) * c->N;
  ensure_lsq_groups(c, batch);
  int bmax = 0;
  for (auto& g : c->groups) bmax = std::max(bmax, (int)g.jl.size());
  ensure_common(c, std::min(chunk, bmax), bmax);
  c->ensure(c->chi, c->chi_slots, size_t(bmax) * c->K * nn);
  c->ensure_once(c->dobj, size_t(c->H) * c->W);
  c->ensure(c->alpha, c->alpha_slots, size_t(bmax));
  c->ensure_once(c->alpha_by_j, size_t(c->J));
  const int nrb = lsq_row_blocks(c->N);  // row blocks of the step sums
  c->ensure_once(c->lsq_pq, nn);
  c->ensure_once(c->lsq_dint, nn);
  const bool refining = p.position_start >= 0 && p.position_start < c->iter + n_iter;
  c->ensure(c->lsq_part, c->lsq_part_n, size_t(bmax) * nrb * (refining ? 9 : 5));
  if (refining) c->ensure(c->shift, c->shift_slots, size_t(bmax));
  const bool poisson = (p.flags & PTY_ITER_POISSON) != 0;
  if (poisson) {
    c->ensure(c->poisp, c->poisp_n, size_t(bmax));
    c->ensure(c->pinten_c, c->pinten_c_n, size_t(std::min(chunk, bmax)) * nn);
  }
  ensure_probe_parts(c, bmax);
  ensure_err_slot(c, n_iter);
  ensure_mode_scratch(c, p);
  c->dm_valid = false;
  for (int it = 0; it < n_iter; ++it) {
    const int t = c->iter;
    const bool pon = probe_on(p, t);
    const bool refine = p.position_start >= 0 && t >= p.position_start;
    for (auto& g : c->groups) {
      const int count = (int)g.jl.size();
      density(c, g);
      fourier_pass(c, g, 0, count, chunk, RowIn::Plain, poisson ? ColOp::Poisson : ColOp::Project,
                   RowOut::StoreChi);
      ObjGatherArgs o = obj_args(c, g);
      o.gamma = g_obj;
      o.out = c->dobj;
      timed(c, kObjGather, [&] { launch_obj_gather(o, ObjOp::LsqDirection); });
      if (pon) {
        probe_reduce(c, g, c->chi, 0, PrbOp::Plain, c->num_p, true);
        probe_apply(c, PrbApply::LsqDirection, c->num_p, g_prb, 1.f);
      }
      LsqStepArgs ls{};
      ls.n = c->N;
      ls.k = c->K;
      ls.obj = c->obj;
      ls.dobj = c->dobj;
      ls.h = c->H;
      ls.w = c->W;
      ls.probe = c->probe;
      ls.dprobe = c->dprobe;
      ls.chi = c->chi;
      ls.contrib = c->contrib;
      ls.pint = c->pint;
      ls.pq = c->lsq_pq;
      ls.dint = c->lsq_dint;
      ls.jlist = g.d_jl;
      ls.pos = c->pos;
      ls.count = count;
      ls.probe_on = pon ? 1 : 0;
      ls.part = c->lsq_part;
      ls.alpha = c->alpha;
      ls.alpha_by_j = c->alpha_by_j;
      ls.shift = refine ? c->shift : nullptr;
      ls.max_shift = p.position_max_shift;
      ls.stream = c->stream;
      timed(c, kLsqSteps, [&] { launch_lsq_steps(ls); });
      if (pon) probe_reduce(c, g, c->chi, 0, PrbOp::AlphaWeighted, c->num_p2, false);
      ObjGatherArgs u = obj_args(c, g);
      u.gamma = g_obj;
      u.beta = p.beta_obj;
      timed(c, kObjGather, [&] { launch_obj_gather(u, ObjOp::LsqUpdate); });
      if (pon) probe_apply(c, PrbApply::LsqUpdate, c->num_p2, g_prb, p.beta_probe);
      if (refine)
        timed(c, kOther, [&] {
          launch_pos_update(c->pos, g.d_jl, c->shift, count, c->H - c->N, c->W - c->N, c->stream);
        });
    }
    maybe_orthogonalise(c, p, pon, nullptr);
    end_iteration(c, t);
    if (refine) refresh_positions(c);
  }
  c->den_valid = false;  // den holds the last group's density only
}

// ---------------------------------------------------------------------------
// ePIE
// ---------------------------------------------------------------------------
uint64_t splitmix64_next(uint64_t& s) {
  s += 0x9E3779B97F4A7C15ull;
  uint64_t z = s;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

void run_epie(pty_ctx* c, int n_iter, const pty_iter_params& p) {
  const size_t nn = size_t(c->N) * c->N;
  ensure_all_group(c);
  ensure_common(c, 1, 1);
  c->ensure(c->chi, c->chi_slots, size_t(c->K) * nn);
  ensure_err_slot(c, n_iter);
  ensure_mode_scratch(c, p);
  c->dm_valid = false;
  FourierArgs a = fourier_args(c, c->all);
  a.nc = 1;
  a.slot_off = 0;
  std::vector<int> order(c->J);
  for (int it = 0; it < n_iter; ++it) {
    const int t = c->iter;
    for (int j = 0; j < c->J; ++j) order[j] = j;
    if (p.order_seed != 0) {
      uint64_t st = p.order_seed + (uint64_t)t;
      for (int i = c->J - 1; i >= 1; --i) {
        const uint64_t k = splitmix64_next(st) % (uint64_t)(i + 1);
        std::swap(order[i], order[k]);
      }
    }
    const bool pon = probe_on(p, t);
    if (epie_fused_supported(c->N, c->K)) {
      // one workgroup runs the whole iteration; positions in `order`
      const int* d_order = c->all.d_jl;   // identity
      if (p.order_seed != 0) {
        c->ensure_once(c->epie_order, size_t(c->J));
        PTY_HIP(hipMemcpyAsync(c->epie_order, order.data(), sizeof(int) * c->J, hipMemcpyHostToDevice,
                               c->stream));
        d_order = c->epie_order;
      }
      EpieRunArgs r{};
      r.n = c->N;
      r.k = c->K;
      r.obj = c->obj;
      r.h = c->H;
      r.w = c->W;
      r.probe0 = c->probe;
      r.probe1 = c->probe_alt;
      r.amp = c->amp;
      r.pos = c->pos;
      r.order = d_order;
      r.count = c->J;
      r.errp = c->errp;
      r.bpp = col_blocks(c->N, c->K);
      r.tw = reinterpret_cast<const float*>(c->tw);
      r.alpha = p.alpha;
      r.beta = p.beta;
      r.probe_on = pon ? 1 : 0;
      r.stream = c->stream;
      timed(c, kEpie, [&] { launch_epie_fused(r); });
      if (c->J % 2 == 1) std::swap(c->probe, c->probe_alt);
      maybe_orthogonalise(c, p, pon, nullptr);
      end_iteration(c, t);
      continue;
    }
    c->ensure_once(c->epie_patch, nn);
    if (epie_wide_supported(c->N, c->K)) {
      // 512 x 512: one wavefront per line, three launches per position; with
      // probe updates the new probe goes to the other buffer
      c->ensure_once(c->epw_max, epie_wide_max_words());
      c->ensure_once(c->epw_err, epie_wide_err_words());
      EpieWideArgs w{};
      w.n = c->N;
      w.k = c->K;
      w.obj = c->obj;
      w.h = c->H;
      w.w = c->W;
      w.amp = c->amp;
      w.zs = c->zs;
      w.patch = c->epie_patch;
      w.contrib = c->contrib;
      w.maxw = c->epw_max;
      w.errw = c->epw_err;
      w.errp = c->errp;
      w.bpp = col_blocks(c->N, c->K);
      w.tw = reinterpret_cast<const float*>(c->tw);
      w.alpha = p.alpha;
      w.beta = p.beta;
      w.probe_on = pon ? 1 : 0;
      w.masked = c->have_mask ? 1 : 0;
      w.stream = c->stream;
      for (int j : order) {
        w.pos = c->hpos[j];
        w.j = j;
        w.probe = c->probe;
        w.probe_out = pon ? c->probe_alt : c->probe;
        timed(c, kEpie, [&] { launch_epie_wide(w); });
        if (pon) std::swap(c->probe, c->probe_alt);
      }
      maybe_orthogonalise(c, p, pon, nullptr);
      end_iteration(c, t);
      continue;
    }
    c->ensure_once(c->epie_max, size_t(2) * c->J);
    timed(c, kOther, [&] { launch_fill_u32(c->epie_max, size_t(2) * c->J, 0u, c->stream); });
    int slot = 0;
    for (int j : order) {
      a.jl_off = j;
      a.obj = c->obj;
      a.probe = c->probe;
      timed(c, kRowsFwd, [&] { launch_rows_fwd(a, RowIn::Plain); });
      timed(c, kCols, [&] { launch_cols(a, ColOp::Project); });
      timed(c, kRowsInv, [&] { launch_rows_inv(a, RowOut::StoreChi); });
      EpieArgs e{};
      e.n = c->N;
      e.k = c->K;
      e.obj = c->obj;
      e.h = c->H;
      e.w = c->W;
      e.probe = c->probe;
      e.probe_out = c->probe_alt;
      e.chi = c->chi;
      e.pos = c->hpos[j];
      e.alpha = p.alpha;
      e.beta = p.beta;
      e.probe_on = pon ? 1 : 0;
      e.maxes = c->epie_max + 2 * slot++;
      e.patch = c->epie_patch;
      e.stream = c->stream;
      timed(c, kEpie, [&] { launch_epie_update(e); });
      std::swap(c->probe, c->probe_alt);
    }
    maybe_orthogonalise(c, p, pon, nullptr);
    end_iteration(c, t);
  }
  c->den_valid = false;
}

// ---------------------------------------------------------------------------
// Poisson-likelihood adjoint
// ---------------------------------------------------------------------------
// The identity slot list 0..J-1 (device), made once.
const int* identity_slots(pty_ctx* c) {
  if (!c->jl_identity) {
    c->jl_identity = c->alloc<int>(size_t(c->J));
    launch_iota_i32(c->jl_identity, c->J, c->stream);
  }
  return c->jl_identity;
}

double run_nll(pty_ctx* c, const float2* obj, const float2* probe, const float* pos_yx, bool grad, float grad_out,
               float2* g_obj, float2* g_probe, float* g_pos) {
  if (!c->have_patterns) throw StateError("patterns not loaded");
  if (!pos_yx && !c->have_positions) throw StateError("positions not loaded (and none supplied)");
  pty_iter_params p;
  pty_default_params(&p);
  const int chunk = chunk_patterns(c, p);
  const size_t nn = size_t(c->N) * c->N;
  if (!pos_yx) ensure_all_group(c);
  ensure_common(c, std::min(chunk, c->J), grad ? c->J : 1);
  c->ensure_once(c->loss_dev, 2);
  if (grad) {
    c->ensure(c->chi, c->chi_slots, size_t(c->J) * c->K * nn);
    c->ensure(c->posgrad, c->posgrad_slots, size_t(c->J) * row_blocks(c->N) * 2);
    ensure_probe_parts(c, c->J);
  }
  Group dev_group;   // positions on the device: identity slots, device-built tiles
  const PosInfo* pos = c->pos;
  if (pos_yx) {
    const int nty = (c->H + kTileH - 1) / kTileH, ntx = (c->W + kTileW - 1) / kTileW;
    c->ensure_once(c->adj_pos, size_t(c->J));
    dev_group.d_jl = const_cast<int*>(identity_slots(c));
    timed(c, kOther, [&] { launch_pos_from_yx(pos_yx, c->J, c->H - c->N, c->W - c->N, c->adj_pos, c->stream); });
    pos = c->adj_pos;
    if (grad && g_obj) {
      c->ensure_once(c->adj_cnt, size_t(nty) * ntx);
      c->ensure_once(c->adj_tiles, size_t(nty) * ntx);
      c->ensure_once(c->adj_refs, device_tile_refs_max(c->N, c->J));
      timed(c, kOther, [&] {
        launch_build_tiles(pos, dev_group.d_jl, c->J, c->N, c->H, c->W, c->adj_cnt, c->adj_tiles, c->adj_refs,
                           c->stream);
      });
      dev_group.tiles.tiles = c->adj_tiles;
      dev_group.tiles.refs = c->adj_refs;
      dev_group.tiles.ntiles = nty * ntx;
    }
    dev_group.jl.resize(c->J);
  }
  const Group& g = pos_yx ? dev_group : c->all;
  FourierArgs a = fourier_args(c, g);
  a.pos = pos;
  a.obj = obj;
  a.probe = probe;
  a.chi = c->chi;
  a.posgrad = c->posgrad;
  a.grad_scale = grad_out;
  for (int off = 0; off < c->J; off += chunk) {
    a.jl_off = off;
    a.slot_off = off;
    a.nc = std::min(chunk, c->J - off);
    timed(c, kRowsFwd, [&] { launch_rows_fwd(a, RowIn::Plain); });
    timed(c, kCols, [&] { launch_cols(a, grad ? ColOp::NllGrad : ColOp::NllLoss); });
    if (grad) timed(c, kRowsInv, [&] { launch_rows_inv(a, RowOut::NllGrad); });
  }
  timed(c, kOther, [&] { launch_err_reduce(c->errp, c->J * col_blocks(c->N, c->K), c->loss_dev, c->stream); });
  if (grad && g_obj) {
    timed(c, kOther, [&] { launch_fill_u32(reinterpret_cast<unsigned*>(g_obj), size_t(c->H) * c->W * 2, 0u, c->stream); });
    ObjGatherArgs o = obj_args(c, g);
    o.pos = pos;
    o.out = g_obj;
    timed(c, kObjGather, [&] { launch_obj_gather(o, ObjOp::Gradient); });
  }
  if (grad && g_probe) probe_reduce(c, g, c->chi, 0, PrbOp::Gradient, g_probe, false, obj, pos);
  if (grad && g_pos)
    timed(c, kOther, [&] { launch_posgrad_reduce(c->posgrad, c->J, row_blocks(c->N), g_pos, g.d_jl, c->stream); });
  double loss = 0.0;
  PTY_HIP(hipMemcpyAsync(&loss, c->loss_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  PTY_HIP(hipStreamSynchronize(c->stream));
  return loss;
}

// ---------------------------------------------------------------------------
// Evaluation and the learned seed
// ---------------------------------------------------------------------------
// Amplitude error E of the current object and probe over all positions
// (forward rows, columns with the projection's error partials, no inverse).
// sub: only the patterns of that group (the others' partials are zeroed).
double model_error(pty_ctx* c, const Group* sub = nullptr) {
  pty_iter_params p;
  pty_default_params(&p);
  const int chunk = chunk_patterns(c, p);
  if (!sub) ensure_all_group(c);
  ensure_common(c, std::min(chunk, c->J), 1);
  c->ensure_once(c->eval_dev, 8);
  if (sub)
    launch_fill_u32(reinterpret_cast<unsigned*>(c->errp), size_t(c->J) * col_blocks(c->N, c->K) * 4, 0u,
                    c->stream);
  const Group& g = sub ? *sub : c->all;
  fourier_pass(c, g, 0, (int)g.jl.size(), chunk, RowIn::Plain, ColOp::Project, RowOut::StoreChi, false);
  launch_err_reduce(c->errp, c->J * col_blocks(c->N, c->K), c->eval_dev, c->stream);
  double e = 0.0;
  PTY_HIP(hipMemcpyAsync(&e, c->eval_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  PTY_HIP(hipStreamSynchronize(c->stream));
  return e;
}

// Placement of each predicted patch: the central N/2 x N/2 of the window at
// the nearest integer position.
// placements of the windows `sel` (all when empty)
std::vector<int2> seed_placements(const pty_ctx* c, const std::vector<int>& sel) {
  const int m = sel.empty() ? c->J : (int)sel.size();
  std::vector<int2> t(m);
  for (int i = 0; i < m; ++i) {
    const PosInfo& p = c->hpos[sel.empty() ? i : sel[i]];
    t[i] = make_int2(p.iy + (p.fy >= 0.5f ? 1 : 0) + c->N / 4, p.ix + (p.fx >= 0.5f ? 1 : 0) + c->N / 4);
  }
  return t;
}

// Stitches the patches of windows `sel` (all when empty; |sel| x 64 x 64 x
// (amplitude, phase), device, in that order) into dst: with `chain`, each
// patch first gets the phase factor of the sequential chain; without, the
// patches are averaged as they are.
void stitch(pty_ctx* c, const float* patches, float2* dst, const std::vector<int>& sel = {}, bool chain = true) {
  if (c->N != 128) throw Unsupported("stitching needs 128 x 128 windows (64 x 64 patches)");
  const std::vector<int2> t = seed_placements(c, sel);
  const int m = (int)t.size();
  const int bh = (c->H + 63) / 64, bw = (c->W + 63) / 64;
  std::vector<int> beg(size_t(bh) * bw + 1, 0), idx(m);
  for (int j = 0; j < m; ++j) beg[size_t(t[j].x / 64) * bw + t[j].y / 64 + 1]++;
  for (size_t b = 0; b < size_t(bh) * bw; ++b) beg[b + 1] += beg[b];
  std::vector<int> fill(beg.begin(), beg.end() - 1);
  for (int j = 0; j < m; ++j) idx[fill[size_t(t[j].x / 64) * bw + t[j].y / 64]++] = j;
  const int gs = seed_chain_grid();
  const int hc = (c->H + gs - 1) / gs, wc = (c->W + gs - 1) / gs;
  c->ensure(c->st_t, c->st_t_n, size_t(std::max(m, 1)));
  c->ensure(c->st_beg, c->st_beg_n, beg.size());
  c->ensure(c->st_idx, c->st_idx_n, size_t(std::max(m, 1)));
  c->ensure(c->st_ph, c->st_ph_n, size_t(std::max(m, 1)));
  if (chain) c->ensure(c->st_S, c->st_S_n, size_t(hc) * wc);
  PTY_HIP(hipMemcpyAsync(c->st_t, t.data(), sizeof(int2) * m, hipMemcpyHostToDevice, c->stream));
  PTY_HIP(hipMemcpyAsync(c->st_beg, beg.data(), sizeof(int) * beg.size(), hipMemcpyHostToDevice, c->stream));
  PTY_HIP(hipMemcpyAsync(c->st_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice, c->stream));
  if (chain) {
    launch_fill_u32(reinterpret_cast<unsigned*>(c->st_S), size_t(hc) * wc * 2, 0u, c->stream);
    launch_seed_chain(patches, c->st_t, m, c->st_S, hc, wc, c->st_ph, c->stream);
  }
  launch_seed_stitch(patches, c->st_t, chain ? c->st_ph : nullptr, c->st_beg, c->st_idx, bw, bh, dst, c->H, c->W,
                     c->stream);
  PTY_HIP(hipStreamSynchronize(c->stream));   // the host lists above must outlive their copies
}

void run_algo(pty_ctx* c, int algo, int n_iter, const pty_iter_params& p) {
  if (algo == PTY_DM)
    run_dm(c, n_iter, p);
  else if (algo == PTY_LSQML)
    run_lsqml(c, n_iter, p);
  else
    run_epie(c, n_iter, p);
}

bool same_params(const pty_iter_params& a, const pty_iter_params& b) {
  return a.alpha == b.alpha && a.beta == b.beta && a.probe_update_start == b.probe_update_start &&
         a.lsqml_batch == b.lsqml_batch && a.gamma_obj == b.gamma_obj && a.gamma_probe == b.gamma_probe &&
         a.beta_obj == b.beta_obj && a.beta_probe == b.beta_probe && a.order_seed == b.order_seed &&
         a.chunk == b.chunk && a.flags == b.flags && a.position_start == b.position_start &&
         a.position_max_shift == b.position_max_shift;
}

// Iterations as replays of captured single iterations (DM and LSQML).  Each
// distinct key (algorithm, parameters, probe update on/off, buffer
// generation, probe buffer, truth on/off, state flags before the iteration)
// is captured once: the capture records the same launches an eager
// iteration makes, then the graph is launched.  The host-side state flags an
// eager iteration would leave are restored after each replay.  All buffers
// are prepared before capturing, so no allocation or synchronisation happens
// inside a capture.
void run_graphed(pty_ctx* c, int algo, int n_iter, const pty_iter_params& p) {
  run_algo(c, algo, 0, p);                 // work buffers
  ensure_err_slot(c, n_iter);              // history capacity for every replay
  const bool timing = c->timing;
  c->timing = false;
  try {
    for (int it = 0; it < n_iter; ++it) {
      const bool pon = probe_on(p, c->iter);
      pty_ctx::GraphEntry* hit = nullptr;
      for (auto& g : c->graphs)
        if (g.algo == algo && g.pon == pon && g.gen == c->gen && g.probe == c->probe &&
            g.dm_valid == c->dm_valid && g.den_valid == c->den_valid && g.have_truth == c->have_truth &&
            same_params(g.p, p)) {
          hit = &g;
          break;
        }
      if (!hit) {
        if (!c->graphs.empty() && c->graphs.front().gen != c->gen) c->drop_graphs();
        if (c->graphs.size() >= 8) c->drop_graphs();
        pty_ctx::GraphEntry g;
        g.algo = algo;
        g.pon = pon;
        g.gen = c->gen;
        g.probe = c->probe;
        g.dm_valid = c->dm_valid;
        g.den_valid = c->den_valid;
        g.have_truth = c->have_truth;
        g.p = p;
        const int iter0 = c->iter;
        PTY_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeRelaxed));
        try {
          run_algo(c, algo, 1, p);
        } catch (...) {
          hipGraph_t dead = nullptr;
          (void)hipStreamEndCapture(c->stream, &dead);
          if (dead) (void)hipGraphDestroy(dead);
          (void)hipGetLastError();
          c->iter = iter0;
          throw;
        }
        PTY_HIP(hipStreamEndCapture(c->stream, &g.graph));
        c->iter = iter0;                   // the capture ran nothing
        if (g.gen != c->gen) throw DeviceError("pty_iterate: buffers changed while capturing");
        PTY_HIP(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
        g.dm_valid_after = c->dm_valid;
        g.den_valid_after = c->den_valid;
        c->graphs.push_back(g);
        hit = &c->graphs.back();
      }
      PTY_HIP(hipGraphLaunch(hit->exec, c->stream));
      c->dm_valid = hit->dm_valid_after;
      c->den_valid = hit->den_valid_after;
      c->iter++;
    }
  } catch (...) {
    c->timing = timing;
    throw;
  }
  c->timing = timing;
}

// ---- chunk autotuning: a small JSON cache {"key": chunk, ...} ----
std::map<std::string, int> read_tune_cache(const char* path) {
  std::map<std::string, int> m;
  std::ifstream f(path);
  if (!f) return m;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while ((i = t.find('"', i)) != std::string::npos) {
    const size_t e = t.find('"', i + 1);
    if (e == std::string::npos) break;
    const std::string key = t.substr(i + 1, e - i - 1);
    size_t k = t.find(':', e);
    if (k == std::string::npos) break;
    const int v = std::atoi(t.c_str() + k + 1);
    if (v > 0) m[key] = v;
    i = t.find_first_of(",}", k);
    if (i == std::string::npos) break;
  }
  return m;
}

void write_tune_cache(const char* path, const std::map<std::string, int>& m) {
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) throw InvalidArg(std::string("pty_autotune: cannot write ") + tmp);
    f << "{\n";
    size_t n = 0;
    for (auto& kv : m) f << "  \"" << kv.first << "\": " << kv.second << (++n < m.size() ? ",\n" : "\n");
    f << "}\n";
  }
  if (std::rename(tmp.c_str(), path) != 0) throw InvalidArg(std::string("pty_autotune: cannot replace ") + path);
}

std::string tune_key(pty_ctx* c, int algo, const pty_iter_params& p) {
  hipDeviceProp_t prop;
  PTY_HIP(hipGetDeviceProperties(&prop, c->device));
  std::string arch = prop.gcnArchName;
  arch = arch.substr(0, arch.find(':'));
  const int batch = p.lsqml_batch > 0 ? p.lsqml_batch : 512;
  return arch + " n=" + std::to_string(c->N) + " k=" + std::to_string(c->K) + " j=" + std::to_string(c->J) +
         (algo == PTY_DM ? " dm" : " lsqml b=" + std::to_string(batch));
}

int tune_chunk(pty_ctx* c, int algo, pty_iter_params p) {
  const size_t hw = size_t(c->H) * c->W, kn = size_t(c->K) * c->N * c->N;
  const int batch = p.lsqml_batch > 0 ? p.lsqml_batch : 512;
  const int G = std::max(1, (c->J + batch - 1) / batch);
  const int slots = algo == PTY_DM ? c->J : (c->J + G - 1) / G;
  std::vector<int> cands;
  for (int v : {8, 16, 24, 32, 48, 64, 96, 128, 192, 256})
    if (v <= std::max(8, slots) && size_t(v) * kn * sizeof(float2) <= (size_t(1) << 30)) cands.push_back(v);
  float2* o_save = c->alloc<float2>(hw);
  float2* p_save = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int iter0 = c->iter;
  const bool timing = c->timing;
  int best = 0;
  try {
    p_save = c->alloc<float2>(kn);
    PTY_HIP(hipMemcpyAsync(o_save, c->obj, hw * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
    PTY_HIP(hipMemcpyAsync(p_save, c->probe, kn * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
    PTY_HIP(hipEventCreate(&e0));
    PTY_HIP(hipEventCreate(&e1));
    c->timing = false;
    p.flags = 0;
    p.position_start = -1;   // tuning iterations never move positions
    float best_ms = 0.f;
    for (int v : cands) {
      p.chunk = v;
      run_algo(c, algo, 1, p);             // warm: buffers for this chunk size
      PTY_HIP(hipEventRecord(e0, c->stream));
      run_algo(c, algo, 1, p);
      PTY_HIP(hipEventRecord(e1, c->stream));
      PTY_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PTY_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (!best || ms < best_ms) {
        best = v;
        best_ms = ms;
      }
    }
  } catch (...) {
    c->timing = timing;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->dfree(o_save);
    c->dfree(p_save);
    throw;
  }
  // then the probe sums' slice size with that chunk
  int best_slice = 0;
  try {
    p.chunk = best;
    float best_ms = 0.f;
    for (int v : {8, 16, 32}) {
      c->tuned_slice = v;
      ensure_probe_parts(c, c->J);
      run_algo(c, algo, 1, p);
      PTY_HIP(hipEventRecord(e0, c->stream));
      run_algo(c, algo, 1, p);
      PTY_HIP(hipEventRecord(e1, c->stream));
      PTY_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      PTY_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (!best_slice || ms < best_ms) {
        best_slice = v;
        best_ms = ms;
      }
    }
  } catch (...) {
    c->tuned_slice = 0;
    c->timing = timing;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    c->dfree(o_save);
    c->dfree(p_save);
    throw;
  }
  c->tuned_slice = best_slice;
  c->timing = timing;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  // restore the state the tuning iterations changed
  PTY_HIP(hipMemcpyAsync(c->obj, o_save, hw * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
  PTY_HIP(hipMemcpyAsync(c->probe, p_save, kn * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
  c->iter = iter0;
  launch_set_i32(c->iter_dev, iter0, c->stream);
  PTY_HIP(hipStreamSynchronize(c->stream));
  c->dfree(o_save);
  c->dfree(p_save);
  c->dm_valid = false;
  c->den_valid = false;
  return best;
}

}  // namespace

// ===========================================================================
// Entry points
// ===========================================================================
extern "C" {

pty_status pty_default_params(pty_iter_params* p) {
  return guarded(nullptr, [&] {
    require(p != nullptr, "pty_default_params: null params");
    std::memset(p, 0, sizeof(*p));
    p->alpha = 1.f;
    p->beta = 1.f;
    p->probe_update_start = 0;
    p->lsqml_batch = 512;
    p->gamma_obj = -1.f;
    p->gamma_probe = -1.f;
    p->beta_obj = 1.f;
    p->beta_probe = 1.f;
    p->order_seed = 0;
    p->chunk = 0;
    p->flags = 0;
    p->position_start = -1;
    p->position_max_shift = 0.5f;
  });
}

pty_status pty_create(const pty_plan_desc* plan, pty_ctx** out) {
  return guarded(nullptr, [&] {
    require(plan != nullptr && out != nullptr, "pty_create: null argument");
    require(supported_n(plan->n), "pty_create: n must be 32, 64, 128, 256 or 512");
    require(plan->modes >= 1 && plan->modes <= 4, "pty_create: modes must be in 1..4");
    require(plan->n < 512 || plan->modes <= 2, "pty_create: 512 x 512 windows take at most 2 modes");
    require(plan->n_pos >= 1, "pty_create: n_pos must be >= 1");
    require(plan->obj_h >= plan->n + 1 && plan->obj_w >= plan->n + 1, "pty_create: object must be at least (n+1) x (n+1)");
    require(plan->flags == 0, "pty_create: flags must be 0");
    require(plan->device >= 0, "pty_create: negative device");
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= plan->device) {
      (void)hipGetLastError();
      throw DeviceError("pty_create: no HIP device " + std::to_string(plan->device) +
                        (e != hipSuccess ? std::string(" (") + hipGetErrorString(e) + ")" : std::string()));
    }
    std::unique_ptr<pty_ctx> c(new pty_ctx());
    c->N = plan->n;
    c->K = plan->modes;
    c->J = plan->n_pos;
    c->H = plan->obj_h;
    c->W = plan->obj_w;
    c->device = plan->device;
    if (const char* lim = std::getenv("PTY_MEM_LIMIT")) c->mem_limit = std::strtoull(lim, nullptr, 10);
    c->set_device();
    (void)noalloc_scratch(c->device);   // once per device, with it current
    if (plan->stream) {
      c->stream = static_cast<hipStream_t>(plan->stream);
    } else {
      PTY_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    const size_t nn = size_t(c->N) * c->N;
    c->obj = c->alloc<float2>(size_t(c->H) * c->W);
    c->probe = c->alloc<float2>(size_t(c->K) * nn);
    c->probe_alt = c->alloc<float2>(size_t(c->K) * nn);
    c->amp = c->alloc<float>(size_t(c->J) * nn);
    c->pos = c->alloc<PosInfo>(size_t(c->J));
    c->tw = c->alloc<float2>(size_t(c->N));
    std::vector<float2> tw(c->N);
    for (int i = 0; i < c->N; ++i) {
      const double ang = -2.0 * M_PI * (double)i / (double)c->N;
      tw[i] = make_float2((float)std::cos(ang), (float)std::sin(ang));
    }
    PTY_HIP(hipMemcpy(c->tw, tw.data(), sizeof(float2) * c->N, hipMemcpyHostToDevice));
    *out = c.release();
  });
}

pty_status pty_load_patterns(pty_ctx* c, const float* counts, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_load_patterns: null context");
    require(counts != nullptr, "pty_load_patterns: null counts");
    c->set_device();
    const size_t n = size_t(c->J) * c->N * c->N;
    const float* src = counts;
    float* tmp = nullptr;
    if (!on_device) {
      tmp = c->alloc<float>(n);
      PTY_HIP(hipMemcpyAsync(tmp, counts, n * sizeof(float), hipMemcpyHostToDevice, c->stream));
      src = tmp;
    }
    try {
      launch_amplitude(src, c->amp, nullptr, c->N, c->J, c->stream);
      if (c->have_mask) launch_apply_mask(c->amp, c->mask, c->N, c->J, c->stream);
      PTY_HIP(hipStreamSynchronize(c->stream));
    } catch (...) {
      c->dfree(tmp);
      throw;
    }
    c->dfree(tmp);
    c->have_patterns = true;
  });
}

pty_status pty_guess_probe(pty_ctx* c, double diameter) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_guess_probe: null context");
    require(std::isfinite(diameter) && diameter > 0.0 && diameter <= 2.0 * c->N,
            "pty_guess_probe: diameter must be in (0, 2 N]");
    if (!c->have_patterns) throw StateError("pty_guess_probe: patterns not loaded");
    c->set_device();
    // mean total counts of the loaded patterns
    std::vector<double> tot(c->J);
    double* d_tot = c->alloc<double>(c->J);
    try {
      launch_amp_totals(c->amp, d_tot, c->N, c->J, c->stream);
      copy_out(c, tot.data(), d_tot, sizeof(double) * c->J, 0);
    } catch (...) {
      c->dfree(d_tot);
      throw;
    }
    c->dfree(d_tot);
    double photons = 0.0;
    for (double t : tot) photons += t;
    photons /= c->J;
    // disk and shape functions, modified Gram-Schmidt in FP64
    const int n = c->N, K = c->K;
    const size_t nn = size_t(n) * n;
    const double cc = 0.5 * (n - 1), r2 = 0.25 * diameter * diameter;
    std::vector<std::vector<double>> m(K, std::vector<double>(nn, 0.0));
    for (int y = 0; y < n; ++y)
      for (int x = 0; x < n; ++x) {
        const double u = y - cc, w = x - cc;
        if (u * u + w * w > r2) continue;
        const double f[4] = {1.0, w, u, u * w};
        for (int k = 0; k < K; ++k) m[k][size_t(y) * n + x] = f[k];
      }
    for (int k = 0; k < K; ++k) {
      for (int l = 0; l < k; ++l) {
        double num = 0.0, den = 0.0;
        for (size_t q = 0; q < nn; ++q) {
          num += m[l][q] * m[k][q];
          den += m[l][q] * m[l][q];
        }
        const double a = num / den;
        for (size_t q = 0; q < nn; ++q) m[k][q] -= a * m[l][q];
      }
      double pw = 0.0;
      for (size_t q = 0; q < nn; ++q) pw += m[k][q] * m[k][q];
      require(pw > 1e-12 * nn, "pty_guess_probe: diameter too small for the number of modes");
      const double s = std::sqrt(photons / K / pw);
      for (size_t q = 0; q < nn; ++q) m[k][q] *= s;
    }
    std::vector<float2> out(size_t(K) * nn);
    for (int k = 0; k < K; ++k)
      for (size_t q = 0; q < nn; ++q) out[size_t(k) * nn + q] = make_float2((float)m[k][q], 0.f);
    copy_in(c, c->probe, out.data(), out.size() * sizeof(float2), 0);
    c->have_probe = true;
    c->dm_valid = false;
    c->den_valid = false;
  });
}

pty_status pty_set_mask(pty_ctx* c, const uint8_t* mask) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_set_mask: null context");
    c->set_device();
    const int n = c->N, h = n / 2;
    if (mask) {
      std::vector<unsigned char> nat(size_t(n) * n);
      for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x)
          nat[size_t(y) * n + x] = mask[size_t((y + h) % n) * n + (x + h) % n] ? 1 : 0;
      c->ensure_once(c->mask, nat.size());
      copy_in(c, c->mask, nat.data(), nat.size(), 0);
    }
    c->have_mask = mask != nullptr;
    c->drop_graphs();   // captured iterations carry the mask flag in their arguments
    if (c->have_patterns) launch_apply_mask(c->amp, c->have_mask ? c->mask : nullptr, c->N, c->J, c->stream);
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_load_positions(pty_ctx* c, const double* yx) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_load_positions: null context");
    require(yx != nullptr, "pty_load_positions: null positions");
    std::vector<PosInfo> hp(c->J);
    for (int j = 0; j < c->J; ++j) {
      const double y = yx[2 * j], x = yx[2 * j + 1];
      if (!(std::isfinite(y) && std::isfinite(x)) || y < 0 || x < 0)
        throw InvalidArg("pty_load_positions: position " + std::to_string(j) + " is negative or not finite");
      const double fy = std::floor(y), fx = std::floor(x);
      const int ey = (int)fy + c->N + (y != fy ? 1 : 0), ex = (int)fx + c->N + (x != fx ? 1 : 0);
      if (ey > c->H || ex > c->W)
        throw InvalidArg("pty_load_positions: patch " + std::to_string(j) + " extends past the object");
      hp[j] = PosInfo{(int)fy, (int)fx, (float)(y - fy), (float)(x - fx)};
    }
    c->set_device();
    PTY_HIP(hipMemcpy(c->pos, hp.data(), sizeof(PosInfo) * c->J, hipMemcpyHostToDevice));
    c->hpos = std::move(hp);
    free_group(c, c->all);
    for (auto& g : c->groups) free_group(c, g);
    c->groups.clear();
    c->groups_batch = -1;
    c->have_positions = true;
    c->dm_valid = false;
    c->den_valid = false;
  });
}

pty_status pty_set_object(pty_ctx* c, const void* src, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr && src != nullptr, "pty_set_object: null argument");
    c->set_device();
    copy_in(c, c->obj, src, size_t(c->H) * c->W * sizeof(float2), on_device);
    c->have_object = true;
    c->dm_valid = false;
  });
}

pty_status pty_set_probe(pty_ctx* c, const void* src, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr && src != nullptr, "pty_set_probe: null argument");
    c->set_device();
    copy_in(c, c->probe, src, size_t(c->K) * c->N * c->N * sizeof(float2), on_device);
    c->have_probe = true;
    c->dm_valid = false;
    c->den_valid = false;
  });
}

pty_status pty_iterate(pty_ctx* c, pty_algo algo, int32_t n_iter, const pty_iter_params* prm) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_iterate: null context");
    require(algo == PTY_EPIE || algo == PTY_DM || algo == PTY_LSQML, "pty_iterate: unknown algorithm");
    require(n_iter >= 0, "pty_iterate: negative iteration count");
    pty_iter_params p;
    pty_default_params(&p);
    if (prm) p = *prm;
    require((p.flags & ~(PTY_ITER_GRAPH | PTY_ITER_ORTHO_MODES | PTY_ITER_POISSON)) == 0,
            "pty_iterate: unknown flags");
    if ((p.flags & PTY_ITER_POISSON) && algo != PTY_LSQML)
      throw Unsupported("pty_iterate: the Poisson exit-wave update runs in LSQML only");
    require(p.chunk >= 0, "pty_iterate: negative chunk");
    require(p.lsqml_batch >= 0, "pty_iterate: negative lsqml_batch");
    if (p.position_start >= 0) {
      require(std::isfinite(p.position_max_shift) && p.position_max_shift > 0.f,
              "pty_iterate: position_max_shift must be positive");
      if (algo != PTY_LSQML) throw Unsupported("pty_iterate: position refinement runs in LSQML only");
      if (p.flags & PTY_ITER_GRAPH)
        throw Unsupported("pty_iterate: position refinement rebuilds the patch lists on the host; no graph replay");
    }
    require_loaded(c);
    if (n_iter == 0 && algo == PTY_EPIE) return;
    c->set_device();
    if ((p.flags & PTY_ITER_GRAPH) && algo != PTY_EPIE && n_iter > 0) {
      run_graphed(c, algo, n_iter, p);
      return;
    }
    run_algo(c, algo, n_iter, p);
    if (n_iter == 0) PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_get_object(pty_ctx* c, void* out, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_get_object: null argument");
    c->set_device();
    copy_out(c, out, c->obj, size_t(c->H) * c->W * sizeof(float2), on_device);
  });
}

pty_status pty_get_probe(pty_ctx* c, void* out, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_get_probe: null argument");
    c->set_device();
    copy_out(c, out, c->probe, size_t(c->K) * c->N * c->N * sizeof(float2), on_device);
  });
}

pty_status pty_get_errors(pty_ctx* c, double* out, int32_t cap, int32_t* n_written) {
  bool finite = true;
  pty_status st = guarded(c, [&] {
    require(c != nullptr && n_written != nullptr, "pty_get_errors: null argument");
    require(cap >= 0 && (cap == 0 || out != nullptr), "pty_get_errors: bad buffer");
    c->set_device();
    const int n = std::min<int>(cap, c->iter);
    if (n > 0)
      copy_out(c, out, c->err_dev, sizeof(double) * n, 0);
    else
      PTY_HIP(hipStreamSynchronize(c->stream));
    *n_written = n;
    for (int i = 0; i < n; ++i) finite = finite && std::isfinite(out[i]);
  });
  if (st == PTY_OK && !finite) return fail(c, PTY_E_NUMERIC, "pty_get_errors: NaN or Inf in the iteration error");
  return st;
}

pty_status pty_get_lsqml_steps(pty_ctx* c, float* out) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_get_lsqml_steps: null argument");
    if (!c->alpha_by_j) throw StateError("pty_get_lsqml_steps: LSQML has not run");
    c->set_device();
    copy_out(c, out, c->alpha_by_j, sizeof(float2) * c->J, 0);
  });
}

pty_status pty_get_exit_waves(pty_ctx* c, void* out, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_get_exit_waves: null argument");
    if (!c->dm_valid || !c->psi) throw StateError("pty_get_exit_waves: no DM exit waves");
    c->set_device();
    copy_out(c, out, c->psi, size_t(c->J) * c->K * c->N * c->N * sizeof(float2), on_device);
  });
}

namespace {
struct StateHeader {
  char magic[8];
  int32_t n, modes, n_pos, obj_h, obj_w, iterations, has_psi, has_nrmse;
  int32_t pad[6];
};
static_assert(sizeof(StateHeader) == PTY_STATE_HEADER_BYTES, "state header layout");
constexpr char kStateMagic[8] = {'P', 'T', 'Y', 'S', 'T', 'A', 'T', '1'};

// DM state: the exit waves and the per-pattern planes sum_k conj(P_k) psi_k
// that the last Fourier pass left for the next object update.
size_t psi_elems(const pty_ctx* c) { return size_t(c->J) * c->K * c->N * c->N; }
size_t contrib_elems(const pty_ctx* c) { return size_t(c->J) * c->N * c->N; }

size_t state_bytes(const pty_ctx* c, const StateHeader& h) {
  size_t b = sizeof(StateHeader) + sizeof(double) * size_t(h.iterations) * (h.has_nrmse ? 2 : 1);
  if (h.has_psi) b += (psi_elems(c) + contrib_elems(c)) * sizeof(float2);
  return b;
}
}  // namespace

pty_status pty_get_state(pty_ctx* c, void* out, size_t cap, size_t* n) {
  return guarded(c, [&] {
    require(c != nullptr && n != nullptr, "pty_get_state: null argument");
    StateHeader h{};
    std::memcpy(h.magic, kStateMagic, sizeof(h.magic));
    h.n = c->N;
    h.modes = c->K;
    h.n_pos = c->J;
    h.obj_h = c->H;
    h.obj_w = c->W;
    h.iterations = c->iter;
    h.has_psi = (c->dm_valid && c->psi && c->contrib && c->contrib_slots >= contrib_elems(c)) ? 1 : 0;
    h.has_nrmse = (c->have_truth && c->iter > 0) ? 1 : 0;
    const size_t bytes = state_bytes(c, h);
    *n = bytes;
    if (out == nullptr) return;
    require(cap >= bytes, "pty_get_state: buffer smaller than the state");
    c->set_device();
    char* p = static_cast<char*>(out);
    std::memcpy(p, &h, sizeof(h));
    p += sizeof(h);
    if (h.iterations > 0) {
      copy_out(c, p, c->err_dev, sizeof(double) * h.iterations, 0);
      p += sizeof(double) * h.iterations;
    }
    if (h.has_nrmse) {
      copy_out(c, p, c->nrmse_dev, sizeof(double) * h.iterations, 0);
      p += sizeof(double) * h.iterations;
    }
    if (h.has_psi) {
      copy_out(c, p, c->psi, psi_elems(c) * sizeof(float2), 0);
      p += psi_elems(c) * sizeof(float2);
      copy_out(c, p, c->contrib, contrib_elems(c) * sizeof(float2), 0);
    }
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_set_state(pty_ctx* c, const void* in, size_t n) {
  return guarded(c, [&] {
    require(c != nullptr && in != nullptr, "pty_set_state: null argument");
    require(n >= sizeof(StateHeader), "pty_set_state: buffer shorter than the header");
    StateHeader h;
    std::memcpy(&h, in, sizeof(h));
    require(std::memcmp(h.magic, kStateMagic, sizeof(h.magic)) == 0, "pty_set_state: not a state buffer");
    require(h.n == c->N && h.modes == c->K && h.n_pos == c->J && h.obj_h == c->H && h.obj_w == c->W,
            "pty_set_state: shape differs from the context's");
    require(h.iterations >= 0 && (h.has_psi == 0 || h.has_psi == 1) && (h.has_nrmse == 0 || h.has_nrmse == 1),
            "pty_set_state: bad header");
    require(n == state_bytes(c, h), "pty_set_state: size does not match the header");
    c->set_device();
    const char* p = static_cast<const char*>(in) + sizeof(h);
    // allocations first, so that a failure leaves the context as it was
    ensure_err_slot(c, std::max(1, h.iterations - c->iter));
    if (h.has_psi) {
      c->ensure_once(c->psi, psi_elems(c));
      c->ensure(c->contrib, c->contrib_slots, contrib_elems(c));
    }
    if (h.iterations > 0) copy_in(c, c->err_dev, p, sizeof(double) * h.iterations, 0);
    p += sizeof(double) * h.iterations;
    if (h.has_nrmse) {
      if (c->have_truth) copy_in(c, c->nrmse_dev, p, sizeof(double) * h.iterations, 0);
      p += sizeof(double) * h.iterations;
    }
    if (h.has_psi) {
      copy_in(c, c->psi, p, psi_elems(c) * sizeof(float2), 0);
      p += psi_elems(c) * sizeof(float2);
      copy_in(c, c->contrib, p, contrib_elems(c) * sizeof(float2), 0);
    }
    c->iter = h.iterations;
    launch_set_i32(c->iter_dev, c->iter, c->stream);
    c->dm_valid = h.has_psi == 1;
    c->den_valid = false;
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_get_positions(pty_ctx* c, double* yx) {
  return guarded(c, [&] {
    require(c != nullptr && yx != nullptr, "pty_get_positions: null argument");
    if (!c->have_positions) throw StateError("pty_get_positions: positions not loaded");
    c->set_device();
    std::vector<PosInfo> hp(c->J);
    copy_out(c, hp.data(), c->pos, sizeof(PosInfo) * c->J, 0);
    for (int j = 0; j < c->J; ++j) {
      yx[2 * j] = double(hp[j].iy) + double(hp[j].fy);
      yx[2 * j + 1] = double(hp[j].ix) + double(hp[j].fx);
    }
  });
}

pty_status pty_mem_bytes(const pty_ctx* c, size_t* out) {
  return guarded(const_cast<pty_ctx*>(c), [&] {
    require(c != nullptr && out != nullptr, "pty_mem_bytes: null argument");
    *out = c->mem;
  });
}

pty_status pty_set_timing(pty_ctx* c, int enable) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_set_timing: null context");
    c->set_device();
    c->drain_timing();
    for (int i = 0; i < pty_ctx::kFamilies; ++i) {
      c->fam_ms[i] = 0.0;
      c->fam_n[i] = 0;
    }
    c->timing = enable != 0;
  });
}

pty_status pty_get_timing(pty_ctx* c, double* ms, int64_t* launches, int32_t cap) {
  return guarded(c, [&] {
    require(c != nullptr && ms != nullptr && launches != nullptr, "pty_get_timing: null argument");
    require(cap >= 0, "pty_get_timing: negative cap");
    c->set_device();
    c->drain_timing();
    for (int i = 0; i < std::min<int>(cap, pty_ctx::kFamilies); ++i) {
      ms[i] = c->fam_ms[i];
      launches[i] = c->fam_n[i];
    }
  });
}

pty_status pty_sync(pty_ctx* c) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_sync: null context");
    c->set_device();
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

void pty_destroy(pty_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  delete c;
}

const char* pty_last_error(const pty_ctx* c) {
  if (c) return c->err.c_str();
  return g_tls_error.c_str();
}

pty_status pty_nll_forward(pty_ctx* c, const void* obj, const void* probe, const float* pos, double* loss) {
  return guarded(c, [&] {
    require(c != nullptr && obj != nullptr && probe != nullptr && loss != nullptr, "pty_nll_forward: null argument");
    c->set_device();
    *loss = run_nll(c, static_cast<const float2*>(obj), static_cast<const float2*>(probe), pos, false, 1.f, nullptr,
                    nullptr, nullptr);
  });
}

pty_status pty_nll_backward(pty_ctx* c, const void* obj, const void* probe, const float* pos, float grad_out,
                            void* g_obj, void* g_probe, float* g_pos, double* loss) {
  return guarded(c, [&] {
    require(c != nullptr && obj != nullptr && probe != nullptr, "pty_nll_backward: null argument");
    require(std::isfinite(grad_out), "pty_nll_backward: grad_out must be finite");
    c->set_device();
    const double l = run_nll(c, static_cast<const float2*>(obj), static_cast<const float2*>(probe), pos, true,
                             grad_out, static_cast<float2*>(g_obj), static_cast<float2*>(g_probe), g_pos);
    if (loss) *loss = l;
  });
}

pty_status pty_nll_forward_noalloc(pty_ctx* c, const void* obj, const void* probe, const float* pos, int32_t count,
                                   double* loss) {
  return guarded(c, [&] {
    require(c != nullptr && obj != nullptr && probe != nullptr && loss != nullptr,
            "pty_nll_forward_noalloc: null argument");
    require(count >= 1 && count <= c->J, "pty_nll_forward_noalloc: count must be in 1..J");
    if (!c->have_patterns) throw StateError("patterns not loaded");
    if (!pos && !c->have_positions) throw StateError("positions not loaded (and none supplied)");
    c->set_device();
    char* base = static_cast<char*>(noalloc_scratch(c->device));
    constexpr size_t cap = PTY_NOALLOC_SCRATCH_BYTES;
    const size_t per = size_t(c->K) * c->N * c->N * sizeof(float2);
    const int cb = col_blocks(c->N, c->K);
    size_t used = 0;
    auto take = [&](size_t bytes) {
      char* p = base + used;
      used += (bytes + 255) / 256 * 256;
      return p;
    };
    int* slots = reinterpret_cast<int*>(take(sizeof(int) * size_t(count)));
    PosInfo* pinfo = pos ? reinterpret_cast<PosInfo*>(take(sizeof(PosInfo) * size_t(count))) : nullptr;
    double* errp = reinterpret_cast<double*>(take(sizeof(double) * 2 * size_t(count) * cb));
    if (used + per > cap)
      throw InvalidArg("pty_nll_forward_noalloc: " + std::to_string(count) + " positions need " +
                       std::to_string(used + per) + " bytes of work space; the no-allocation scratch holds " +
                       std::to_string(cap));
    float2* zs = reinterpret_cast<float2*>(base + used);
    int chunk = (int)std::min<size_t>((cap - used) / per, size_t(count));
    const int wave = std::max(1, 256 / row_blocks(c->N));
    if (chunk >= wave) chunk = chunk / wave * wave;
    launch_iota_i32(slots, count, c->stream);
    if (pos) launch_pos_from_yx(pos, count, c->H - c->N, c->W - c->N, pinfo, c->stream);
    Group g;
    g.d_jl = slots;
    FourierArgs a = fourier_args(c, g);
    a.obj = static_cast<const float2*>(obj);
    a.probe = static_cast<const float2*>(probe);
    a.pos = pos ? pinfo : c->pos;
    a.zs = zs;
    a.errp = errp;
    a.psi = nullptr;
    a.chi = nullptr;
    a.contrib = nullptr;
    a.posgrad = nullptr;
    for (int off = 0; off < count; off += chunk) {
      a.jl_off = off;
      a.slot_off = off;
      a.nc = std::min(chunk, count - off);
      launch_rows_fwd(a, RowIn::Plain);
      launch_cols(a, ColOp::NllLoss);
    }
    launch_err_reduce(errp, count * cb, loss, c->stream);
  });
}

pty_status pty_simulate(pty_ctx* c, double photons, float* out, int on_device) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_simulate: null argument");
    require(std::isfinite(photons) && photons >= 0, "pty_simulate: photons must be finite and >= 0");
    if (!c->have_positions) throw StateError("positions not loaded");
    if (!c->have_object) throw StateError("object not set");
    if (!c->have_probe) throw StateError("probe not set");
    c->set_device();
    pty_iter_params p;
    pty_default_params(&p);
    const int chunk = chunk_patterns(c, p);
    ensure_all_group(c);
    ensure_common(c, std::min(chunk, c->J), 1);
    const size_t n = size_t(c->J) * c->N * c->N;
    float* dst = on_device ? out : c->alloc<float>(n);
    try {
      FourierArgs a = fourier_args(c, c->all);
      a.intensity_out = dst;
      for (int off = 0; off < c->J; off += chunk) {
        a.jl_off = off;
        a.slot_off = off;
        a.nc = std::min(chunk, c->J - off);
        launch_rows_fwd(a, RowIn::Plain);
        launch_cols(a, ColOp::Intensity);
      }
      if (photons > 0) {
        double* tot = c->alloc<double>(c->J);
        std::vector<double> ht(c->J);
        try {
          launch_pattern_totals(dst, tot, c->N, c->J, c->stream);
          PTY_HIP(hipMemcpyAsync(ht.data(), tot, sizeof(double) * c->J, hipMemcpyDeviceToHost, c->stream));
          PTY_HIP(hipStreamSynchronize(c->stream));
        } catch (...) {
          c->dfree(tot);
          throw;
        }
        c->dfree(tot);
        double mean = 0;
        for (double v : ht) mean += v;
        mean /= c->J;
        if (!(mean > 0)) throw InvalidArg("pty_simulate: zero total intensity");
        const double s = photons / mean;
        launch_scale_f32(dst, n, (float)s, c->stream);
        launch_scale_c64(c->probe, size_t(c->K) * c->N * c->N, (float)std::sqrt(s), c->stream);
        c->dm_valid = false;
        c->den_valid = false;
      }
      if (!on_device) {
        PTY_HIP(hipMemcpyAsync(out, dst, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
      }
      PTY_HIP(hipStreamSynchronize(c->stream));
    } catch (...) {
      if (!on_device) c->dfree(dst);
      throw;
    }
    if (!on_device) c->dfree(dst);
  });
}

pty_status pty_model_error(pty_ctx* c, double* out) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_model_error: null argument");
    if (!c->have_patterns) throw StateError("patterns not loaded");
    if (!c->have_positions) throw StateError("positions not loaded");
    if (!c->have_object) throw StateError("object not set");
    if (!c->have_probe) throw StateError("probe not set");
    c->set_device();
    *out = model_error(c);
  });
}

pty_status pty_set_truth(pty_ctx* c, const void* truth, int on_device, float roi_frac) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_set_truth: null context");
    c->set_device();
    if (!truth) {
      c->have_truth = false;
      return;
    }
    require(roi_frac >= 0.f && roi_frac <= 1.f, "pty_set_truth: roi_frac must be in [0, 1]");
    if (!c->have_positions) throw StateError("positions not loaded");
    if (!c->have_probe) throw StateError("probe not set");
    const size_t hw = size_t(c->H) * c->W;
    ensure_all_group(c);
    ensure_common(c, 1, 1);
    c->ensure_once(c->truth, hw);
    c->ensure_once(c->roi, hw);
    c->ensure_once(c->nrmse_part, nrmse_part_doubles());
    copy_in(c, c->truth, truth, hw * sizeof(float2), on_device);
    // the density pass writes only tiles that some patch overlaps
    launch_fill_u32(reinterpret_cast<unsigned*>(c->den), hw, 0u, c->stream);
    density(c, c->all);
    c->den_valid = true;
    launch_roi_mask(c->den, c->scal, roi_frac, hw, c->roi, c->stream);
    PTY_HIP(hipStreamSynchronize(c->stream));
    c->have_truth = true;
  });
}

pty_status pty_nrmse(pty_ctx* c, double* out) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_nrmse: null argument");
    if (!c->have_truth) throw StateError("no truth set");
    if (!c->have_object) throw StateError("object not set");
    c->set_device();
    c->ensure_once(c->eval_dev, 8);
    launch_nrmse(c->obj, c->truth, c->roi, size_t(c->H) * c->W, c->nrmse_part, c->eval_dev, c->stream);
    PTY_HIP(hipMemcpyAsync(out, c->eval_dev, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_get_nrmse(pty_ctx* c, double* out, int32_t cap, int32_t* n_written) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr && n_written != nullptr && cap >= 0, "pty_get_nrmse: bad argument");
    c->set_device();
    const int n = std::min(cap, c->iter);
    if (n > 0) copy_out(c, out, c->nrmse_dev, sizeof(double) * n, 0);
    else PTY_HIP(hipStreamSynchronize(c->stream));
    *n_written = n;
  });
}

pty_status pty_stitch(pty_ctx* c, const float* patches, void* out) {
  return guarded(c, [&] {
    require(c != nullptr && patches != nullptr, "pty_stitch: null argument");
    if (!c->have_positions) throw StateError("positions not loaded");
    c->set_device();
    if (out) {
      stitch(c, patches, static_cast<float2*>(out));
    } else {
      stitch(c, patches, c->obj);
      c->have_object = true;
      c->dm_valid = false;
    }
  });
}

pty_status pty_seed_object(pty_ctx* c, pty_cnn* net, int32_t batch, int32_t stride, int32_t fallback,
                           int32_t* used_fallback, double* e_seed, double* e_flat) {
  return guarded(c, [&] {
    require(c != nullptr && net != nullptr, "pty_seed_object: null argument");
    require(batch >= 1 && batch <= cnn_max_batch(net), "pty_seed_object: batch must be in 1..max_batch");
    require(stride >= 1, "pty_seed_object: stride must be >= 1");
    if (c->N != 128) throw Unsupported("the learned seed needs 128 x 128 windows");
    if (cnn_device(net) != c->device) throw InvalidArg("pty_seed_object: network on another device");
    if (!c->have_patterns) throw StateError("patterns not loaded");
    if (!c->have_positions) throw StateError("positions not loaded");
    if (!c->have_probe) throw StateError("probe not set");
    c->set_device();
    std::vector<int> sel;
    for (int j = 0; j < c->J; j += stride) sel.push_back(j);
    const int m = (int)sel.size();
    const size_t nn = size_t(c->N) * c->N;
    const size_t per = size_t(64) * 64 * 2;
    c->ensure(c->seed_patches, c->seed_patches_n, size_t(m) * per + 4 * nn + size_t(m));
    float2* planes = reinterpret_cast<float2*>(c->seed_patches + size_t(m) * per);
    int* d_sel = reinterpret_cast<int*>(planes + 2 * nn);
    PTY_HIP(hipMemcpyAsync(d_sel, sel.data(), sizeof(int) * m, hipMemcpyHostToDevice, c->stream));
    launch_seed_planes(c->probe, planes, planes + nn, c->stream);
    float* x = cnn_input_buffer(net);
    for (int i0 = 0; i0 < m; i0 += batch) {
      const int nb = std::min(batch, m - i0);
      launch_seed_input_amp(c->amp, d_sel + i0, nb, planes, planes + nn, x, c->stream);
      const float* y = cnn_forward_batch(net, x, nb, c->stream);
      PTY_HIP(hipMemcpyAsync(c->seed_patches + size_t(i0) * per, y, sizeof(float) * per * nb,
                             hipMemcpyDeviceToDevice, c->stream));
    }
    const size_t hw = size_t(c->H) * c->W;
    if (!fallback) {
      stitch(c, c->seed_patches, c->obj, sel, false);
      c->have_object = true;
      c->dm_valid = false;
      if (used_fallback) *used_fallback = 0;
      return;
    }
    c->ensure_once(c->seed_obj, hw);
    stitch(c, c->seed_patches, c->seed_obj, sel, false);
    PTY_HIP(hipMemcpyAsync(c->obj, c->seed_obj, hw * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
    // the two model errors over the seeded windows
    Group sub;
    sub.jl = sel;
    sub.d_jl = d_sel;
    const double es = model_error(c, stride > 1 ? &sub : nullptr);
    launch_fill_c64(c->obj, hw, make_float2(1.f, 0.f), c->stream);
    const double ef = model_error(c, stride > 1 ? &sub : nullptr);
    const bool use_seed = std::isfinite(es) && es <= ef;
    if (use_seed)
      PTY_HIP(hipMemcpyAsync(c->obj, c->seed_obj, hw * sizeof(float2), hipMemcpyDeviceToDevice, c->stream));
    PTY_HIP(hipStreamSynchronize(c->stream));
    c->have_object = true;
    c->dm_valid = false;
    if (used_fallback) *used_fallback = use_seed ? 0 : 1;
    if (e_seed) *e_seed = es;
    if (e_flat) *e_flat = ef;
  });
}

pty_status pty_training_targets(pty_ctx* c, float* out) {
  return guarded(c, [&] {
    require(c != nullptr && out != nullptr, "pty_training_targets: null argument");
    if (!c->have_positions) throw StateError("positions not loaded");
    if (!c->have_object) throw StateError("object not set");
    for (const PosInfo& p : c->hpos)
      require(p.fy == 0.f && p.fx == 0.f, "pty_training_targets: positions must be integers");
    c->set_device();
    launch_targets(c->obj, c->W, c->pos, c->J, c->N, out, c->stream);
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_poisson(pty_ctx* c, const float* lam, float* out, size_t n, uint64_t seed) {
  return guarded(c, [&] {
    require(c != nullptr && lam != nullptr && out != nullptr, "pty_poisson: null argument");
    c->set_device();
    launch_poisson(lam, out, n, seed, c->stream);
    PTY_HIP(hipStreamSynchronize(c->stream));
  });
}

pty_status pty_get_tuning(pty_ctx* c, int32_t* chunk, int32_t* probe_slice) {
  return guarded(c, [&] {
    require(c != nullptr && chunk != nullptr && probe_slice != nullptr, "pty_get_tuning: null argument");
    *chunk = c->tuned_chunk;
    *probe_slice = c->tuned_slice;
  });
}

pty_status pty_autotune(pty_ctx* c, pty_algo algo, const pty_iter_params* prm, const char* cache_path,
                        int32_t* chunk) {
  return guarded(c, [&] {
    require(c != nullptr, "pty_autotune: null context");
    if (algo != PTY_DM && algo != PTY_LSQML) throw Unsupported("pty_autotune: DM and LSQML only");
    pty_iter_params p;
    pty_default_params(&p);
    if (prm) p = *prm;
    require((p.flags & ~PTY_ITER_GRAPH) == 0, "pty_autotune: unknown flags");
    require_loaded(c);
    c->set_device();
    const std::string key = tune_key(c, algo, p);
    std::map<std::string, int> cache;
    if (cache_path) cache = read_tune_cache(cache_path);
    auto it = cache.find(key);
    auto its = cache.find(key + " slice");
    int best;
    if (it != cache.end() && its != cache.end()) {
      best = it->second;
      c->tuned_slice = std::min(its->second, 32);
    } else {
      best = tune_chunk(c, algo, p);   // also sets tuned_slice
      if (cache_path) {
        cache[key] = best;
        cache[key + " slice"] = c->tuned_slice;
        write_tune_cache(cache_path, cache);
      }
    }
    c->tuned_chunk = best;
    if (chunk) *chunk = best;
  });
}

}  // extern "C"

struct pty_batch {
  std::vector<pty_ctx*> ctxs;
  std::string err;
};

extern "C" {

pty_status pty_batch_create(pty_ctx* const* ctxs, int32_t n, pty_batch** out) {
  return guarded(nullptr, [&] {
    require(ctxs != nullptr && out != nullptr && n >= 1, "pty_batch_create: bad argument");
    std::unique_ptr<pty_batch> b(new pty_batch());
    for (int i = 0; i < n; ++i) {
      require(ctxs[i] != nullptr, "pty_batch_create: null context");
      b->ctxs.push_back(ctxs[i]);
    }
    *out = b.release();
  });
}

pty_status pty_batch_iterate(pty_batch* b, pty_algo algo, int32_t n_iter, const pty_iter_params* prm) {
  if (!b) return fail(nullptr, PTY_E_INVALID, "pty_batch_iterate: null batch");
  if (n_iter < 0) return fail(nullptr, PTY_E_INVALID, (b->err = "pty_batch_iterate: negative iteration count"));
  // buffers first (allocation synchronises), then the iterations back to back
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    const pty_status st = pty_iterate(b->ctxs[i], algo, 0, prm);
    if (st != PTY_OK) {
      b->err = "context " + std::to_string(i) + ": " + pty_last_error(b->ctxs[i]);
      return st;
    }
  }
  for (int t = 0; t < n_iter; ++t)
    for (size_t i = 0; i < b->ctxs.size(); ++i) {
      const pty_status st = pty_iterate(b->ctxs[i], algo, 1, prm);
      if (st != PTY_OK) {
        b->err = "context " + std::to_string(i) + ": " + pty_last_error(b->ctxs[i]);
        return st;
      }
    }
  return PTY_OK;
}

pty_status pty_batch_autotune(pty_batch* b, pty_algo algo, const pty_iter_params* prm, const char* cache_path) {
  if (!b) return fail(nullptr, PTY_E_INVALID, "pty_batch_autotune: null batch");
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    const pty_status st = pty_autotune(b->ctxs[i], algo, prm, cache_path, nullptr);
    if (st != PTY_OK) {
      b->err = "context " + std::to_string(i) + ": " + pty_last_error(b->ctxs[i]);
      return st;
    }
  }
  return PTY_OK;
}

pty_status pty_batch_sync(pty_batch* b) {
  if (!b) return fail(nullptr, PTY_E_INVALID, "pty_batch_sync: null batch");
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    const pty_status st = pty_sync(b->ctxs[i]);
    if (st != PTY_OK) {
      b->err = "context " + std::to_string(i) + ": " + pty_last_error(b->ctxs[i]);
      return st;
    }
  }
  return PTY_OK;
}

void pty_batch_destroy(pty_batch* b) { delete b; }

const char* pty_batch_last_error(const pty_batch* b) { return b ? b->err.c_str() : g_tls_error.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Strip decomposition of DM and LSQML (the multi-GPU layout of Sec. 1 and
// Sec. 2.2's overlap between sub-regions, shown on one GPU)
// ---------------------------------------------------------------------------
// The positions are split by their row into strips of equal counts; each strip
// is a context of its own holding the object rows its patches touch.  Every
// global object row has one owning strip (the owned ranges partition the
// object).  Wherever the method sums over positions, each strip sums its own;
// the object-plane sums are completed by halo messages (strip -> owner, added
// in strip order, then owner -> strip, copied), the probe sums by an
// all-reduce of one packed message per strip, the maxima behind the
// regularisers and the error by the same exchange.  On several GPUs each
// message would be one RCCL send/receive or all-reduce; here the strips run
// one after another on one stream.
struct pty_domains {
  int S = 0, N = 0, K = 0, J = 0, H = 0, W = 0, device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  std::vector<pty_ctx*> sub;
  std::vector<int> lo, hi, own_lo, own_hi;   // local and owned global rows [lo, hi)
  std::vector<std::vector<int>> jmap;        // strip -> global pattern indices, ascending
  std::vector<int*> d_jmap;
  struct Seg {
    int src, dst, a, b;   // global rows [a, b) of src's local rows owned by dst
  };
  std::vector<Seg> segs;
  std::vector<void*> allocs;
  float* msg = nullptr;                      // halo message staging
  std::vector<float*> pmsg;                  // one probe message per strip
  float* ptot = nullptr;                     // summed probe message
  size_t pwords = 0;
  double* errp_all = nullptr;                // J x column blocks x 2, by global pattern
  double* err_dev = nullptr;
  int err_cap = 0;
  int* iter_dev = nullptr;
  unsigned* dmax = nullptr;
  std::vector<float2*> num2;                 // per strip: LSQML update numerator
  std::vector<std::vector<Group>> groups;    // per strip: LSQML groups (global j mod G)
  int groups_batch = -1;
  int iter = 0;
  size_t halo_bytes = 0, probe_bytes = 0;    // sent so far

  void* dalloc(size_t bytes) {
    void* p = nullptr;
    const hipError_t e = hipMalloc(&p, std::max<size_t>(bytes, 16));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      throw NoMemError(std::string("hipMalloc of ") + std::to_string(bytes) + " bytes: " + hipGetErrorString(e));
    }
    allocs.push_back(p);
    return p;
  }
  ~pty_domains() {
    for (size_t s = 0; s < sub.size(); ++s) {
      if (s < groups.size())
        for (auto& g : groups[s]) free_group(sub[s], g);
      pty_destroy(sub[s]);
    }
    for (void* p : allocs) (void)hipFree(p);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

template <typename F>
pty_status guarded_d(pty_domains* d, F&& f) {
  const pty_status st = guarded(nullptr, std::forward<F>(f));
  if (st != PTY_OK && d) d->err = g_tls_error;
  return st;
}

void dd_check_sub(pty_domains* d, int s, pty_status st) {
  if (st == PTY_OK) return;
  const std::string m = "strip " + std::to_string(s) + ": " + pty_last_error(d->sub[s]);
  switch (st) {
    case PTY_E_INVALID: throw InvalidArg(m);
    case PTY_E_STATE: throw StateError(m);
    case PTY_E_NOMEM: throw NoMemError(m);
    case PTY_E_UNSUPPORTED: throw Unsupported(m);
    default: throw DeviceError(m);
  }
}

// Object-plane halos: partial sums of rows held by several strips go to the
// rows' owner, which adds them in strip order; the totals go back.  Planes:
// p0 (w0 words per row) and optionally p1 (w1 words per row), one message.
void dd_halo(pty_domains* d, const std::vector<float*>& p0, int w0, const std::vector<float*>& p1, int w1) {
  for (int pass = 0; pass < 2; ++pass) {
    for (const auto& g : d->segs) {
      const int from = pass == 0 ? g.src : g.dst, to = pass == 0 ? g.dst : g.src;
      const int rows = g.b - g.a;
      HaloPlanes a{{p0[from], w1 ? p1[from] : nullptr}, {w0, w1}, g.a - d->lo[from]};
      HaloPlanes b{{p0[to], w1 ? p1[to] : nullptr}, {w0, w1}, g.a - d->lo[to]};
      launch_halo_pack(a, rows, d->msg, d->stream);
      launch_halo_unpack(b, rows, d->msg, pass == 0, d->stream);
      d->halo_bytes += size_t(rows) * (w0 + w1) * sizeof(float);
    }
  }
}

// All-reduce of the probe sums: every strip's numerator (K x N x N complex)
// and, with den, its denominator (N x N) are packed into one message; the
// messages are summed in strip order and copied back into every strip.  With
// den, the maximum of the summed denominator goes to every strip's slot 1.
void dd_probe_allreduce(pty_domains* d, bool num2, bool with_den) {
  const size_t nn = size_t(d->N) * d->N;
  const int wn = int(2 * d->K * nn), wd = with_den ? int(nn) : 0;
  std::vector<const float*> m(d->S);
  for (int s = 0; s < d->S; ++s) {
    pty_ctx* c = d->sub[s];
    HaloPlanes a{{reinterpret_cast<float*>(num2 ? c->num_p2 : c->num_p), c->den_p}, {wn, wd}, 0};
    launch_halo_pack(a, 1, d->pmsg[s], d->stream);
    m[s] = d->pmsg[s];
    d->probe_bytes += size_t(wn + wd) * sizeof(float);
  }
  launch_sum_messages(m.data(), d->S, size_t(wn + wd), d->ptot, d->stream);
  for (int s = 0; s < d->S; ++s) {
    pty_ctx* c = d->sub[s];
    HaloPlanes b{{reinterpret_cast<float*>(num2 ? c->num_p2 : c->num_p), c->den_p}, {wn, wd}, 0};
    launch_halo_unpack(b, 1, d->ptot, false, d->stream);
  }
  if (with_den) {
    launch_fill_u32(d->dmax, 1, 0u, d->stream);
    launch_plane_max(d->ptot + wn, nn, d->dmax, d->stream);
    for (pty_ctx* c : d->sub)
      PTY_HIP(hipMemcpyAsync(c->scal + 1, d->dmax, sizeof(unsigned), hipMemcpyDeviceToDevice, d->stream));
  }
}

// After the halo exchange every strip holds complete object denominators on
// its rows: their overall maximum goes to every strip's slot 0.
void dd_den_max(pty_domains* d) {
  launch_fill_u32(d->dmax, 1, 0u, d->stream);
  for (pty_ctx* c : d->sub) launch_plane_max(c->den, size_t(c->H) * c->W, d->dmax, d->stream);
  for (pty_ctx* c : d->sub)
    PTY_HIP(hipMemcpyAsync(c->scal, d->dmax, sizeof(unsigned), hipMemcpyDeviceToDevice, d->stream));
}

// Object numerator (raw gather of the contribution planes: plain, or weighted
// by the step lengths) and, with den, the denominator, over group g of strip c.
void dd_object_sums(pty_ctx* c, const Group& g, float2* num, ObjOp op, bool with_den) {
  const size_t hw = size_t(c->H) * c->W;
  if (with_den) {
    launch_probe_intensity(c->probe, c->pint, c->N, c->K, c->stream);
    launch_fill_u32(reinterpret_cast<unsigned*>(c->den), hw, 0u, c->stream);
    launch_fill_u32(c->scal, 1, 0u, c->stream);
    ObjGatherArgs o = obj_args(c, g);
    launch_obj_gather(o, ObjOp::Density);
  }
  launch_fill_u32(reinterpret_cast<unsigned*>(num), hw * 2, 0u, c->stream);
  ObjGatherArgs o = obj_args(c, g);
  o.out = num;
  launch_obj_gather(o, op);
}

std::vector<float*> dd_planes(pty_domains* d, const std::function<void*(int)>& f) {
  std::vector<float*> v(d->S);
  for (int s = 0; s < d->S; ++s) v[s] = static_cast<float*>(f(s));
  return v;
}

void dd_ensure_err(pty_domains* d, int n_iter) {
  if (!d->iter_dev) {
    d->iter_dev = static_cast<int*>(d->dalloc(sizeof(int)));
    launch_set_i32(d->iter_dev, d->iter, d->stream);
  }
  if (d->err_dev && d->iter + n_iter <= d->err_cap) return;
  int cap = std::max(256, d->err_cap);
  while (cap < d->iter + n_iter) cap *= 2;
  double* nb = static_cast<double*>(d->dalloc(sizeof(double) * cap));
  if (d->err_dev && d->iter > 0)
    PTY_HIP(hipMemcpyAsync(nb, d->err_dev, sizeof(double) * d->iter, hipMemcpyDeviceToDevice, d->stream));
  d->err_dev = nb;   // the old buffer stays in allocs until destroy
  d->err_cap = cap;
}

void dd_end_iteration(pty_domains* d) {
  const int cb = col_blocks(d->N, d->K);
  for (int s = 0; s < d->S; ++s)
    launch_err_scatter(d->sub[s]->errp, d->d_jmap[s], d->sub[s]->J, 2 * cb, d->errp_all, d->stream);
  launch_err_reduce(d->errp_all, d->J * cb, d->err_dev, d->stream, d->iter_dev, true);
  d->iter++;
  for (pty_ctx* c : d->sub) c->iter = d->iter;
}

void dd_dm(pty_domains* d, int n_iter, const pty_iter_params& p) {
  const float g_obj = p.gamma_obj < 0 ? 1e-6f : p.gamma_obj;
  const float g_prb = p.gamma_probe < 0 ? 1e-6f : p.gamma_probe;
  for (pty_ctx* c : d->sub) {
    const int chunk = chunk_patterns(c, p);
    ensure_all_group(c);
    ensure_common(c, std::min(chunk, c->J), c->J);
    c->ensure_once(c->psi, size_t(c->J) * c->K * c->N * c->N);
    c->ensure_once(c->dobj, size_t(c->H) * c->W);
    ensure_probe_parts(c, c->J);
    if (!c->dm_valid) {
      DmInitArgs di{};
      di.n = c->N;
      di.k = c->K;
      di.obj = c->obj;
      di.h = c->H;
      di.w = c->W;
      di.probe = c->probe;
      di.pos = c->pos;
      di.j = c->J;
      di.psi = c->psi;
      di.contrib = c->contrib;
      di.stream = c->stream;
      launch_dm_init(di);
      c->dm_valid = true;
    }
  }
  dd_ensure_err(d, n_iter);
  const auto num = dd_planes(d, [&](int s) { return (void*)d->sub[s]->dobj; });
  const auto den = dd_planes(d, [&](int s) { return (void*)d->sub[s]->den; });
  for (int it = 0; it < n_iter; ++it) {
    const bool pon = probe_on(p, d->iter);
    for (pty_ctx* c : d->sub) dd_object_sums(c, c->all, c->dobj, ObjOp::Gradient, true);
    dd_halo(d, num, 2 * d->W, den, d->W);
    dd_den_max(d);
    for (pty_ctx* c : d->sub)
      launch_obj_apply(c->dobj, c->den, c->scal, g_obj, 1.f, c->obj, nullptr, size_t(c->H) * c->W, ObjApply::Dm,
                       c->stream);
    if (pon) {
      for (pty_ctx* c : d->sub) probe_reduce(c, c->all, c->psi, 1, PrbOp::Plain, c->num_p, true);
      dd_probe_allreduce(d, false, true);
      for (pty_ctx* c : d->sub) probe_apply(c, PrbApply::Dm, c->num_p, g_prb, 1.f);
    }
    for (pty_ctx* c : d->sub)
      fourier_pass(c, c->all, 0, c->J, chunk_patterns(c, p), RowIn::DmReflect, ColOp::Project, RowOut::DmUpdate);
    dd_end_iteration(d);
  }
}

void dd_ensure_lsq_groups(pty_domains* d, int batch) {
  if (d->groups_batch == batch) return;
  const int G = std::max(1, (d->J + batch - 1) / batch);
  for (int s = 0; s < d->S; ++s) {
    for (auto& g : d->groups[s]) free_group(d->sub[s], g);
    d->groups[s].assign(G, Group{});
    for (int g = 0; g < G; ++g) {
      std::vector<int> jl;
      for (int l = 0; l < (int)d->jmap[s].size(); ++l)
        if (d->jmap[s][l] % G == g) jl.push_back(l);
      make_group(d->sub[s], d->groups[s][g], std::move(jl));
    }
  }
  d->groups_batch = batch;
}

void dd_lsqml(pty_domains* d, int n_iter, const pty_iter_params& p) {
  const float g_obj = p.gamma_obj < 0 ? 1e-3f : p.gamma_obj;
  const float g_prb = p.gamma_probe < 0 ? 1e-3f : p.gamma_probe;
  const int batch = p.lsqml_batch > 0 ? p.lsqml_batch : 512;
  dd_ensure_lsq_groups(d, batch);
  const size_t nn = size_t(d->N) * d->N;
  for (int s = 0; s < d->S; ++s) {
    pty_ctx* c = d->sub[s];
    int bmax = 1;
    for (auto& g : d->groups[s]) bmax = std::max(bmax, (int)g.jl.size());
    const int chunk = chunk_patterns(c, p);
    ensure_common(c, std::min(chunk, bmax), bmax);
    c->ensure(c->chi, c->chi_slots, size_t(bmax) * c->K * nn);
    c->ensure_once(c->dobj, size_t(c->H) * c->W);
    c->ensure(c->alpha, c->alpha_slots, size_t(bmax));
    c->ensure_once(c->alpha_by_j, size_t(c->J));
    c->ensure_once(c->lsq_pq, nn);
    c->ensure_once(c->lsq_dint, nn);
    c->ensure(c->lsq_part, c->lsq_part_n, size_t(bmax) * lsq_row_blocks(c->N) * 5);
    ensure_probe_parts(c, bmax);
    if (!d->num2[s]) d->num2[s] = c->alloc<float2>(size_t(c->H) * c->W);
    c->dm_valid = false;
  }
  dd_ensure_err(d, n_iter);
  const auto dirp = dd_planes(d, [&](int s) { return (void*)d->sub[s]->dobj; });
  const auto den = dd_planes(d, [&](int s) { return (void*)d->sub[s]->den; });
  const auto upd = dd_planes(d, [&](int s) { return (void*)d->num2[s]; });
  const int G = (int)d->groups[0].size();
  for (int it = 0; it < n_iter; ++it) {
    const bool pon = probe_on(p, d->iter);
    for (int g = 0; g < G; ++g) {
      // pass A: chi, the object direction and the probe direction
      for (int s = 0; s < d->S; ++s) {
        pty_ctx* c = d->sub[s];
        const Group& grp = d->groups[s][g];
        const int count = (int)grp.jl.size();
        if (count > 0)
          fourier_pass(c, grp, 0, count, chunk_patterns(c, p), RowIn::Plain, ColOp::Project, RowOut::StoreChi);
        dd_object_sums(c, grp, c->dobj, ObjOp::Gradient, true);
      }
      dd_halo(d, dirp, 2 * d->W, den, d->W);
      dd_den_max(d);
      for (pty_ctx* c : d->sub)
        launch_obj_apply(c->dobj, c->den, c->scal, g_obj, 1.f, nullptr, c->dobj, size_t(c->H) * c->W,
                         ObjApply::LsqDirection, c->stream);
      if (pon) {
        for (int s = 0; s < d->S; ++s)
          probe_reduce(d->sub[s], d->groups[s][g], d->sub[s]->chi, 0, PrbOp::Plain, d->sub[s]->num_p, true);
        dd_probe_allreduce(d, false, true);
        for (pty_ctx* c : d->sub) probe_apply(c, PrbApply::LsqDirection, c->num_p, g_prb, 1.f);
      }
      // pass B: per-position step lengths
      for (int s = 0; s < d->S; ++s) {
        pty_ctx* c = d->sub[s];
        const Group& grp = d->groups[s][g];
        LsqStepArgs ls{};
        ls.n = c->N;
        ls.k = c->K;
        ls.obj = c->obj;
        ls.dobj = c->dobj;
        ls.h = c->H;
        ls.w = c->W;
        ls.probe = c->probe;
        ls.dprobe = c->dprobe;
        ls.chi = c->chi;
        ls.contrib = c->contrib;
        ls.pint = c->pint;
        ls.pq = c->lsq_pq;
        ls.dint = c->lsq_dint;
        ls.jlist = grp.d_jl;
        ls.pos = c->pos;
        ls.count = (int)grp.jl.size();
        ls.probe_on = pon ? 1 : 0;
        ls.part = c->lsq_part;
        ls.alpha = c->alpha;
        ls.alpha_by_j = c->alpha_by_j;
        ls.shift = nullptr;
        ls.stream = c->stream;
        launch_lsq_steps(ls);
      }
      // the step-weighted updates
      if (pon) {
        for (int s = 0; s < d->S; ++s)
          probe_reduce(d->sub[s], d->groups[s][g], d->sub[s]->chi, 0, PrbOp::AlphaWeighted, d->sub[s]->num_p2,
                       false);
        dd_probe_allreduce(d, true, false);
      }
      for (int s = 0; s < d->S; ++s) dd_object_sums(d->sub[s], d->groups[s][g], d->num2[s], ObjOp::WeightedSum, false);
      dd_halo(d, upd, 2 * d->W, {}, 0);
      for (int s = 0; s < d->S; ++s) {
        pty_ctx* c = d->sub[s];
        launch_obj_apply(d->num2[s], c->den, c->scal, g_obj, p.beta_obj, c->obj, nullptr, size_t(c->H) * c->W,
                         ObjApply::LsqUpdate, c->stream);
      }
      if (pon)
        for (pty_ctx* c : d->sub) probe_apply(c, PrbApply::LsqUpdate, c->num_p2, g_prb, p.beta_probe);
    }
    dd_end_iteration(d);
  }
  for (pty_ctx* c : d->sub) c->den_valid = false;
}

}  // namespace

extern "C" {

pty_status pty_domains_create(const pty_plan_desc* plan, const double* yx, int32_t strips, pty_domains** out) {
  pty_domains* created = nullptr;
  const pty_status st = guarded(nullptr, [&] {
    require(plan != nullptr && yx != nullptr && out != nullptr, "pty_domains_create: null argument");
    require(strips >= 1 && strips <= 16, "pty_domains_create: strips must be in 1..16");
    require(plan->n_pos >= strips, "pty_domains_create: fewer positions than strips");
    require(plan->flags == 0, "pty_domains_create: flags must be 0");
    const int J = plan->n_pos, N = plan->n, H = plan->obj_h, W = plan->obj_w;
    std::vector<int> iy(J), ey(J);
    for (int j = 0; j < J; ++j) {
      const double y = yx[2 * j], x = yx[2 * j + 1];
      if (!(std::isfinite(y) && std::isfinite(x)) || y < 0 || x < 0)
        throw InvalidArg("pty_domains_create: position " + std::to_string(j) + " is negative or not finite");
      const double fy = std::floor(y);
      iy[j] = (int)fy;
      ey[j] = (int)fy + N + (y != fy ? 1 : 0);
      if (ey[j] > H) throw InvalidArg("pty_domains_create: patch " + std::to_string(j) + " extends past the object");
    }
    std::unique_ptr<pty_domains> d(new pty_domains());
    d->S = strips;
    d->N = N;
    d->K = plan->modes;
    d->J = J;
    d->H = H;
    d->W = W;
    d->device = plan->device;
    PTY_HIP(hipSetDevice(plan->device));
    if (plan->stream) {
      d->stream = static_cast<hipStream_t>(plan->stream);
    } else {
      PTY_HIP(hipStreamCreateWithFlags(&d->stream, hipStreamNonBlocking));
      d->own_stream = true;
    }
    // equal counts by row (stable in the pattern index), then ascending index per strip
    std::vector<int> order(J);
    for (int j = 0; j < J; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return yx[2 * a] < yx[2 * b]; });
    d->jmap.resize(strips);
    int at = 0;
    for (int s = 0; s < strips; ++s) {
      const int cnt = J / strips + (s < J % strips ? 1 : 0);
      d->jmap[s].assign(order.begin() + at, order.begin() + at + cnt);
      std::sort(d->jmap[s].begin(), d->jmap[s].end());
      at += cnt;
    }
    std::vector<int> plo(strips), phi(strips);
    for (int s = 0; s < strips; ++s) {
      plo[s] = H;
      phi[s] = 0;
      for (int j : d->jmap[s]) {
        plo[s] = std::min(plo[s], iy[j]);
        phi[s] = std::max(phi[s], ey[j]);
      }
    }
    d->own_lo.resize(strips);
    d->own_hi.resize(strips);
    d->lo.resize(strips);
    d->hi.resize(strips);
    for (int s = 0; s < strips; ++s) d->own_lo[s] = s == 0 ? 0 : std::max(d->own_lo[s - 1], plo[s]);
    for (int s = 0; s < strips; ++s) d->own_hi[s] = s + 1 < strips ? d->own_lo[s + 1] : H;
    for (int s = 0; s < strips; ++s) {
      d->lo[s] = std::min(plo[s], d->own_lo[s]);
      d->hi[s] = std::max({phi[s], d->own_hi[s], std::min(H, d->lo[s] + N + 1)});
    }
    for (int s = 0; s < strips; ++s)
      for (int o = 0; o < strips; ++o) {
        if (o == s) continue;
        const int a = std::max(d->lo[s], d->own_lo[o]), b = std::min(d->hi[s], d->own_hi[o]);
        if (a < b) d->segs.push_back({s, o, a, b});
      }
    std::stable_sort(d->segs.begin(), d->segs.end(),
                     [](const pty_domains::Seg& x, const pty_domains::Seg& y) { return x.dst < y.dst; });
    // one context per strip, all on the decomposition's stream
    d->sub.assign(strips, nullptr);
    d->d_jmap.assign(strips, nullptr);
    d->num2.assign(strips, nullptr);
    d->groups.resize(strips);
    for (int s = 0; s < strips; ++s) {
      pty_plan_desc sp = *plan;
      sp.n_pos = (int)d->jmap[s].size();
      sp.obj_h = d->hi[s] - d->lo[s];
      sp.stream = d->stream;
      dd_check_sub(d.get(), s, pty_create(&sp, &d->sub[s]));
      std::vector<double> loc(2 * d->jmap[s].size());
      for (size_t l = 0; l < d->jmap[s].size(); ++l) {
        loc[2 * l] = yx[2 * d->jmap[s][l]] - d->lo[s];
        loc[2 * l + 1] = yx[2 * d->jmap[s][l] + 1];
      }
      dd_check_sub(d.get(), s, pty_load_positions(d->sub[s], loc.data()));
      d->d_jmap[s] = d->sub[s]->alloc<int>(d->jmap[s].size());
      PTY_HIP(hipMemcpy(d->d_jmap[s], d->jmap[s].data(), sizeof(int) * d->jmap[s].size(), hipMemcpyHostToDevice));
    }
    size_t mrows = 1;
    for (const auto& g : d->segs) mrows = std::max<size_t>(mrows, size_t(g.b - g.a));
    d->msg = static_cast<float*>(d->dalloc(mrows * 3 * W * sizeof(float)));
    d->pwords = size_t(2 * d->K + 1) * N * N;
    for (int s = 0; s < strips; ++s) d->pmsg.push_back(static_cast<float*>(d->dalloc(d->pwords * sizeof(float))));
    d->ptot = static_cast<float*>(d->dalloc(d->pwords * sizeof(float)));
    d->errp_all = static_cast<double*>(d->dalloc(sizeof(double) * 2 * size_t(J) * col_blocks(N, d->K)));
    d->dmax = static_cast<unsigned*>(d->dalloc(sizeof(unsigned)));
    created = d.release();
  });
  if (st == PTY_OK) *out = created;
  return st;
}

pty_status pty_domains_load_patterns(pty_domains* d, const float* counts, int on_device) {
  return guarded_d(d, [&] {
    require(d != nullptr && counts != nullptr, "pty_domains_load_patterns: null argument");
    PTY_HIP(hipSetDevice(d->device));
    const size_t nn = size_t(d->N) * d->N;
    for (int s = 0; s < d->S; ++s) {
      const auto& jm = d->jmap[s];
      if (!on_device) {
        std::vector<float> buf(jm.size() * nn);
        for (size_t l = 0; l < jm.size(); ++l) std::memcpy(&buf[l * nn], counts + size_t(jm[l]) * nn, nn * sizeof(float));
        dd_check_sub(d, s, pty_load_patterns(d->sub[s], buf.data(), 0));
      } else {
        float* tmp = d->sub[s]->alloc<float>(jm.size() * nn);
        for (size_t l = 0; l < jm.size(); ++l)
          PTY_HIP(hipMemcpyAsync(tmp + l * nn, counts + size_t(jm[l]) * nn, nn * sizeof(float),
                                 hipMemcpyDeviceToDevice, d->stream));
        const pty_status st = pty_load_patterns(d->sub[s], tmp, 1);
        d->sub[s]->dfree(tmp);
        dd_check_sub(d, s, st);
      }
    }
  });
}

pty_status pty_domains_set_object(pty_domains* d, const void* obj, int on_device) {
  return guarded_d(d, [&] {
    require(d != nullptr && obj != nullptr, "pty_domains_set_object: null argument");
    const float2* src = static_cast<const float2*>(obj);
    for (int s = 0; s < d->S; ++s)
      dd_check_sub(d, s, pty_set_object(d->sub[s], src + size_t(d->lo[s]) * d->W, on_device));
  });
}

pty_status pty_domains_set_probe(pty_domains* d, const void* probe, int on_device) {
  return guarded_d(d, [&] {
    require(d != nullptr && probe != nullptr, "pty_domains_set_probe: null argument");
    for (int s = 0; s < d->S; ++s) dd_check_sub(d, s, pty_set_probe(d->sub[s], probe, on_device));
  });
}

pty_status pty_domains_iterate(pty_domains* d, pty_algo algo, int32_t n_iter, const pty_iter_params* prm) {
  return guarded_d(d, [&] {
    require(d != nullptr, "pty_domains_iterate: null argument");
    require(n_iter >= 0, "pty_domains_iterate: negative iteration count");
    pty_iter_params p;
    if (prm)
      p = *prm;
    else
      pty_default_params(&p);
    if (algo != PTY_DM && algo != PTY_LSQML)
      throw Unsupported("pty_domains_iterate: only DM and LSQML are decomposed (ePIE is sequential)");
    if (p.flags != 0 || p.position_start >= 0)
      throw Unsupported("pty_domains_iterate: no flags and no position refinement in the strip decomposition");
    for (pty_ctx* c : d->sub) require_loaded(c);
    PTY_HIP(hipSetDevice(d->device));
    if (algo == PTY_DM)
      dd_dm(d, n_iter, p);
    else
      dd_lsqml(d, n_iter, p);
  });
}

pty_status pty_domains_get_object(pty_domains* d, void* out, int on_device) {
  return guarded_d(d, [&] {
    require(d != nullptr && out != nullptr, "pty_domains_get_object: null argument");
    PTY_HIP(hipSetDevice(d->device));
    float2* dst = static_cast<float2*>(out);
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    for (int s = 0; s < d->S; ++s) {
      const size_t rows = size_t(d->own_hi[s] - d->own_lo[s]);
      if (!rows) continue;
      PTY_HIP(hipMemcpyAsync(dst + size_t(d->own_lo[s]) * d->W,
                             d->sub[s]->obj + size_t(d->own_lo[s] - d->lo[s]) * d->W, rows * d->W * sizeof(float2),
                             kind, d->stream));
    }
    PTY_HIP(hipStreamSynchronize(d->stream));
  });
}

pty_status pty_domains_get_probe(pty_domains* d, void* out, int on_device) {
  return guarded_d(d, [&] {
    require(d != nullptr && out != nullptr, "pty_domains_get_probe: null argument");
    dd_check_sub(d, 0, pty_get_probe(d->sub[0], out, on_device));
  });
}

pty_status pty_domains_get_errors(pty_domains* d, double* out, int32_t cap, int32_t* n_written) {
  return guarded_d(d, [&] {
    require(d != nullptr && n_written != nullptr && (out != nullptr || cap == 0),
            "pty_domains_get_errors: null argument");
    const int n = std::min<int>(cap, d->iter);
    if (n > 0) {
      PTY_HIP(hipMemcpyAsync(out, d->err_dev, sizeof(double) * n, hipMemcpyDeviceToHost, d->stream));
      PTY_HIP(hipStreamSynchronize(d->stream));
    }
    *n_written = d->iter;
  });
}

pty_status pty_domains_strip(const pty_domains* d, int32_t s, int32_t* info) {
  return guarded(nullptr, [&] {
    require(d != nullptr && info != nullptr, "pty_domains_strip: null argument");
    require(s >= 0 && s < d->S, "pty_domains_strip: strip out of range");
    info[0] = d->lo[s];
    info[1] = d->hi[s];
    info[2] = d->own_lo[s];
    info[3] = d->own_hi[s];
    info[4] = (int32_t)d->jmap[s].size();
  });
}

pty_status pty_domains_traffic(const pty_domains* d, uint64_t* halo_bytes, uint64_t* probe_bytes) {
  return guarded(nullptr, [&] {
    require(d != nullptr && halo_bytes != nullptr && probe_bytes != nullptr, "pty_domains_traffic: null argument");
    *halo_bytes = d->halo_bytes;
    *probe_bytes = d->probe_bytes;
  });
}

pty_status pty_domains_sync(pty_domains* d) {
  return guarded_d(d, [&] {
    require(d != nullptr, "pty_domains_sync: null argument");
    PTY_HIP(hipStreamSynchronize(d->stream));
    PTY_HIP(hipGetLastError());
  });
}

void pty_domains_destroy(pty_domains* d) { delete d; }

const char* pty_domains_last_error(const pty_domains* d) { return d ? d->err.c_str() : g_tls_error.c_str(); }

}  // extern "C"
