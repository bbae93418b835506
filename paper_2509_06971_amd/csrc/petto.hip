// Host side of the C ABI declared in include/petto.h: argument checks, device
// workspace, and the orchestration of the relaxation (graph-captured blocks of
// sweeps polled through a host-mapped ring), the FP32/FP64 refinement loop, the
// sensitivity and the design update.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <algorithm>
#include <vector>

#include "kernels.hpp"
#include "petto.h"

using namespace petto;

// Partial sums of petto_adjoint_noalloc: a fixed device array (one per GPU, held
// until the process ends) in place of the context's workspace.  Slots
// [0, kScratchSlots) take the F.u partials, [kScratchSlots, 2 kScratchSlots) the
// energy partials.  Host code never passes this name to a kernel: it stands for
// the array only on the host side; the device address comes from
// hipGetSymbolAddress (scratch_resolve below).
constexpr int kScratchSlots = 65536;
static __device__ __align__(256) double scratch[2 * kScratchSlots];

namespace {

thread_local std::string g_err;

petto_status fail(petto_status s, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess) return fail(PETTO_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define PETTO_TRY(expr)                    \
  do {                                     \
    petto_status s_ = (expr);              \
    if (s_ < 0) return s_;                 \
  } while (0)

// Device addresses of `scratch`, one per GPU, resolved at context creation with
// that GPU current.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_addr[kMaxDevices] = {};

petto_status scratch_resolve() {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PETTO_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr[dev] == nullptr) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) return fail(PETTO_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_addr[dev] = static_cast<double*>(p);
  }
  return PETTO_OK;
}

petto_status scratch_lookup(double** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PETTO_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *out = g_scratch_addr[dev];
  if (*out == nullptr) return fail(PETTO_ERR_INVALID, "no context was created on device %d", dev);
  return PETTO_OK;
}

constexpr int kBpd = 256;          // material-kernel blocks per design
// Rayleigh-quotient blocks per design: about one per 4096 unknowns of the
// largest design, so that the pass over a large state fills the chip
constexpr long kRqPerBlock = 4096;
constexpr int kRqBlocksMin = 64, kRqBlocksMax = 1024;
constexpr int kGroup = 4;          // check blocks per graph launch
constexpr int kMaxOuter = 64;      // refinement: correction solves per call
constexpr double kDivFactor = 1e4;

struct TileList {            // heat work list for one sweeps-per-launch choice
  HeatTile* tiles = nullptr;
  int* tile0 = nullptr;      // [ndes + 1] per-design tile ranges
  int ntile = 0;
};

struct GraphEntry {
  std::vector<const void*> key;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct petto_ctx {
  int physics = 0, ndim = 2, prec = 0, nprob = 1, nphase = 1;
  std::vector<petto_problem> probs;
  ElGeom geom{};                       // elastic (single design)
  long nstate = 0;                     // elements of a state-layout buffer (all designs)
  long ncell = 0;                      // cells of one phase (all designs)
  std::vector<long> state_off, cell_off;
  long max_cells = 0;
  // problem data on the device
  double* F64 = nullptr;               // load in double (state layout), nullptr for uniform heat
  void* Ft = nullptr;                  // load in context precision
  uint32_t* pins = nullptr;
  HeatDesign* d_des = nullptr;
  HeatTile* d_tiles = nullptr;
  uint8_t* d_dir = nullptr;
  uint8_t* d_region = nullptr;         // PETTO_REGION_* per cell, or nullptr
  int* d_tile0 = nullptr;
  int ntile = 0;                       // partial-sum slots (largest tiling)
  std::map<int, TileList> heat_lists;  // heat work lists per sweeps-per-launch
  std::vector<HeatDesign> h_des;
  CellRange* d_ranges = nullptr;
  std::vector<CellRange> h_ranges;
  long* d_ncell = nullptr;
  double* d_fnorm = nullptr;
  double* d_h = nullptr;
  StateRange* d_srange = nullptr;      // per-design state ranges (Rayleigh-quotient sums)
  double* prq = nullptr;               // [nprob][rq_blocks][3]
  int rq_blocks = kRqBlocksMin;
  std::vector<double> fnorm;
  double m0 = 1.0;
  // workspace
  void* ualt = nullptr;
  void* valt = nullptr;                // velocity ping-pong partner of multi-sweep launches
  void* E = nullptr;
  double* E64 = nullptr;
  float* d32a = nullptr;
  float* d32b = nullptr;
  float* b32 = nullptr;
  double* partial = nullptr;
  double* partial2 = nullptr;
  double* partial_max = nullptr;
  SolveState* st = nullptr;
  int* ctl = nullptr;
  PollRecord* ring_host = nullptr;
  PollRecord* ring_dev = nullptr;
  double* phase_scal = nullptr;
  double* phase_work = nullptr;
  double* phase_partial = nullptr;
  double* pen_work = nullptr;          // penalty update: phi' per phase, mu, partition sum
  double* phase_used = nullptr;        // Allen-Cahn update: sum of the phases already updated
  double* comp = nullptr;
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_end[kRing] = {};
  hipEvent_t ev_beg[kRing] = {};
  bool events = false;
  std::vector<GraphEntry> graphs;
  int blocking = 0;                    // sweeps per launch (2D); 0: tune on the first solve
  bool tuned3d = false;                // 3D tiling timed (or set by the caller)
  void* tune_a = nullptr;              // FP64 contexts: state, partner and right-hand side for timing
  void* tune_b = nullptr;
  void* tune_c = nullptr;
  int ncu = 256;                       // compute units of the device (3D tiling choice)
  SolveState* st_t = nullptr;          // running copy of st for kernel timing (done = 0)
  bool timing = false;
  double timed_ms = 0.0;
  int64_t timed_sweeps = 0;
  std::vector<void*> allocations;
};

namespace {

size_t elem_size(const petto_ctx* c) { return c->prec == PETTO_FP64 ? sizeof(double) : sizeof(float); }

petto_status dalloc(petto_ctx* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(PETTO_ERR_OOM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  c->allocations.push_back(*p);
  return PETTO_OK;
}

template <typename P>
petto_status dalloc_t(petto_ctx* c, P** p, size_t count) {
  void* v = nullptr;
  petto_status s = dalloc(c, &v, count * sizeof(P));
  *p = static_cast<P*>(v);
  return s;
}

template <typename P>
petto_status upload(petto_ctx* c, P** p, const std::vector<P>& h) {
  PETTO_TRY(dalloc_t(c, p, h.size()));
  if (!h.empty()) HIP_TRY(hipMemcpy(*p, h.data(), h.size() * sizeof(P), hipMemcpyHostToDevice));
  return PETTO_OK;
}

long padded_state(const petto_problem& p) {
  long n = 1;
  for (int a = 0; a < p.ndim; ++a) n *= (long)p.n[a] + 1;
  return n * p.ndim;
}

long cells(const petto_problem& p) {
  long n = 1;
  for (int a = 0; a < p.ndim; ++a) n *= p.n[a];
  return n;
}

// canonical flat index of component a at (i, j, k)
long sidx(const petto_problem& p, int a, long i, long j, long k) {
  const long px = p.n[0] + 1, py = p.n[1] + 1;
  const long pz = p.ndim == 3 ? p.n[2] + 1 : 1;
  return (long)a * px * py * pz + (k * py + j) * px + i;
}

bool is_finite(double x) { return std::isfinite(x); }

petto_status validate_problem(const petto_problem& p, int idx) {
  if (p.physics != PETTO_ELASTIC && p.physics != PETTO_HEAT)
    return fail(PETTO_ERR_INVALID, "problem %d: physics must be PETTO_ELASTIC or PETTO_HEAT", idx);
  if (p.ndim != 2 && p.ndim != 3) return fail(PETTO_ERR_INVALID, "problem %d: ndim must be 2 or 3", idx);
  for (int a = 0; a < p.ndim; ++a) {
    if (p.n[a] < 2 || p.n[a] > (1 << 16))
      return fail(PETTO_ERR_INVALID, "problem %d: n[%d]=%d outside [2, 65536]", idx, a, p.n[a]);
  }
  if (!(p.h > 0.0) || !is_finite(p.h)) return fail(PETTO_ERR_INVALID, "problem %d: h must be positive", idx);
  if (p.region != nullptr) {
    long n = (long)p.n[0] * p.n[1] * (p.ndim == 3 ? p.n[2] : 1);
    for (long q = 0; q < n; ++q)
      if (p.region[q] > PETTO_REGION_SOLID)
        return fail(PETTO_ERR_INVALID, "problem %d: region[%ld] = %d is not a cell role", idx, q, (int)p.region[q]);
  }
  if (p.nphase < 1 || p.nphase > kMaxPhase)
    return fail(PETTO_ERR_INVALID, "problem %d: nphase must be in [1, %d]", idx, kMaxPhase);
  if (!(p.p >= 1.0) || !is_finite(p.p)) return fail(PETTO_ERR_INVALID, "problem %d: penalty p must be >= 1", idx);
  if (p.nphase == 1) {
    if (!(p.e0 > 0.0) || !(p.emin >= 0.0) || !(p.emin < p.e0) || !is_finite(p.e0))
      return fail(PETTO_ERR_INVALID, "problem %d: need 0 <= emin < e0", idx);
  } else {
    if (p.physics != PETTO_ELASTIC)
      return fail(PETTO_ERR_INVALID, "problem %d: several phases are elastic only", idx);
    for (int m = 0; m <= p.nphase; ++m)
      if (!(p.e_phase[m] >= 0.0) || !is_finite(p.e_phase[m]))
        return fail(PETTO_ERR_INVALID, "problem %d: e_phase[%d] must be >= 0", idx, m);
    if (!(p.e_phase[0] > 0.0)) return fail(PETTO_ERR_INVALID, "problem %d: e_phase[0] must be > 0", idx);
  }
  if (p.physics == PETTO_ELASTIC && p.ndim == 3 && (long)(p.n[0] + 1) * (p.n[1] + 1) >= (1L << 29))
    // the 3D sweep addresses within one xy layer by 32-bit byte offsets (FP64: 8 B)
    return fail(PETTO_ERR_UNSUPPORTED, "problem %d: an xy layer of %d x %d positions is too large for the 3D sweep",
                idx, p.n[0] + 1, p.n[1] + 1);
  if (p.physics == PETTO_ELASTIC) {
    if (!(p.nu >= 0.0 && p.nu < 0.5)) return fail(PETTO_ERR_INVALID, "problem %d: nu must be in [0, 0.5)", idx);
    for (int s = 0; s < 2 * p.ndim; ++s)
      if (p.side[s] < 0 || p.side[s] > 2) return fail(PETTO_ERR_INVALID, "problem %d: side[%d] invalid", idx, s);
    if (p.load == nullptr) return fail(PETTO_ERR_INVALID, "problem %d: elastic problem needs a load", idx);
  } else {
    if (p.fixed == nullptr) return fail(PETTO_ERR_INVALID, "problem %d: heat problem needs Dirichlet faces", idx);
    if (p.load == nullptr && !is_finite(p.q)) return fail(PETTO_ERR_INVALID, "problem %d: q must be finite", idx);
  }
  return PETTO_OK;
}

// Elastic: check the mask against the sides, build the extra-pin bitmask and the load.
petto_status prepare_elastic(petto_ctx* c, const petto_problem& p, std::vector<uint32_t>& pins_words,
                             bool& any_pin, std::vector<double>& F) {
  const long ns = padded_state(p);
  const int nx = p.n[0], ny = p.n[1], nz = p.ndim == 3 ? p.n[2] : 1;
  const int n3[3] = {nx, ny, nz};
  std::vector<uint8_t> valid(ns, 0), side_fixed(ns, 0);
  for (int a = 0; a < p.ndim; ++a)
    for (int k = 0; k < (p.ndim == 3 ? nz + 1 : 1); ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
          const int id[3] = {i, j, k};
          bool ok = true;
          for (int b = 0; b < p.ndim; ++b) {
            if (b == a) continue;
            if (id[b] >= n3[b]) ok = false;
          }
          if (!ok) continue;
          const long q = sidx(p, a, i, j, k);
          valid[q] = 1;
          if ((id[a] == 0 && p.side[2 * a] != PETTO_SIDE_FREE) || (id[a] == n3[a] && p.side[2 * a + 1] != PETTO_SIDE_FREE))
            side_fixed[q] = 1;
        }
  pins_words.assign((ns + 31) / 32, 0u);
  any_pin = false;
  long nfixed = 0;
  for (long q = 0; q < ns; ++q) {
    const bool f = p.fixed != nullptr && p.fixed[q] != 0;
    if (f && !valid[q]) return fail(PETTO_ERR_INVALID, "fixed mask marks padding slot %ld", q);
    if (side_fixed[q] && p.fixed != nullptr && !f)
      return fail(PETTO_ERR_INVALID, "fixed mask misses the normal unknown %ld of a clamped/roller side", q);
    if (f && !side_fixed[q]) {
      pins_words[q >> 5] |= 1u << (q & 31);
      any_pin = true;
    }
    if (f || side_fixed[q]) ++nfixed;
  }
  if (nfixed == 0) return fail(PETTO_ERR_INVALID, "elastic problem has no Dirichlet unknown (rigid modes)");
  F.assign(ns, 0.0);
  double ss = 0.0;
  for (long q = 0; q < ns; ++q) {
    const double v = p.load[q];
    if (!is_finite(v)) return fail(PETTO_ERR_INVALID, "load is not finite at %ld", q);
    if (!valid[q] || side_fixed[q] || (p.fixed && p.fixed[q])) continue;
    F[q] = v;
    ss += v * v;
  }
  if (!(ss > 0.0)) return fail(PETTO_ERR_INVALID, "elastic load is zero on the free unknowns");
  c->fnorm.push_back(std::sqrt(ss));
  return PETTO_OK;
}

petto_status check_heat_mask(const petto_problem& p, int idx) {
  const int nx = p.n[0], ny = p.n[1];
  long nd = 0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const uint8_t b = p.fixed[(long)j * nx + i];
      if ((b & 1) && i != 0) return fail(PETTO_ERR_INVALID, "problem %d: -x Dirichlet bit on interior cell", idx);
      if ((b & 2) && i != nx - 1) return fail(PETTO_ERR_INVALID, "problem %d: +x Dirichlet bit on interior cell", idx);
      if ((b & 4) && j != 0) return fail(PETTO_ERR_INVALID, "problem %d: -y Dirichlet bit on interior cell", idx);
      if ((b & 8) && j != ny - 1) return fail(PETTO_ERR_INVALID, "problem %d: +y Dirichlet bit on interior cell", idx);
      if (b & 0xF0) return fail(PETTO_ERR_INVALID, "problem %d: unknown Dirichlet bits", idx);
      nd += (b & 1) + ((b >> 1) & 1) + ((b >> 2) & 1) + ((b >> 3) & 1);
    }
  if (nd == 0) return fail(PETTO_ERR_INVALID, "problem %d: heat design has no Dirichlet face", idx);
  return PETTO_OK;
}

void destroy_graphs(petto_ctx* c) {
  for (auto& g : c->graphs)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
}

petto_status ensure_events(petto_ctx* c) {
  if (c->events) return PETTO_OK;
  for (int i = 0; i < kRing; ++i) {
    HIP_TRY(hipEventCreate(&c->ev_end[i]));
    HIP_TRY(hipEventCreate(&c->ev_beg[i]));
  }
  c->events = true;
  return PETTO_OK;
}

// Enqueue one block of sweeps either through a cached graph (captured on the
// context's private stream, replayed on the caller's) or directly.
petto_status enqueue_block(petto_ctx* c, hipStream_t stream, bool use_graph, const std::vector<const void*>& key,
                           const std::function<void(hipStream_t)>& body) {
  if (!use_graph) {
    body(stream);
    HIP_TRY(hipGetLastError());
    return PETTO_OK;
  }
  for (auto& g : c->graphs) {
    if (g.key == key) {
      HIP_TRY(hipGraphLaunch(g.exec, stream));
      return PETTO_OK;
    }
  }
  if (c->cap_stream == nullptr) HIP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  body(c->cap_stream);
  hipError_t le = hipGetLastError();
  hipGraph_t graph = nullptr;
  hipError_t ee = hipStreamEndCapture(c->cap_stream, &graph);
  if (le != hipSuccess) return fail(PETTO_ERR_HIP, "kernel launch during capture failed: %s", hipGetErrorString(le));
  if (ee != hipSuccess) return fail(PETTO_ERR_HIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ee));
  hipGraphExec_t exec = nullptr;
  hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ie != hipSuccess) return fail(PETTO_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
  if (c->graphs.size() >= 16) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({key, exec});
  HIP_TRY(hipGraphLaunch(exec, stream));
  return PETTO_OK;
}

// Run blocks until the finalize kernel reports every design done.  Blocks go to
// the GPU in groups of kGroup per graph launch (with graphs; one poll event per
// group): the GPU idles at every launch boundary, and groups cut their number.  Two groups are kept in flight; the device applies the stop rule after
// every block, so a block enqueued after the stop finds the done flags set and its
// kernels return at once.  Blocks timed (when enabled) are those of the groups up
// to the stop.  With last == nullptr (a fixed block count whose caller wants no
// report) the groups are only enqueued.
petto_status run_blocks(petto_ctx* c, hipStream_t stream, bool use_graph, const std::vector<const void*>& key,
                        const std::function<void(hipStream_t)>& body, int sweeps_per_block, PollRecord* last,
                        long max_blocks) {
  PETTO_TRY(ensure_events(c));
  const int G = (use_graph && max_blocks >= kGroup) ? kGroup : 1;
  std::vector<const void*> gkey = key;
  gkey.push_back((const void*)(long)G);
  const std::function<void(hipStream_t)> group = [&](hipStream_t st) {
    for (int q = 0; q < G; ++q) body(st);
  };
  const long ngroups = (max_blocks + G - 1) / G;
  if (last == nullptr) {
    // a fixed count with nothing to report: enqueue every group and return; the
    // host neither waits nor reads the poll ring (the finalize kernels still
    // apply the stop rule on the device)
    for (long b = 0; b < ngroups; ++b) PETTO_TRY(enqueue_block(c, stream, use_graph, gkey, group));
    return PETTO_OK;
  }
  long launched = 0, checked = 0;
  for (;;) {
    // never more groups than the stop rule can use
    while (launched - checked < 2 && launched < ngroups) {
      if (c->timing) HIP_TRY(hipEventRecord(c->ev_beg[launched % kRing], stream));
      PETTO_TRY(enqueue_block(c, stream, use_graph, gkey, group));
      HIP_TRY(hipEventRecord(c->ev_end[launched % kRing], stream));
      ++launched;
    }
    HIP_TRY(hipEventSynchronize(c->ev_end[checked % kRing]));
    // the record of the group's last block (every finalize writes one)
    const long seq = (checked + 1) * G - 1;
    volatile PollRecord* r = &c->ring_host[seq % kRing];
    const PollRecord rec{r->all_done, r->any_diverged, r->any_not_converged, r->seq};
    if (rec.seq != (int)(seq % 0x7fffffff)) {
      (void)hipStreamSynchronize(stream);
      return fail(PETTO_ERR_HIP, "poll ring out of step (seq %d, expected %ld)", rec.seq, seq);
    }
    if (c->timing) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, c->ev_beg[checked % kRing], c->ev_end[checked % kRing]));
      c->timed_ms += ms;
      c->timed_sweeps += (long)sweeps_per_block * G;
    }
    ++checked;
    if (rec.all_done || checked == ngroups) {
      *last = rec;
      break;
    }
  }
  HIP_TRY(hipStreamSynchronize(stream));
  return PETTO_OK;
}

petto_status check_apt_params(const petto_ctx* c, const petto_apt_params* p) {
  if (p == nullptr) return fail(PETTO_ERR_INVALID, "apt params are NULL");
  if (!(p->theta >= 0.0) || !is_finite(p->theta)) return fail(PETTO_ERR_INVALID, "theta must be >= 0");
  if (!is_finite(p->dt)) return fail(PETTO_ERR_INVALID, "dt must be finite (<= 0 selects the default)");
  if (p->check_every < 2 || (p->check_every & 1))
    return fail(PETTO_ERR_INVALID, "check_every must be even and >= 2");
  if (p->max_iter < p->check_every) return fail(PETTO_ERR_INVALID, "max_iter must be >= check_every");
  if (p->replay_iters < 0 || (p->replay_iters % p->check_every) != 0)
    return fail(PETTO_ERR_INVALID, "replay_iters must be a nonnegative multiple of check_every");
  if (p->replay_iters == 0 && !(p->tol > 0.0)) return fail(PETTO_ERR_INVALID, "tol must be > 0");
  if (p->adapt) {
    if (p->dt > 0.0) return fail(PETTO_ERR_INVALID, "adapt needs the automatic step (dt <= 0)");
    if (!(p->theta > 0.0)) return fail(PETTO_ERR_INVALID, "adapt needs theta > 0 (the damping floor)");
  }
  if (p->refine) {
    if (c->prec != PETTO_FP32) return fail(PETTO_ERR_INVALID, "refine applies to FP32 contexts only");
    if (p->replay_iters) return fail(PETTO_ERR_INVALID, "replay_iters cannot be combined with refine");
  }
  if (p->n_pt < 0 || (p->n_pt & 1)) return fail(PETTO_ERR_INVALID, "n_pt must be even and >= 0");
  if (!is_finite(p->dt_pt)) return fail(PETTO_ERR_INVALID, "dt_pt must be finite (<= 0 selects the default)");
  return PETTO_OK;
}

// ------------------------------------------------------------------------------ sweep bodies

// Sweeps per launch for a block of nchk sweeps: the context's choice when the
// block splits into an even number of launches of that size, else 1.
int block_k(const petto_ctx* c, int nchk) {
  if (c->ndim != 2) return 1;
  const int k = c->blocking > 0 ? c->blocking : 1;
  return (k > 1 && nchk % (2 * k) == 0) ? k : 1;
}

template <typename T, bool CHECK>
int launch_tb(int k, const ElGeom& g, const ElSweep<T>& a, hipStream_t s) {
  switch (k) {
    case 2: return launch_el2d_tb<T, 2, CHECK>(g, a, s);
    case 4: return launch_el2d_tb<T, 4, CHECK>(g, a, s);
    case 5: return launch_el2d_tb<T, 5, CHECK>(g, a, s);
    case 8: return launch_el2d_tb<T, 8, CHECK>(g, a, s);
    case 10: return launch_el2d_tb<T, 10, CHECK>(g, a, s);
    default: return 0;
  }
}

template <>
int launch_tb<double, false>(int k, const ElGeom& g, const ElSweep<double>& a, hipStream_t s) {
  switch (k) {
    case 2: return launch_el2d_tb<double, 2, false>(g, a, s);
    case 4: return launch_el2d_tb<double, 4, false>(g, a, s);
    case 5: return launch_el2d_tb<double, 5, false>(g, a, s);
    default: return 0;
  }
}

template <>
int launch_tb<double, true>(int k, const ElGeom& g, const ElSweep<double>& a, hipStream_t s) {
  switch (k) {
    case 2: return launch_el2d_tb<double, 2, true>(g, a, s);
    case 4: return launch_el2d_tb<double, 4, true>(g, a, s);
    case 5: return launch_el2d_tb<double, 5, true>(g, a, s);
    default: return 0;
  }
}

// nchk sweeps ping-ponging u <-> ualt (an even number of launches: the result
// lands in u).  With `check`, the last sweep also sums r^2 for the finalize
// kernel.  Returns the number of partial-sum slots the check launch writes.
template <typename T>
int elastic_sweeps(const petto_ctx* c, hipStream_t s, T* u, T* ualt, T* v, const T* E, const T* b,
                   SolveState* st, int nchk, bool check = false) {
  ElSweep<T> a{};
  a.v = v;
  a.E = E;
  a.b = b;
  a.st = st;
  a.partial = c->partial;
  const int k = block_k(c, nchk);
  const int nl = nchk / k;
  T* valt = static_cast<T*>(c->valt);
  int nt = 0;
  for (int q = 0; q < nl; ++q) {
    a.uin = (q & 1) ? ualt : u;
    a.uout = (q & 1) ? u : ualt;
    a.v = (k > 1 && (q & 1)) ? valt : v;
    a.vout = (k > 1 && !(q & 1)) ? valt : v;
    const bool chk = check && q == nl - 1;
    if (c->ndim == 2) {
      if (k > 1) nt = chk ? launch_tb<T, true>(k, c->geom, a, s) : launch_tb<T, false>(k, c->geom, a, s);
      else nt = chk ? launch_el2d<T, kCheck>(c->geom, a, s) : launch_el2d<T, kSweep>(c->geom, a, s);
    } else {
      nt = chk ? launch_el3d<T, kCheck>(c->geom, a, s) : launch_el3d<T, kSweep>(c->geom, a, s);
    }
  }
  return nt;
}

template <typename T, bool CHECK>
void launch_htb(int k, const HeatSweep<T>& a, hipStream_t s) {
  switch (k) {
    case 2: launch_heat2d_tb<T, 2, CHECK>(a, s); break;
    case 4: launch_heat2d_tb<T, 4, CHECK>(a, s); break;
    case 5: launch_heat2d_tb<T, 5, CHECK>(a, s); break;
    case 8: if (std::is_same<T, float>::value) launch_heat2d_tb<float, 8, CHECK>(reinterpret_cast<const HeatSweep<float>&>(a), s); break;
    case 10: if (std::is_same<T, float>::value) launch_heat2d_tb<float, 10, CHECK>(reinterpret_cast<const HeatSweep<float>&>(a), s); break;
    default: break;
  }
}

// nchk heat sweeps of every unconverged design; returns the work list the last
// (checking) launch used, whose tile ranges the finalize kernel needs.
template <typename T>
const TileList* heat_sweeps(const petto_ctx* c, hipStream_t s, T* u, T* ualt, T* v, const T* k, const T* b,
                            SolveState* st, int nchk, bool check = false, int* all_done = nullptr) {
  const int kk = block_k(c, nchk);
  const TileList& L = c->heat_lists.at(kk);
  HeatSweep<T> a{};
  a.v = v;
  a.k = k;
  a.b = b;
  a.des = c->d_des;
  a.tiles = L.tiles;
  a.dir = c->d_dir;
  a.st = st;
  a.all_done = all_done != nullptr ? all_done : c->ctl + 1;
  a.partial = c->partial;
  a.ntile = L.ntile;
  const int nl = nchk / kk;
  T* valt = static_cast<T*>(c->valt);
  for (int q = 0; q < nl; ++q) {
    a.uin = (q & 1) ? ualt : u;
    a.uout = (q & 1) ? u : ualt;
    a.v = (kk > 1 && (q & 1)) ? valt : v;
    a.vout = (kk > 1 && !(q & 1)) ? valt : v;
    const bool chk = check && q == nl - 1;
    if (kk == 1) {
      if (chk) launch_heat2d<T, kCheck>(a, s);
      else launch_heat2d<T, kSweep>(a, s);
    } else {
      if (chk) launch_htb<T, true>(kk, a, s);
      else launch_htb<T, false>(kk, a, s);
    }
  }
  return &L;
}

int el_tiles_for(const petto_ctx* c, bool fp64) {
  if (c->ndim == 2) return el2d_tiles(c->geom);
  return el3d_tiles_prec(c->geom, fp64);   // 3D tiles depend on the kernel precision
}

// The partial sums the checking launch wrote: per-design ranges tile0 (heat
// batches) or, for one design, slots [0, ntile).
void finalize(const petto_ctx* c, hipStream_t s, SolveState* st, const int* tile0, int ntile, int mode,
              bool adapt = false) {
  FinalizeArgs f{};
  f.prq = adapt ? c->prq : nullptr;
  f.rq_blocks = c->rq_blocks;
  f.st = st;
  f.partial = c->partial;
  f.tile0 = tile0;
  f.ntile = ntile;
  f.ndes = c->nprob;
  f.ncell = c->d_ncell;
  f.ctl = c->ctl;
  f.ring = c->ring_dev;
  f.mode = mode;
  f.div_factor = kDivFactor;
  launch_finalize(f, s);
}

template <typename T>
petto_status material(petto_ctx* c, const void* phi, hipStream_t s, bool with64) {
  const petto_problem& p = c->probs[0];
  const double* ep = p.e_phase;
  launch_material<T>(static_cast<const T*>(phi), static_cast<T*>(c->E), with64 ? c->E64 : nullptr, c->d_ranges,
                     c->nprob, c->max_cells, c->nphase, c->ncell, p.e0, p.emin, p.p, ep, c->partial_max, kBpd, s);
  HIP_TRY(hipGetLastError());
  return PETTO_OK;
}

petto_status setup(petto_ctx* c, hipStream_t s, SolveState* st, const petto_apt_params* ap, double tol, int replay,
                   int max_iter) {
  SetupArgs a{};
  a.adapt = ap->adapt != 0;
  a.st = st;
  a.partial_max = c->partial_max;
  a.blocks_per_design = kBpd;
  a.ndes = c->nprob;
  a.fnorm = c->d_fnorm;
  a.h = c->d_h;
  a.m0 = c->m0;
  a.ndim = c->ndim;
  a.theta = ap->theta;
  a.dt_user = ap->dt;
  a.tol = tol;
  a.max_iter = max_iter;
  a.check_every = ap->check_every;
  a.replay = replay;
  a.ctl = c->ctl;
  launch_setup(a, s);
  HIP_TRY(hipGetLastError());
  return PETTO_OK;
}

petto_status read_states(petto_ctx* c, SolveState* dev, std::vector<SolveState>& h, hipStream_t s) {
  h.resize(c->nprob);
  HIP_TRY(hipMemcpyAsync(h.data(), dev, sizeof(SolveState) * c->nprob, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return PETTO_OK;
}

petto_status status_of(const std::vector<SolveState>& h) {
  petto_status worst = PETTO_OK;
  for (const auto& s : h) {
    if (s.status == -3) return fail(PETTO_ERR_DIVERGED, "relaxation diverged (residual non-finite or grew 1e4x)");
    if (s.status == 1) worst = PETTO_NOT_CONVERGED;
  }
  return worst;
}

// Sweeps-per-launch autotuner (2D elastic, FP32): after setup has written the
// sweep coefficients, time each candidate on workspace buffers (the caller's
// state is untouched) and keep the fastest per swept cell.  Results do not depend
// on the choice (all candidates are bit-identical).
// ------------------------------------------------------------------------------ launch autotuner
//
// On the first solve of a context the launch choices that leave results
// unchanged are timed on workspace buffers and the fastest kept: the sweeps per
// launch of the 2D relaxations (elastic and heat, FP32 and FP64) and the tiling
// of the 3D sweep.  Choices are cached for the process per (physics, dimension,
// precision, check interval, compute units, grid sizes of every design), so a
// new context of the same shape skips the timing.

struct TuneChoice {
  int blocking = 0;
  int tile3d = 0;
};
std::mutex g_tune_mu;
std::map<std::vector<long>, TuneChoice> g_tune_cache;

std::vector<long> tune_key(const petto_ctx* c, int nchk) {
  std::vector<long> k = {c->physics, c->ndim, c->prec, nchk, c->ncu, c->nprob};
  for (const petto_problem& p : c->probs) {
    k.push_back(p.n[0]);
    k.push_back(p.n[1]);
    k.push_back(c->ndim == 3 ? p.n[2] : 1);
  }
  return k;
}

// Mean milliseconds per sweep of `n` sweeps (after one untimed block of the same
// size) with the context's current launch choice, from zero state on workspace
// buffers.
template <typename T>
petto_status time_choice(petto_ctx* c, hipStream_t s, T* u, T* ua, T* v, const T* b, int n, double* ms_out) {
  const T* E = static_cast<const T*>(c->E);
  launch_fill<T>(u, c->nstate, T(0), s);
  launch_fill<T>(v, c->nstate, T(0), s);
  auto run = [&]() {
    if (c->physics == PETTO_ELASTIC) elastic_sweeps<T>(c, s, u, ua, v, E, b, c->st, n);
    else heat_sweeps<T>(c, s, u, ua, v, E, nullptr, c->st, n);
  };
  run();
  HIP_TRY(hipEventRecord(c->ev_beg[0], s));
  run();
  HIP_TRY(hipEventRecord(c->ev_end[0], s));
  HIP_TRY(hipEventSynchronize(c->ev_end[0]));
  HIP_TRY(hipGetLastError());
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev_beg[0], c->ev_end[0]));
  *ms_out = ms / (double)n;
  return PETTO_OK;
}

// Time the candidates of whichever choice is still open (blocking == 0 for 2D,
// tuned3d false for 3D elastic).  c->st must hold the coefficients of the solve
// about to run, with its stop flag clear.
template <typename T>
petto_status ensure_tuning(petto_ctx* c, hipStream_t s, int nchk) {
  const bool three = c->physics == PETTO_ELASTIC && c->ndim == 3;
  if (three ? c->tuned3d : c->blocking != 0) return PETTO_OK;
  const std::vector<long> key = tune_key(c, nchk);
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      if (three) {
        c->geom.tile3d = it->second.tile3d;
        c->tuned3d = true;
        destroy_graphs(c);
      } else {
        c->blocking = it->second.blocking;
      }
      return PETTO_OK;
    }
  }
  PETTO_TRY(ensure_events(c));
  T* u;
  T* ua;
  T* b;
  if (std::is_same<T, float>::value) {
    u = reinterpret_cast<T*>(c->d32a);
    ua = reinterpret_cast<T*>(c->d32b);
    b = reinterpret_cast<T*>(c->b32);
  } else {
    u = static_cast<T*>(c->tune_a);
    ua = static_cast<T*>(c->tune_b);
    b = static_cast<T*>(c->tune_c);
  }
  T* v = static_cast<T*>(c->ualt);
  launch_fill<T>(b, c->nstate, T(0), s);
  TuneChoice choice;
  double best = 1e300;
  if (three) {
    const int cands[] = {1, 2, 3};
    for (int t : cands) {
      c->geom.tile3d = t;
      double ms = 0.0;
      PETTO_TRY(time_choice<T>(c, s, u, ua, v, b, 20, &ms));
      if (ms < best) {
        best = ms;
        choice.tile3d = t;
      }
    }
    c->geom.tile3d = choice.tile3d;
    c->tuned3d = true;
    destroy_graphs(c);
  } else {
    const bool fp64 = c->prec == PETTO_FP64;
    const int cands32[] = {1, 2, 4, 5, 8, 10};
    const int cands64[] = {1, 2, 4, 5};
    const int* cands = fp64 ? cands64 : cands32;
    const int ncand = fp64 ? 4 : 6;
    choice.blocking = 1;
    for (int q = 0; q < ncand; ++q) {
      const int k = cands[q];
      if (nchk % (2 * k) != 0) continue;
      c->blocking = k;
      double ms = 0.0;
      // 40 sweeps or at least 4 launches, an even count
      const int n = (40 / k < 4 ? 4 : (40 / k + 1) / 2 * 2) * k;
      PETTO_TRY(time_choice<T>(c, s, u, ua, v, b, n, &ms));
      if (ms < best) {
        best = ms;
        choice.blocking = k;
      }
    }
    c->blocking = choice.blocking;
  }
  std::lock_guard<std::mutex> lock(g_tune_mu);
  TuneChoice& slot = g_tune_cache[key];
  if (three) slot.tile3d = choice.tile3d;
  else slot.blocking = choice.blocking;
  return PETTO_OK;
}

// Plain relaxation in the context precision.
template <typename T>
petto_status solve_plain(petto_ctx* c, const void* phi, void* u, void* v, const petto_apt_params* ap,
                         hipStream_t s, petto_solve_info* info, bool material_ready) {
  if (!material_ready) PETTO_TRY(material<T>(c, phi, s, false));
  const int replay = ap->replay_iters > 0;
  PETTO_TRY(setup(c, s, c->st, ap, replay ? -1.0 : ap->tol, replay, replay ? ap->replay_iters : ap->max_iter));
  launch_fill<T>(static_cast<T*>(v), c->nstate, T(0), s);
  HIP_TRY(hipGetLastError());
  T* uu = static_cast<T*>(u);
  T* ua = static_cast<T*>(c->ualt);
  T* vv = static_cast<T*>(v);
  const T* E = static_cast<const T*>(c->E);
  const T* b = static_cast<const T*>(c->Ft);
  const int nchk = ap->check_every;
  PETTO_TRY(ensure_tuning<T>(c, s, nchk));
  const bool adapt = ap->adapt != 0;
  // adaptive damping: the residual of the state in u into the free ping-pong
  // buffer, then the Rayleigh-quotient sums
  const auto rq_pass = [=](hipStream_t st) {
    if (c->physics == PETTO_ELASTIC) {
      ElSweep<T> a{};
      a.uin = uu;
      a.v = ua;
      a.E = E;
      a.b = b;
      if (c->ndim == 2) launch_el2d<T, kResid>(c->geom, a, st);
      else launch_el3d<T, kResid>(c->geom, a, st);
    } else {
      HeatSweep<T> a{};
      a.uin = uu;
      a.v = ua;
      a.k = E;
      a.b = b;
      a.des = c->d_des;
      a.tiles = c->heat_lists.at(1).tiles;
      a.dir = c->d_dir;
      a.ntile = c->heat_lists.at(1).ntile;
      launch_heat2d<T, kResid>(a, st);
    }
    launch_rq<T, T>(uu, ua, c->F64, c->d_srange, c->nprob, c->rq_blocks, c->prq, st);
  };
  if (adapt) {
    // a warm start begins at the damping of its own state (a state of zeros
    // keeps the floor); the checks re-choose it after every block
    rq_pass(s);
    launch_adapt(c->st, c->prq, c->rq_blocks, c->nprob, s);
    HIP_TRY(hipGetLastError());
  }
  std::function<void(hipStream_t)> body = [=](hipStream_t st) {
    const int* tile0 = nullptr;
    int nt = 0;
    if (c->physics == PETTO_ELASTIC) {
      nt = elastic_sweeps<T>(c, st, uu, ua, vv, E, b, c->st, nchk, true);
    } else {
      const TileList* L = heat_sweeps<T>(c, st, uu, ua, vv, E, b, c->st, nchk, true);
      tile0 = L->tile0;
      nt = L->ntile;
    }
    if (adapt) rq_pass(st);
    finalize(c, st, c->st, tile0, nt, 0, adapt);
  };
  std::vector<const void*> key = {uu, ua, vv, E, b, (const void*)(long)nchk, (const void*)(long)sizeof(T),
                                  (const void*)1, (const void*)(long)block_k(c, nchk), (const void*)(long)adapt};
  PollRecord last{};
  // the finalize of the last block marks the stop at max_iter (replay: exactly there)
  const long max_blocks = replay ? ap->replay_iters / nchk : ((long)ap->max_iter + nchk - 1) / nchk;
  // a fixed count whose caller wants no report runs without the host (unless the
  // sweep blocks are being timed)
  const bool detached = replay && info == nullptr && !c->timing;
  PETTO_TRY(run_blocks(c, s, ap->use_graph != 0, key, body, nchk, detached ? nullptr : &last, max_blocks));
  if (detached) return PETTO_OK;
  std::vector<SolveState> h;
  PETTO_TRY(read_states(c, c->st, h, s));
  if (info) {
    for (int d = 0; d < c->nprob; ++d) {
      info[d].iters = h[d].iters;
      info[d].status = h[d].status == -3 ? PETTO_ERR_DIVERGED : h[d].status == 1 ? PETTO_NOT_CONVERGED : PETTO_OK;
      info[d].outer = 0;
      info[d].rel_res = h[d].rho;
      info[d].r_pde = h[d].r_pde;
      info[d].dt = h[d].dt;
      info[d].theta = h[d].theta;
    }
  }
  return status_of(h);
}

// FP32 sweeps on a correction d of a double state u.  Each block: fold the
// correction into u (u += d, d = 0), form r = F - K u in double (rounded to float
// as the sweeps' right-hand side), check ||r|| / ||F|| against tol, then run
// check_every FP32 sweeps on K d = r with the velocity carried over.  In exact
// arithmetic the pair (u + d, v) follows the plain iteration.
petto_status solve_refine(petto_ctx* c, const void* phi, void* u, void* v, const petto_apt_params* ap,
                          hipStream_t s, petto_solve_info* info, bool material_ready) {
  if (!material_ready) PETTO_TRY(material<float>(c, phi, s, true));
  PETTO_TRY(setup(c, s, c->st, ap, ap->tol, 0, ap->max_iter));
  PETTO_TRY(ensure_tuning<float>(c, s, ap->check_every));
  double* u64 = static_cast<double*>(u);
  float* v32 = static_cast<float*>(v);
  float* da = c->d32a;
  float* db = c->d32b;
  launch_fill<float>(v32, c->nstate, 0.f, s);
  launch_fill<float>(da, c->nstate, 0.f, s);
  HIP_TRY(hipGetLastError());
  const int nchk = ap->check_every;
  const float* E = static_cast<const float*>(c->E);
  const float* b = c->b32;
  const bool adapt = ap->adapt != 0;
  std::function<void(hipStream_t)> body = [=](hipStream_t st) {
    launch_fold(u64, da, c->nstate, c->ctl + 1, st);
    if (c->physics == PETTO_ELASTIC) {
      ElSweep<double> a{};
      a.uin = u64;
      a.E = c->E64;
      a.b = c->F64;
      a.st = c->st;
      a.partial = c->partial;
      a.b32 = c->b32;
      if (c->ndim == 2) launch_el2d<double, kRefine>(c->geom, a, st);
      else launch_el3d<double, kRefine>(c->geom, a, st);
    } else {
      HeatSweep<double> a{};
      a.uin = u64;
      a.k = c->E64;
      a.b = c->F64;
      a.des = c->d_des;
      a.tiles = c->heat_lists.at(1).tiles;
      a.dir = c->d_dir;
      a.st = c->st;
      a.all_done = c->ctl + 1;
      a.partial = c->partial;
      a.b32 = c->b32;
      a.ntile = c->heat_lists.at(1).ntile;
      launch_heat2d<double, kRefine>(a, st);
    }
    if (adapt) launch_rq<double, float>(u64, c->b32, c->F64, c->d_srange, c->nprob, c->rq_blocks, c->prq, st);
    if (c->physics == PETTO_ELASTIC) finalize(c, st, c->st, nullptr, el_tiles_for(c, true), 1, adapt);
    else finalize(c, st, c->st, c->heat_lists.at(1).tile0, c->heat_lists.at(1).ntile, 1, adapt);
    if (c->physics == PETTO_ELASTIC) elastic_sweeps<float>(c, st, da, db, v32, E, b, c->st, nchk);
    else heat_sweeps<float>(c, st, da, db, v32, E, b, c->st, nchk);
  };
  std::vector<const void*> key = {u64, da, db, v32, E, b, (const void*)(long)nchk, (const void*)2,
                                  (const void*)(long)block_k(c, nchk), (const void*)(long)adapt};
  PollRecord last{};
  // a block checks the state its predecessors produced: one block more than the
  // sweeps need, for the check that stops at max_iter
  const long max_blocks = ((long)ap->max_iter + nchk - 1) / nchk + 1;
  // tol = 0 (a fixed-count stage) never stops early: with no report wanted, the
  // host need not follow it
  const bool detached = !(ap->tol > 0.0) && info == nullptr && !c->timing;
  PETTO_TRY(run_blocks(c, s, ap->use_graph != 0, key, body, nchk, detached ? nullptr : &last, max_blocks));
  if (detached) return PETTO_OK;
  std::vector<SolveState> h;
  PETTO_TRY(read_states(c, c->st, h, s));
  if (info) {
    for (int d = 0; d < c->nprob; ++d) {
      info[d].iters = h[d].iters;
      info[d].status = h[d].status == -3 ? PETTO_ERR_DIVERGED : h[d].status == 1 ? PETTO_NOT_CONVERGED : PETTO_OK;
      info[d].outer = h[d].checks;
      info[d].rel_res = h[d].rho;
      info[d].r_pde = h[d].r_pde;
      info[d].dt = h[d].dt;
      info[d].theta = h[d].theta;
    }
  }
  return status_of(h);
}

// Returns the partial-sum slots written (elastic; heat uses the design ranges).
template <typename U, typename T>
int adjoint_launch(petto_ctx* c, const void* phi, const void* u, const void* w, void* grad, double* pfu, double* pen,
                   hipStream_t s) {
  const petto_problem& p = c->probs[0];
  if (c->physics == PETTO_ELASTIC) {
    ElAdjoint<U, T> a{};
    a.u = static_cast<const U*>(u);
    a.w = static_cast<const U*>(w ? w : u);
    a.phi = static_cast<const T*>(phi);
    a.grad = static_cast<T*>(grad);
    a.F = c->F64;
    a.partial_fu = pfu;
    a.partial_en = pen;
    a.nphase = c->nphase;
    a.e0 = p.e0;
    a.emin = p.emin;
    a.p = p.p;
    for (int m = 0; m <= kMaxPhase; ++m) a.ep[m] = p.e_phase[m];
    return c->ndim == 2 ? launch_el2d_adjoint<U, T>(c->geom, a, s) : launch_el3d_adjoint<U, T>(c->geom, a, s);
  } else {
    HeatAdjoint<U, T> a{};
    a.u = static_cast<const U*>(u);
    a.w = static_cast<const U*>(w ? w : u);
    a.phi = static_cast<const T*>(phi);
    a.grad = static_cast<T*>(grad);
    a.F = c->F64;
    a.des = c->d_des;
    a.tiles = c->heat_lists.at(1).tiles;
    a.dir = c->d_dir;
    a.partial_fu = pfu;
    a.partial_en = pen;
    a.e0 = p.e0;
    a.emin = p.emin;
    a.p = p.p;
    a.ntile = c->heat_lists.at(1).ntile;
    launch_heat2d_adjoint<U, T>(a, s);
    return 0;
  }
}

// Partial-sum slots the sensitivity launch writes (one per workgroup; heat: one
// per tile of the one-sweep work list).
int adjoint_slots(const petto_ctx* c) {
  if (c->physics == PETTO_HEAT) return c->heat_lists.at(1).ntile;
  return c->ndim == 2 ? el2d_tiles(c->geom) : el3d_adjoint_tiles(c->geom);
}

// The sensitivity launch and the fixed-order compliance sums, with the partial
// sums in pfu / pen (each at least adjoint_slots(c) doubles).
petto_status adjoint_run(petto_ctx* c, const void* phi, const void* u, const void* w, int32_t state_fp64,
                         void* grad, double* compliance, double* pfu, double* pen, hipStream_t s) {
  int nt = 0;
  if (c->prec == PETTO_FP64) nt = adjoint_launch<double, double>(c, phi, u, w, grad, pfu, pen, s);
  else if (state_fp64) nt = adjoint_launch<double, float>(c, phi, u, w, grad, pfu, pen, s);
  else nt = adjoint_launch<float, float>(c, phi, u, w, grad, pfu, pen, s);
  launch_dot_finalize(pfu, pen, c->physics == PETTO_HEAT ? c->d_tile0 : nullptr, nt, c->nprob,
                      compliance ? compliance : c->comp, s);
  HIP_TRY(hipGetLastError());
  return PETTO_OK;
}

template <typename T>
petto_status phase_update_impl(petto_ctx* c, void* phi, const void* grad, const petto_phase_params* pp,
                               hipStream_t s, petto_phase_info* info) {
  T* ph = static_cast<T*>(phi);
  const T* g = static_cast<const T*>(grad);
  const int passes = pp->bisect_passes > 0 ? pp->bisect_passes : 9;
  if (pp->model == PETTO_UPDATE_PENALTY_CH) {
    // every stored phase of a design per launch: totals, phi' and mu per phase into
    // the work buffer, then the Cahn-Hilliard step in place
    if (c->pen_work == nullptr) PETTO_TRY(dalloc_t(c, &c->pen_work, (size_t)2 * c->nphase * c->max_cells));
    for (int d = 0; d < c->nprob; ++d) {
      const CellRange& R = c->h_ranges[d];
      const double h = R.h;
      PenaltyArgs<T> a{};
      a.phi = ph + R.off;
      a.g = g + R.off;
      a.pstride = c->ncell;
      a.nphase = c->nphase;
      a.p1 = c->pen_work;
      a.mu = c->pen_work + (long)c->nphase * c->max_cells;
      a.mstride = c->max_cells;
      a.partial = c->phase_partial;
      a.scal = c->phase_scal + (long)kMaxPhase * d * 8;
      a.nx = R.nx;
      a.ny = R.ny;
      a.nz = R.nz;
      a.ndim = c->ndim;
      a.n = R.n;
      a.h = h;
      a.alpha = pp->alpha_h;
      a.gamma = pp->gamma;
      a.alpha_v = pp->alpha_v;
      a.alpha_1 = pp->alpha_1;
      for (int m = 0; m < kMaxPhase; ++m) a.vol_frac[m] = pp->vol_frac[m];
      a.mobility = pp->mobility > 0.0 ? pp->mobility : 1.0;
      if (pp->dt_ch > 0.0) {
        a.dt_ch = pp->dt_ch;
      } else {
        // the printed 500 h^4, capped at 0.9 of the explicit step's stability
        // limit 2 / (D lam (pi^2/32 + gamma lam)), lam = 4 d / h^2
        const double pi = 3.141592653589793;
        const double lam = 4.0 * c->ndim / (h * h);
        const double limit = 2.0 / (a.mobility * lam * (pi * pi / 32.0 + pp->gamma * lam));
        a.dt_ch = std::fmin(500.0 * h * h * h * h, 0.9 * limit);
      }
      a.region = c->d_region != nullptr ? c->d_region + R.off : nullptr;
      a.alpha_b = pp->alpha_b;
      a.nblocks = phase_blocks(R.n);
      launch_penalty_update<T>(a, s);
      HIP_TRY(hipGetLastError());
    }
  } else {
  if (c->nphase > 1 && c->phase_used == nullptr) PETTO_TRY(dalloc_t(c, &c->phase_used, c->max_cells));
  for (int d = 0; d < c->nprob; ++d) {
    const CellRange& R = c->h_ranges[d];
    const double h = R.h;
    double dt_ac = pp->dt_ac;
    if (!(dt_ac > 0.0)) {
      const double pi = 3.141592653589793;
      dt_ac = pp->gamma > 0.0 ? 0.9 * std::fmin(h * h / (4.0 * c->ndim * pp->gamma), 32.0 / (pi * pi))
                              : 0.9 * 32.0 / (pi * pi);
    }
    for (int m = 0; m < c->nphase; ++m) {
      PhaseArgs<T> a{};
      a.phi = ph + (long)m * c->ncell + R.off;
      a.g = g + (long)m * c->ncell + R.off;
      // later phases are bounded by what the earlier ones (already updated) leave
      a.used = m == 0 ? nullptr : c->phase_used;
      a.used_out = m + 1 < c->nphase ? c->phase_used : nullptr;
      a.work = c->phase_work;
      a.partial = c->phase_partial;
      a.scal = c->phase_scal + (long)(kMaxPhase * d + m) * 8;
      a.nx = R.nx;
      a.ny = R.ny;
      a.nz = R.nz;
      a.ndim = c->ndim;
      a.n = R.n;
      a.h = h;
      a.alpha = pp->alpha_h;
      a.gamma = pp->gamma;
      a.dt_ac = dt_ac;
      a.target = pp->vol_frac[m] * (double)R.n;
      a.region = c->d_region != nullptr ? c->d_region + R.off : nullptr;
      a.first = m == 0;
      a.nblocks = phase_blocks(R.n);
      launch_phase_gmax<T>(a, s);
      launch_phase_step<T>(a, s);
      for (int q = 0; q < passes; ++q) launch_phase_pass<T>(a, s);
      launch_phase_apply<T>(a, s);
      HIP_TRY(hipGetLastError());
    }
  }
  }
  if (info) {
    std::vector<double> sc((size_t)c->nprob * kMaxPhase * 8);
    HIP_TRY(hipMemcpyAsync(sc.data(), c->phase_scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int d = 0; d < c->nprob; ++d) {
      for (int m = 0; m < kMaxPhase; ++m) {
        const double* q = sc.data() + (kMaxPhase * d + m) * 8;
        info[d].gmax[m] = m < c->nphase ? q[0] : 0.0;
        info[d].shift[m] = m < c->nphase ? q[3] : 0.0;
        info[d].volume[m] = m < c->nphase ? q[4] : 0.0;
      }
    }
  }
  return PETTO_OK;
}

}  // namespace

// ====================================================================================== C ABI

extern "C" {

const char* petto_last_error(void) { return g_err.c_str(); }

const char* petto_version(void) { return "petto-mi355x 0.1 (gfx950)"; }

petto_status petto_create(const petto_problem* probs, int32_t nprob, int32_t prec, petto_ctx** out) {
  g_err.clear();
  if (out == nullptr) return fail(PETTO_ERR_INVALID, "out is NULL");
  *out = nullptr;
  if (probs == nullptr) return fail(PETTO_ERR_INVALID, "probs is NULL");
  if (nprob < 1 || nprob > kMaxDesigns) return fail(PETTO_ERR_INVALID, "nprob must be in [1, %d]", kMaxDesigns);
  if (prec != PETTO_FP32 && prec != PETTO_FP64) return fail(PETTO_ERR_INVALID, "prec must be PETTO_FP32 or PETTO_FP64");
  for (int d = 0; d < nprob; ++d) {
    PETTO_TRY(validate_problem(probs[d], d));
    if (probs[d].physics != probs[0].physics || probs[d].ndim != probs[0].ndim || probs[d].nphase != probs[0].nphase)
      return fail(PETTO_ERR_INVALID, "all designs of a batch need the same physics, ndim and nphase");
    if (probs[d].physics == PETTO_HEAT) PETTO_TRY(check_heat_mask(probs[d], d));
  }
  if (probs[0].physics == PETTO_ELASTIC && nprob != 1)
    return fail(PETTO_ERR_UNSUPPORTED, "elastic contexts hold one design");
  if (probs[0].physics == PETTO_HEAT && probs[0].ndim != 2)
    return fail(PETTO_ERR_UNSUPPORTED, "heat conduction is implemented in 2D");

  petto_ctx* c = new petto_ctx();
  c->physics = probs[0].physics;
  c->ndim = probs[0].ndim;
  c->prec = prec;
  c->nprob = nprob;
  c->nphase = probs[0].nphase;
  c->probs.assign(probs, probs + nprob);
  // host-side preparation (no GPU yet)
  std::vector<uint32_t> pin_words;
  bool any_pin = false;
  std::vector<double> F;
  if (c->physics == PETTO_ELASTIC) {
    petto_status st = prepare_elastic(c, probs[0], pin_words, any_pin, F);
    if (st < 0) {
      delete c;
      return st;
    }
    const petto_problem& p = probs[0];
    c->nstate = padded_state(p);
    c->ncell = cells(p);
    c->max_cells = c->ncell;
    c->state_off = {0, c->nstate};
    c->cell_off = {0, c->ncell};
    ElGeom& g = c->geom;
    g.nx = p.n[0];
    g.ny = p.n[1];
    g.nz = p.ndim == 3 ? p.n[2] : 1;
    g.px = g.nx + 1;
    g.py = g.ny + 1;
    g.plane = (long)g.px * g.py * (p.ndim == 3 ? g.nz + 1 : 1);
    g.h = p.h;
    g.lam0 = p.nu / ((1.0 + p.nu) * (1.0 - 2.0 * p.nu));
    g.mu0 = 1.0 / (2.0 * (1.0 + p.nu));
    for (int s = 0; s < 6; ++s) {
      const int sd = s < 2 * p.ndim ? p.side[s] : PETTO_SIDE_FREE;
      g.clamp[s] = sd == PETTO_SIDE_CLAMPED;
      g.fixn[s] = sd != PETTO_SIDE_FREE;
    }
    c->m0 = g.lam0 + 2.0 * g.mu0;
    c->h_ranges.push_back({0, c->ncell, g.nx, g.ny, g.nz, 0, p.h});
    // partial-sum slots: every sweep tiling, and the sensitivity launch (whose 3D
    // tiling is its own)
    c->ntile = c->ndim == 2 ? el2d_tiles(g) : std::max(el3d_tiles(g), el3d_adjoint_tiles(g));
    if (c->ndim == 2)
      for (int k : {2, 4, 5, 8, 10}) c->ntile = std::max(c->ntile, el2d_tb_tiles(g, k));
  } else {
    long soff = 0;
    int t0 = 0;
    std::vector<HeatTile> tiles;
    std::vector<int> tile0;
    std::vector<uint8_t> dir;
    F.clear();
    bool dense = false;
    for (int d = 0; d < nprob; ++d) dense = dense || probs[d].load != nullptr;
    for (int d = 0; d < nprob; ++d) {
      const petto_problem& p = probs[d];
      const int nx = p.n[0], ny = p.n[1];
      const long n = (long)nx * ny;
      HeatDesign hd{};
      hd.nx = nx;
      hd.ny = ny;
      hd.off = soff;
      hd.tile0 = t0;
      hd.dir_off = (int)dir.size();
      hd.h = p.h;
      hd.fsrc = p.q * p.h * p.h;
      for (int j = 0; j < ny; ++j) dir.push_back(p.fixed[(long)j * nx] & 1);
      for (int j = 0; j < ny; ++j) dir.push_back((p.fixed[(long)j * nx + nx - 1] >> 1) & 1);
      for (int i = 0; i < nx; ++i) dir.push_back((p.fixed[i] >> 2) & 1);
      for (int i = 0; i < nx; ++i) dir.push_back((p.fixed[(long)(ny - 1) * nx + i] >> 3) & 1);
      tile0.push_back(t0);
      for (int j0 = 0; j0 < ny; j0 += 8)
        for (int i0 = 0; i0 < nx; i0 += 64) tiles.push_back({d, i0, j0, 0});
      hd.ntile = (int)tiles.size() - t0;
      t0 = (int)tiles.size();
      double ss = 0.0;
      if (dense) {
        for (long q = 0; q < n; ++q) {
          const double v = p.load ? p.load[q] : hd.fsrc;
          if (!is_finite(v)) {
            delete c;
            return fail(PETTO_ERR_INVALID, "problem %d: source not finite", d);
          }
          F.push_back(v);
          ss += v * v;
        }
      } else {
        ss = hd.fsrc * hd.fsrc * (double)n;
      }
      if (!(ss > 0.0)) {
        delete c;
        return fail(PETTO_ERR_INVALID, "problem %d: source is zero", d);
      }
      c->fnorm.push_back(std::sqrt(ss));
      c->h_des.push_back(hd);
      c->h_ranges.push_back({soff, n, nx, ny, 1, 0, p.h});
      c->state_off.push_back(soff);
      c->cell_off.push_back(soff);
      soff += n;
      if (n > c->max_cells) c->max_cells = n;
    }
    tile0.push_back(t0);
    c->state_off.push_back(soff);
    c->cell_off.push_back(soff);
    c->nstate = soff;
    c->ncell = soff;
    c->ntile = t0;
    c->m0 = 1.0;
    // device copies; work lists for one sweep per launch (64 x 8 tiles) and for
    // every multi-sweep choice ((64-2K) x (32-2K) inner blocks)
    auto up = [&]() -> petto_status {
      PETTO_TRY(upload(c, &c->d_des, c->h_des));
      PETTO_TRY(upload(c, &c->d_tiles, tiles));
      PETTO_TRY(upload(c, &c->d_dir, dir));
      PETTO_TRY(upload(c, &c->d_tile0, tile0));
      c->heat_lists[1] = TileList{c->d_tiles, c->d_tile0, t0};
      std::vector<int> ks = {2, 4, 5};
      if (prec == PETTO_FP32) ks.insert(ks.end(), {8, 10});
      for (int k : ks) {
        const int txi = 64 - 2 * k, tyi = 32 - 2 * k;
        std::vector<HeatTile> tl;
        std::vector<int> t0k;
        for (int d = 0; d < nprob; ++d) {
          t0k.push_back((int)tl.size());
          for (int j0 = 0; j0 < probs[d].n[1]; j0 += tyi)
            for (int i0 = 0; i0 < probs[d].n[0]; i0 += txi) tl.push_back({d, i0, j0, 0});
        }
        t0k.push_back((int)tl.size());
        TileList L;
        L.ntile = (int)tl.size();
        PETTO_TRY(upload(c, &L.tiles, tl));
        PETTO_TRY(upload(c, &L.tile0, t0k));
        c->heat_lists[k] = L;
        c->ntile = std::max(c->ntile, L.ntile);
      }
      return PETTO_OK;
    };
    petto_status st = up();
    if (st < 0) {
      petto_destroy(c);
      return st;
    }
  }
  auto build = [&]() -> petto_status {
    // set-up of the allocation-free sensitivity entry point on this GPU
    PETTO_TRY(scratch_resolve());
    const size_t es = elem_size(c);
    if (!F.empty()) {
      PETTO_TRY(upload(c, &c->F64, F));
      PETTO_TRY(dalloc(c, &c->Ft, F.size() * es));
      if (prec == PETTO_FP64) {
        HIP_TRY(hipMemcpy(c->Ft, F.data(), F.size() * es, hipMemcpyHostToDevice));
      } else {
        std::vector<float> f32(F.begin(), F.end());
        HIP_TRY(hipMemcpy(c->Ft, f32.data(), F.size() * es, hipMemcpyHostToDevice));
      }
    }
    if (any_pin) PETTO_TRY(upload(c, &c->pins, pin_words));
    c->geom.pins = c->pins;
    c->geom.tile3d = 1;
    if (c->physics == PETTO_ELASTIC && c->ndim == 3) {
      int dev = 0;
      HIP_TRY(hipGetDevice(&dev));
      HIP_TRY(hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, dev));
      c->geom.tile3d = el3d_choose_tiling(c->geom, prec == PETTO_FP64, c->ncu);
    }
    std::vector<long> nc;
    std::vector<double> hh;
    for (const auto& r : c->h_ranges) {
      nc.push_back(r.n);
      hh.push_back(r.h);
    }
    PETTO_TRY(upload(c, &c->d_ranges, c->h_ranges));
    // cell roles, concatenated like the cell arrays (only when a design has them)
    bool any_region = false;
    for (int d = 0; d < nprob; ++d) any_region = any_region || probs[d].region != nullptr;
    if (any_region) {
      std::vector<uint8_t> reg((size_t)c->ncell, 0);
      for (int d = 0; d < nprob; ++d)
        if (probs[d].region != nullptr)
          std::copy(probs[d].region, probs[d].region + c->h_ranges[d].n, reg.begin() + c->h_ranges[d].off);
      PETTO_TRY(upload(c, &c->d_region, reg));
    }
    PETTO_TRY(upload(c, &c->d_ncell, nc));
    PETTO_TRY(upload(c, &c->d_fnorm, c->fnorm));
    PETTO_TRY(upload(c, &c->d_h, hh));
    std::vector<StateRange> sr;
    if (c->physics == PETTO_ELASTIC) sr.push_back({0, c->nstate, 0.0});
    else
      for (int d = 0; d < nprob; ++d) sr.push_back({c->h_des[d].off, (long)c->h_des[d].nx * c->h_des[d].ny,
                                                    c->h_des[d].fsrc});
    PETTO_TRY(upload(c, &c->d_srange, sr));
    long maxn = 0;
    for (const StateRange& r : sr) maxn = std::max(maxn, r.n);
    const long rqb = (maxn + kRqPerBlock - 1) / kRqPerBlock;
    c->rq_blocks = (int)std::min<long>(kRqBlocksMax, std::max<long>(kRqBlocksMin, rqb));
    PETTO_TRY(dalloc_t(c, &c->prq, (size_t)nprob * c->rq_blocks * 3));
    PETTO_TRY(dalloc(c, &c->ualt, c->nstate * es));
    PETTO_TRY(dalloc(c, &c->valt, c->nstate * es));
    PETTO_TRY(dalloc(c, &c->E, c->ncell * es));
    if (prec == PETTO_FP32) {
      PETTO_TRY(dalloc_t(c, &c->E64, c->ncell));
      PETTO_TRY(dalloc_t(c, &c->d32a, c->nstate));
      PETTO_TRY(dalloc_t(c, &c->d32b, c->nstate));
      PETTO_TRY(dalloc_t(c, &c->b32, c->nstate));
    } else {
      PETTO_TRY(dalloc(c, &c->tune_a, c->nstate * es));
      PETTO_TRY(dalloc(c, &c->tune_b, c->nstate * es));
      PETTO_TRY(dalloc(c, &c->tune_c, c->nstate * es));
    }
    PETTO_TRY(dalloc_t(c, &c->partial, c->ntile + 64));
    PETTO_TRY(dalloc_t(c, &c->partial2, c->ntile + 64));
    PETTO_TRY(dalloc_t(c, &c->partial_max, (size_t)kBpd * nprob));
    PETTO_TRY(dalloc_t(c, &c->st, nprob));
    PETTO_TRY(dalloc_t(c, &c->ctl, 4));
    HIP_TRY(hipMemset(c->ctl, 0, 4 * sizeof(int)));
    HIP_TRY(hipMemset(c->st, 0, nprob * sizeof(SolveState)));
    void* ring = nullptr;
    HIP_TRY(hipHostMalloc(&ring, sizeof(PollRecord) * kRing, hipHostMallocMapped));
    c->ring_host = static_cast<PollRecord*>(ring);
    for (int i = 0; i < kRing; ++i) c->ring_host[i] = {0, 0, 0, -1};
    void* rd = nullptr;
    HIP_TRY(hipHostGetDevicePointer(&rd, ring, 0));
    c->ring_dev = static_cast<PollRecord*>(rd);
    PETTO_TRY(dalloc_t(c, &c->phase_scal, (size_t)nprob * kMaxPhase * 8));
    PETTO_TRY(dalloc_t(c, &c->phase_work, c->max_cells));
    PETTO_TRY(dalloc_t(c, &c->phase_partial, (size_t)phase_blocks(c->max_cells) * (kCand + 1) + 64));
    PETTO_TRY(dalloc_t(c, &c->comp, (size_t)2 * nprob));
    return PETTO_OK;
  };
  petto_status st = build();
  if (st < 0) {
    petto_destroy(c);
    return st;
  }
  c->blocking = 0;
  *out = c;
  return PETTO_OK;
}

petto_status petto_destroy(petto_ctx* ctx) {
  if (ctx == nullptr) return PETTO_OK;
  destroy_graphs(ctx);
  if (ctx->events) {
    for (int i = 0; i < kRing; ++i) {
      (void)hipEventDestroy(ctx->ev_end[i]);
      (void)hipEventDestroy(ctx->ev_beg[i]);
    }
  }
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  for (void* p : ctx->allocations) (void)hipFree(p);
  if (ctx->ring_host) (void)hipHostFree(ctx->ring_host);
  delete ctx;
  return PETTO_OK;
}

size_t petto_field_offset(const petto_ctx* ctx, int32_t iprob, int32_t field) {
  if (ctx == nullptr || iprob < 0 || iprob > ctx->nprob) return (size_t)-1;
  if (field == PETTO_FIELD_STATE) return (size_t)ctx->state_off[iprob];
  if (field == PETTO_FIELD_CELL) return (size_t)ctx->cell_off[iprob];
  return (size_t)-1;
}

petto_status petto_set_timing(petto_ctx* ctx, int32_t on) {
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  ctx->timing = on != 0;
  ctx->timed_ms = 0.0;
  ctx->timed_sweeps = 0;
  return PETTO_OK;
}

double petto_last_sweep_ms(const petto_ctx* ctx, int64_t* sweeps) {
  if (ctx == nullptr || ctx->timed_sweeps == 0) {
    if (sweeps) *sweeps = 0;
    return 0.0;
  }
  if (sweeps) *sweeps = ctx->timed_sweeps;
  return ctx->timed_ms / (double)ctx->timed_sweeps;
}

petto_status petto_set_blocking(petto_ctx* ctx, int32_t k) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  const bool ok = k == 0 || k == 1 || k == 2 || k == 4 || k == 5 || (ctx->prec == PETTO_FP32 && (k == 8 || k == 10));
  if (!ok) return fail(PETTO_ERR_INVALID, "unsupported sweeps per launch %d", k);
  ctx->blocking = k;
  destroy_graphs(ctx);
  return PETTO_OK;
}

int32_t petto_blocking(const petto_ctx* ctx) { return ctx ? ctx->blocking : 0; }

petto_status petto_time_sweeps(petto_ctx* ctx, int32_t launches, void* stream, double* ms_per_launch,
                               int32_t* sweeps_per_launch) {
  g_err.clear();
  if (ctx == nullptr || ms_per_launch == nullptr || sweeps_per_launch == nullptr)
    return fail(PETTO_ERR_INVALID, "ctx and outputs must not be NULL");
  if (launches < 2 || launches > 100000) return fail(PETTO_ERR_INVALID, "launches must be in [2, 100000]");
  if (ctx->prec != PETTO_FP32) return fail(PETTO_ERR_UNSUPPORTED, "sweep timing is for FP32 contexts");
  petto_ctx* c = ctx;
  hipStream_t s = static_cast<hipStream_t>(stream);
  PETTO_TRY(ensure_events(c));
  if (c->st_t == nullptr) PETTO_TRY(dalloc_t(c, &c->st_t, c->nprob));
  // the coefficients of the last solve, with the stop flags cleared
  std::vector<SolveState> hs(c->nprob);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(hs.data(), c->st, c->nprob * sizeof(SolveState), hipMemcpyDeviceToHost));
  for (auto& x : hs) x.done = 0;
  HIP_TRY(hipMemcpy(c->st_t, hs.data(), c->nprob * sizeof(SolveState), hipMemcpyHostToDevice));
  float* u = c->d32a;
  float* ua = c->d32b;
  float* v = static_cast<float*>(c->ualt);
  launch_fill<float>(u, c->nstate, 0.f, s);
  launch_fill<float>(v, c->nstate, 0.f, s);
  launch_fill<float>(c->b32, c->nstate, 0.f, s);
  const float* E = static_cast<const float*>(c->E);
  const int k = c->physics == PETTO_ELASTIC && c->ndim == 3 ? 1 : (c->blocking > 0 ? c->blocking : 1);
  const int n = launches + (launches & 1);           // even: the state ends where it began
  auto run = [&](int nl) {
    if (c->physics == PETTO_ELASTIC) elastic_sweeps<float>(c, s, u, ua, v, E, c->b32, c->st_t, nl * k);
    else heat_sweeps<float>(c, s, u, ua, v, E, nullptr, c->st_t, nl * k, false, c->ctl + 2);
  };
  run(2);
  HIP_TRY(hipEventRecord(c->ev_beg[0], s));
  run(n);
  HIP_TRY(hipEventRecord(c->ev_end[0], s));
  HIP_TRY(hipEventSynchronize(c->ev_end[0]));
  HIP_TRY(hipGetLastError());
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev_beg[0], c->ev_end[0]));
  *ms_per_launch = ms / (double)n;
  *sweeps_per_launch = k;
  return PETTO_OK;
}

petto_status petto_set_tile3d(petto_ctx* ctx, int32_t t) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (ctx->physics != PETTO_ELASTIC || ctx->ndim != 3)
    return fail(PETTO_ERR_INVALID, "the 3D tiling applies to 3D elastic contexts");
  if (t < 0 || t > 3) return fail(PETTO_ERR_INVALID, "unsupported 3D tiling %d", t);
  ctx->tuned3d = t != 0;
  if (t == 0) t = el3d_choose_tiling(ctx->geom, ctx->prec == PETTO_FP64, ctx->ncu);
  ctx->geom.tile3d = t;
  destroy_graphs(ctx);
  return PETTO_OK;
}

int32_t petto_tile3d(const petto_ctx* ctx) { return ctx ? ctx->geom.tile3d : 0; }

petto_status petto_apt_solve(petto_ctx* ctx, const void* phi, void* u, void* v, const petto_apt_params* params,
                             void* stream, petto_solve_info* info) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (phi == nullptr || u == nullptr || v == nullptr) return fail(PETTO_ERR_INVALID, "phi, u and v must be non-NULL");
  PETTO_TRY(check_apt_params(ctx, params));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->timing) {
    ctx->timed_ms = 0.0;
    ctx->timed_sweeps = 0;
  }
  // (the second stage runs on the moduli the first one formed from the same design)
  auto stage = [&](const petto_apt_params* p, petto_solve_info* inf, bool ready) -> petto_status {
    if (p->refine) return solve_refine(ctx, phi, u, v, p, s, inf, ready);
    if (ctx->prec == PETTO_FP64) return solve_plain<double>(ctx, phi, u, v, p, s, inf, ready);
    return solve_plain<float>(ctx, phi, u, v, p, s, inf, ready);
  };
  const petto_status s1 = stage(params, info, false);
  if (s1 < 0 || params->n_pt == 0) return s1;
  // the hybrid schedule's second stage: n_pt plain PT sweeps (theta = 0: the
  // velocity plays no part), a fixed count without the stop rule
  petto_apt_params q = *params;
  q.theta = 0.0;
  q.dt = params->dt_pt;
  q.adapt = 0;
  q.n_pt = 0;
  q.check_every = (params->n_pt % params->check_every == 0) ? params->check_every : params->n_pt;
  if (params->refine) {
    q.tol = 0.0;                      // never met: the stage ends at max_iter
    q.max_iter = params->n_pt;
    q.replay_iters = 0;
  } else {
    q.replay_iters = params->n_pt;
    q.max_iter = params->n_pt;
  }
  std::vector<petto_solve_info> pt(ctx->nprob);
  const petto_status s2 = stage(&q, info ? pt.data() : nullptr, true);
  if (s2 < 0) return s2;
  if (info) {
    for (int d = 0; d < ctx->nprob; ++d) {
      info[d].iters += pt[d].iters;
      info[d].outer += pt[d].outer;
      info[d].rel_res = pt[d].rel_res;
      info[d].r_pde = pt[d].r_pde;
    }
  }
  return s1;
}

petto_status petto_residual(petto_ctx* ctx, const void* phi, const void* u, void* r, void* stream) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (phi == nullptr || u == nullptr || r == nullptr) return fail(PETTO_ERR_INVALID, "phi, u and r must be non-NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto run = [&](auto tag) -> petto_status {
    using T = decltype(tag);
    PETTO_TRY(material<T>(ctx, phi, s, false));
    if (ctx->physics == PETTO_ELASTIC) {
      ElSweep<T> a{};
      a.uin = static_cast<const T*>(u);
      a.v = static_cast<T*>(r);
      a.E = static_cast<const T*>(ctx->E);
      a.b = static_cast<const T*>(ctx->Ft);
      if (ctx->ndim == 2) launch_el2d<T, kResid>(ctx->geom, a, s);
      else launch_el3d<T, kResid>(ctx->geom, a, s);
    } else {
      HeatSweep<T> a{};
      a.uin = static_cast<const T*>(u);
      a.v = static_cast<T*>(r);
      a.k = static_cast<const T*>(ctx->E);
      a.b = static_cast<const T*>(ctx->Ft);
      a.des = ctx->d_des;
      a.tiles = ctx->heat_lists.at(1).tiles;
      a.dir = ctx->d_dir;
      a.ntile = ctx->heat_lists.at(1).ntile;
      launch_heat2d<T, kResid>(a, s);
    }
    HIP_TRY(hipGetLastError());
    return PETTO_OK;
  };
  if (ctx->prec == PETTO_FP64) return run(double{});
  return run(float{});
}

petto_status petto_adjoint(petto_ctx* ctx, const void* phi, const void* u, const void* w, int32_t state_fp64,
                           void* grad_phi, double* compliance, void* stream) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (phi == nullptr || u == nullptr || grad_phi == nullptr)
    return fail(PETTO_ERR_INVALID, "phi, u and grad_phi must be non-NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int need = adjoint_slots(ctx);
  if (need > ctx->ntile)
    return fail(PETTO_ERR_UNSUPPORTED, "sensitivity launch needs %d partial-sum slots, the context holds %d",
                need, ctx->ntile);
  return adjoint_run(ctx, phi, u, w, state_fp64, grad_phi, compliance, ctx->partial, ctx->partial2, s);
}

petto_status petto_adjoint_noalloc(petto_ctx* ctx, const void* phi, const void* u, const void* w,
                                   int32_t state_fp64, void* grad_phi, double* compliance, void* stream) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (phi == nullptr || u == nullptr || grad_phi == nullptr)
    return fail(PETTO_ERR_INVALID, "phi, u and grad_phi must be non-NULL");
  const int need = adjoint_slots(ctx);
  if (need > kScratchSlots)
    return fail(PETTO_ERR_UNSUPPORTED, "sensitivity launch needs %d partial-sum slots, the fixed scratch holds %d",
                need, kScratchSlots);
  double* sp = nullptr;
  PETTO_TRY(scratch_lookup(&sp));
  return adjoint_run(ctx, phi, u, w, state_fp64, grad_phi, compliance, sp, sp + kScratchSlots,
                     static_cast<hipStream_t>(stream));
}

petto_status petto_phase_update(petto_ctx* ctx, void* phi, const void* grad_phi, const petto_phase_params* pp,
                                void* stream, petto_phase_info* info) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (phi == nullptr || grad_phi == nullptr) return fail(PETTO_ERR_INVALID, "phi and grad_phi must be non-NULL");
  if (pp == nullptr) return fail(PETTO_ERR_INVALID, "phase params are NULL");
  if (!(pp->alpha_h >= 0.0) || !is_finite(pp->alpha_h)) return fail(PETTO_ERR_INVALID, "alpha_h must be >= 0");
  if (!(pp->gamma >= 0.0) || !is_finite(pp->gamma)) return fail(PETTO_ERR_INVALID, "gamma must be >= 0");
  if (!is_finite(pp->dt_ac)) return fail(PETTO_ERR_INVALID, "dt_ac must be finite");
  if (pp->model != PETTO_UPDATE_ALLEN_CAHN && pp->model != PETTO_UPDATE_PENALTY_CH)
    return fail(PETTO_ERR_INVALID, "unknown update model %d", pp->model);
  if (pp->model == PETTO_UPDATE_PENALTY_CH) {
    if (!(pp->alpha_v >= 0.0) || !is_finite(pp->alpha_v) || !(pp->alpha_1 >= 0.0) || !is_finite(pp->alpha_1))
      return fail(PETTO_ERR_INVALID, "alpha_v and alpha_1 must be finite and >= 0");
    if (!is_finite(pp->dt_ch) || !is_finite(pp->mobility))
      return fail(PETTO_ERR_INVALID, "dt_ch and mobility must be finite (<= 0 selects the default)");
    if (!(pp->alpha_b >= 0.0) || !is_finite(pp->alpha_b)) return fail(PETTO_ERR_INVALID, "alpha_b must be >= 0");
  }
  double vs = 0.0;
  for (int m = 0; m < ctx->nphase; ++m) {
    if (!(pp->vol_frac[m] > 0.0 && pp->vol_frac[m] < 1.0))
      return fail(PETTO_ERR_INVALID, "vol_frac[%d] must be in (0, 1)", m);
    vs += pp->vol_frac[m];
  }
  if (!(vs < 1.0 || ctx->nphase == 1)) return fail(PETTO_ERR_INVALID, "phase volume fractions must sum below 1");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (ctx->prec == PETTO_FP64) return phase_update_impl<double>(ctx, phi, grad_phi, pp, s, info);
  return phase_update_impl<float>(ctx, phi, grad_phi, pp, s, info);
}

petto_status petto_step(petto_ctx* ctx, void* phi, void* u, void* v, void* grad_phi, double* compliance,
                        const petto_apt_params* ap, const petto_phase_params* pp, void* stream,
                        petto_solve_info* sinfo, petto_phase_info* pinfo) {
  g_err.clear();
  if (ctx == nullptr) return fail(PETTO_ERR_INVALID, "ctx is NULL");
  if (grad_phi == nullptr) return fail(PETTO_ERR_INVALID, "grad_phi must be non-NULL");
  if (pp == nullptr) return fail(PETTO_ERR_INVALID, "phase params are NULL");
  petto_status s1 = petto_apt_solve(ctx, phi, u, v, ap, stream, sinfo);
  if (s1 < 0) return s1;
  petto_status s2 = petto_adjoint(ctx, phi, u, nullptr, ap->refine ? 1 : 0, grad_phi, compliance, stream);
  if (s2 < 0) return s2;
  petto_status s3 = petto_phase_update(ctx, phi, grad_phi, pp, stream, pinfo);
  if (s3 < 0) return s3;
  return s1;
}

}  // extern "C"
