// xtm_api.cpp -- C ABI of the tracking library (see include/xtm.h).
//
// Host side: validation, packing of the element table (forward and inverse
// direction), per-set work buffers, and the chunk loop that drives the
// gfx950 kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <cstring>
#include <random>
#include <exception>
#include <new>
#include <string>
#include <vector>

#include "../../include/xtm.h"
#include "xtm_internal.h"

namespace {

thread_local std::string g_err;

xtm_status fail(xtm_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

xtm_status hip_fail(hipError_t e, const char* where) {
  return fail(XTM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(expr, where)               \
  do {                                     \
    hipError_t _e = (expr);                \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

constexpr double kClight = 299792458.0;

struct RefQ {
  double mass0, charge0, p0c, beta0, gamma0;
};

bool make_ref(const xtm_reference* r, RefQ* q) {
  if (!r || !(r->mass0_eV > 0.0) || !(r->p0c_eV > 0.0) || !std::isfinite(r->charge0)) return false;
  q->mass0 = r->mass0_eV;
  q->charge0 = r->charge0;
  q->p0c = r->p0c_eV;
  const double e0 = std::sqrt(q->p0c * q->p0c + q->mass0 * q->mass0);
  q->gamma0 = e0 / q->mass0;
  q->beta0 = q->p0c / e0;
  return true;
}

bool same_ref(const RefQ& a, const RefQ& b) {
  return a.mass0 == b.mass0 && a.charge0 == b.charge0 && a.p0c == b.p0c;
}

}  // namespace

// identities of lattices and batches, unique for the life of the process
// (captured graphs are keyed on them, never on a handle's address, which the
// heap may hand to a new lattice after a destroy)
static std::atomic<uint64_t> g_next_id{1};

struct xtm_lattice_s {
  const uint64_t id = g_next_id.fetch_add(1);
  int32_t n_el = 0;
  RefQ ref{};
  std::vector<uint64_t> fwd_h, bwd_h;
  uint64_t* fwd_d = nullptr;
  uint64_t* bwd_d = nullptr;
  // LDS segments of each table: (first word, word count, element count)
  std::vector<int32_t> fwd_seg_h, bwd_seg_h;
  int32_t* fwd_seg_d = nullptr;
  int32_t* bwd_seg_d = nullptr;
  // per-line kernels, compiled on first use: forward ones for each radiation
  // form, backward ones (never radiating)
  bool radiates = false;  // the line holds radiating multipoles
  xtm::LineKernel fwd_line[xtm::kRadForms][xtm::kLineStyles], bwd_line[xtm::kLineStyles];
  // generated recording kernel of optics by tracking, compiled on first use
  xtm::LineKernel rec_line;
  // launch plan chosen by xtm_autotune (0 = none): kernel form and block
  // used when the caller's options leave both at 0, turns per chunk and
  // compaction period when the caller leaves those at 0
  int32_t plan_variant = 0, plan_block = 0, plan_chunk = 0, plan_compact_every = 0;
  // the element descriptions of the sliced line (thick elements replaced by
  // their slices) and the user element of each
  std::vector<xtm_element_desc> desc_h;
  std::vector<int32_t> user_h;
  // loss-refinement geometry for one polygon size, built on first use
  int32_t refine_M = 0;
  void* refine_buf = nullptr;
  xtm::RefineGeom refine{};
};

struct xtm_batch_s {
  const uint64_t id = g_next_id.fetch_add(1);
  std::vector<xtm_lattice_s*> lats;
  int32_t n_el = 0;
  RefQ ref{};
  uint64_t** tabs_d = nullptr;       // forward element table of each variant
  int32_t* first_d = nullptr;        // slot partition (n_variants + 1), device
  std::vector<int64_t> first_h;      // the partition last uploaded
  int32_t plan_block = 0;
  int32_t plan_variant = 0;
  int32_t plan_chunk = 0;
  int32_t plan_compact_every = 0;
  // batched per-line kernels (one-wave forms) for each radiation form, built
  // on first use when every variant has the same element structure
  xtm::LineKernel line[xtm::kRadForms][xtm::kLineStyles];
};

struct GraphKey {
  uint64_t owner;  // lattice or batch id
  int32_t n_turns, chunk, block, variant, backward, compact, compact_every, cur, rad_mode;
  int64_t alive_upper;
  uint64_t seed;
  const float* rec;
  int32_t rec_turns;
  int32_t ramp;
  bool operator==(const GraphKey& o) const {
    return owner == o.owner && n_turns == o.n_turns && chunk == o.chunk && block == o.block &&
           variant == o.variant && backward == o.backward && compact == o.compact &&
           compact_every == o.compact_every && cur == o.cur && rad_mode == o.rad_mode && alive_upper == o.alive_upper &&
           seed == o.seed && rec == o.rec && rec_turns == o.rec_turns && ramp == o.ramp;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec;
  int32_t launches;
};

struct xtm_particles_s {
  std::vector<GraphEntry> graphs;      // captured chunk sequences (use_graph)
  hipStream_t capture_stream = nullptr;
  xtm_arrays a{};
  RefQ ref{};
  int64_t n = 0;
  int32_t turn = 0;
  bool initialised = false;
  int32_t* idx[2] = {nullptr, nullptr};
  int32_t* lost = nullptr;  // particles lost during the last chunk
  int32_t cur = 0;          // which idx buffer holds the alive list
  int32_t* ctrl = nullptr;  // [0] alive count, [2] count scanned by the last epilogue
  int32_t* blockcnt = nullptr;
  int64_t* passes = nullptr;
  int64_t alive_upper = 0;  // host-side upper bound of the alive count
};

namespace {

using namespace xtm;

void put_d(std::vector<uint64_t>& v, double d) {
  uint64_t u;
  std::memcpy(&u, &d, 8);
  v.push_back(u);
}

// Pack one element; sgn = +1 forward map, -1 its exact inverse (parameters
// negated so that the same kernel code applies the inverse).
xtm_status pack(const xtm_element_desc& e, int32_t index, const RefQ& r, double sgn,
                std::vector<uint64_t>& out) {
  auto hdr = [&](uint32_t kt, uint32_t order, uint32_t nw) {
    out.push_back(make_header(kt, order, nw, (uint32_t)index));
  };
  const std::string where = "element " + std::to_string(index) + ": ";
  switch (e.type) {
    case XTM_DRIFT:
    case XTM_DRIFT_EXPANDED:
      if (!std::isfinite(e.length)) return fail(XTM_E_ELEMENT, where + "non-finite drift length");
      if (e.type == XTM_DRIFT) {
        // the length's class for the device's short quotient sequence:
        // 0, |L| in [2^-600, 2^600] and not a power of two (served for every
        // momentum); 1, a power of two in that range (served unless pz has
        // an all-ones significand); 2, any other length, zero included
        // (generic division)
        int ex = 0;
        const double m = std::frexp(std::fabs(e.length), &ex);
        const bool in_range = std::fabs(e.length) >= 0x1p-600 && std::fabs(e.length) <= 0x1p600;
        hdr(K_DRIFT, in_range ? (m != 0.5 ? 0 : 1) : 2, 1);
      } else {
        hdr(K_DRIFT_EXP, 0, 1);
      }
      put_d(out, sgn * e.length);
      return XTM_OK;
    case XTM_MULTIPOLE: {
      if (e.order < 0 || e.order > XTM_MAX_ORDER)
        return fail(XTM_E_ELEMENT, where + "multipole order outside 0..10");
      if (!std::isfinite(e.length)) return fail(XTM_E_ELEMENT, where + "non-finite multipole length");
      const bool curv = (e.hxl != 0.0);
      const bool has_len = e.length > 0.0;  // radiation length
      const uint32_t N = (uint32_t)e.order;
      hdr(curv ? K_MULT_CURV : (has_len ? K_MULT_LR : K_MULT), N,
          2 * (N + 1) + (curv ? 3 : (has_len ? 1 : 0)));
      // c_n = (knl_n + i ksl_n)/n!, stored from the top order down
      double fact[XTM_MAX_ORDER + 1];
      fact[0] = 1.0;
      for (int n = 1; n <= XTM_MAX_ORDER; ++n) fact[n] = fact[n - 1] * (double)n;
      for (int n = (int)N; n >= 0; --n) {
        const double cr = e.knl[n] / fact[n];
        const double ci = e.ksl[n] / fact[n];
        put_d(out, sgn * cr);
        put_d(out, sgn * ci);
      }
      if (curv) {
        put_d(out, sgn * e.hxl);
        put_d(out, sgn * (e.knl[0] * e.hxl));
        put_d(out, e.length);
      } else if (has_len) {
        put_d(out, e.length);
      }
      return XTM_OK;
    }
    case XTM_RF: {
      const double V = e.p[0], f = e.p[1], lag = e.p[2];
      if (!std::isfinite(V) || !std::isfinite(f) || !std::isfinite(lag) || f < 0.0)
        return fail(XTM_E_ELEMENT, where + "RF needs finite V, f >= 0, lag");
      hdr(K_RF, 0, 3);
      const double amp = r.charge0 * V / r.p0c;
      const double k = 2.0 * M_PI * f / (r.beta0 * kClight);
      const double phi = lag * M_PI / 180.0;
      put_d(out, sgn * amp);
      put_d(out, k);
      put_d(out, phi);
      return XTM_OK;
    }
    case XTM_XYSHIFT:
      hdr(K_SHIFT, 0, 2);
      put_d(out, sgn * e.p[0]);
      put_d(out, sgn * e.p[1]);
      return XTM_OK;
    case XTM_SROTATION:
      hdr(K_SROT, 0, 2);
      put_d(out, std::cos(e.p[0]));
      put_d(out, sgn * std::sin(e.p[0]));
      return XTM_OK;
    case XTM_AP_CIRCLE:
      if (!(e.p[0] > 0.0)) return fail(XTM_E_ELEMENT, where + "aperture radius must be > 0");
      hdr(K_AP_CIRC, 0, 1);
      put_d(out, e.p[0] * e.p[0]);
      return XTM_OK;
    case XTM_AP_ELLIPSE:
      if (!(e.p[0] > 0.0) || !(e.p[1] > 0.0))
        return fail(XTM_E_ELEMENT, where + "ellipse half-axes must be > 0");
      hdr(K_AP_ELL, 0, 2);
      put_d(out, 1.0 / (e.p[0] * e.p[0]));
      put_d(out, 1.0 / (e.p[1] * e.p[1]));
      return XTM_OK;
    case XTM_AP_RECT:
      if (!(e.p[0] < e.p[1]) || !(e.p[2] < e.p[3]))
        return fail(XTM_E_ELEMENT, where + "rectangle needs xmin < xmax and ymin < ymax");
      hdr(K_AP_RECT, 0, 4);
      for (int k = 0; k < 4; ++k) put_d(out, e.p[k]);
      return XTM_OK;
    case XTM_MARKER:
      hdr(K_MARKER, 0, 0);
      return XTM_OK;
    default:
      return fail(XTM_E_ELEMENT, where + "unknown element type " + std::to_string(e.type));
  }
}

// Greedy split of a packed table into segments of at most kSegWords words.
std::vector<int32_t> segment(const std::vector<uint64_t>& tab, int32_t n_el) {
  std::vector<int32_t> seg;
  size_t off = 0, start = 0;
  int32_t count = 0;
  for (int32_t e = 0; e < n_el; ++e) {
    const size_t len = 1 + ((tab[off] >> 16) & 0xffffu);
    if (off + len - start > (size_t)kSegWords) {
      seg.push_back((int32_t)start);
      seg.push_back((int32_t)(off - start));
      seg.push_back(count);
      start = off;
      count = 0;
    }
    off += len;
    ++count;
  }
  if (count > 0 || seg.empty()) {
    seg.push_back((int32_t)start);
    seg.push_back((int32_t)(off - start));
    seg.push_back(count);
  }
  return seg;
}

SoA soa_of(const xtm_particles_s* p) {
  SoA s;
  s.x = p->a.x; s.px = p->a.px; s.y = p->a.y; s.py = p->a.py; s.zeta = p->a.zeta;
  s.delta = p->a.delta; s.ptau = p->a.ptau; s.rpp = p->a.rpp; s.rvv = p->a.rvv;
  s.state = p->a.state; s.at_element = p->a.at_element; s.at_turn = p->a.at_turn;
  s.pid = p->a.particle_id;
  return s;
}

// CODATA 2018, the same data the oracle and the input generators use
constexpr double kRElectron = 2.8179403262e-15;  // m
constexpr double kMElectronEV = 0.51099895000e6;
constexpr double kHbarCEVM = 197.3269804e-9;     // eV m

KernelRef kref(const RefQ& r, int32_t rad_mode = 0, uint64_t seed = 0) {
  KernelRef k{};
  k.beta0 = r.beta0;
  k.two_over_beta0 = 2.0 / r.beta0;
  k.gamma0 = r.gamma0;
  // classical radius of the tracked species, scaled from the electron's
  const double rclass = kRElectron * (kMElectronEV / r.mass0) * r.charge0 * r.charge0;
  k.c_mean = 2.0 / 3.0 * rclass * r.mass0;
  k.c_quant = 55.0 / (24.0 * std::sqrt(3.0)) * rclass * r.mass0 * kHbarCEVM;
  k.c_nphot = 5.0 / (2.0 * std::sqrt(3.0)) * rclass * r.mass0 / kHbarCEVM;
  k.c_ucrit = 1.5 * kHbarCEVM;
  k.photon_table = nullptr;
  k.p0c = r.p0c;
  k.seed = seed;
  k.rad_mode = rad_mode;
  k.pad = 0;
  return k;
}

xtm_status read_alive(xtm_particles_s* p, hipStream_t s, int64_t* alive, int64_t* passes) {
  int32_t c[4];
  HIP_TRY(hipMemcpyAsync(c, p->ctrl, sizeof c, hipMemcpyDeviceToHost, s), "read counters");
  int64_t np = 0;
  HIP_TRY(hipMemcpyAsync(&np, p->passes, sizeof np, hipMemcpyDeviceToHost, s), "read passes");
  HIP_TRY(hipStreamSynchronize(s), "synchronise");
  if (alive) *alive = c[0];
  if (passes) *passes = np;
  p->alive_upper = c[0];
  return XTM_OK;
}

// Per-line kernel when the caller leaves the choice to the library: one-wave
// workgroups with each element's parameters fetched one element ahead
// (variant 10), the fastest form on the dynamic-aperture scans measured,
// whose surviving particles are too few to give every SIMD two waves.
// the default per-line form: one-wave workgroups with the next element's
// parameters read ahead, long cells (14); measured on one GPU against the
// same form with short cells (10), as fast or faster from 10^3 to 2^22
// particles
int32_t default_line_variant(int64_t) { return 14; }

int32_t auto_chunk(int64_t n, int32_t n_el, int32_t n_turns) {
  // aim at ~2e10 passes per launch so launch and epilogue costs vanish, while
  // compacting often enough that lost lanes stop costing issue slots
  const double per_turn = (double)(n > 0 ? n : 1) * (double)(n_el > 0 ? n_el : 1);
  double k = 2e10 / per_turn;
  if (k < 1.0) k = 1.0;
  if (k > (double)n_turns) k = (double)n_turns;
  return (int32_t)k;
}

struct ChunkPlan {
  const xtm_batch_s* batch;  // batched tracking, or null
  int32_t rad_mode;
  uint64_t seed;
  const double* photon_table;  // device inverse photon spectrum (radiation 3)
  float* rec;
  int32_t rec_turns;
  const LineKernel* line;  // variant 5
  const uint64_t* tab;
  int32_t n_turns, chunk, block, variant;
  int32_t compact_every;  // compact the alive list after every this many chunks (and the last)
  bool backward, compact;
  bool ramp;  // chunk lengths 1, 2, 4, ... up to `chunk` (automatic chunking)
};

// Turns of each launch: with automatic chunking the lengths start at one
// turn and double up to the target, so the losses of a fresh set (most of a
// dynamic-aperture grid is lost in its first turns) are replayed over short
// chunks; the sequence is a fixed function of the plan, so a captured graph
// replays it exactly.
std::vector<int32_t> chunk_sizes(const ChunkPlan& c) {
  std::vector<int32_t> v;
  int32_t done = 0, next = c.ramp ? 1 : c.chunk;
  while (done < c.n_turns) {
    const int32_t k = std::min(std::min(next, c.chunk), c.n_turns - done);
    v.push_back(k);
    done += k;
    if (next < c.chunk) next = (next > c.chunk / 2) ? c.chunk : 2 * next;
  }
  return v;
}

// Whether the alive list is compacted after chunk j of n: every
// compact_every chunks and after the last one.
bool compacts_after(const ChunkPlan& c, size_t j, size_t n) {
  if (!c.compact) return false;
  const size_t every = c.compact_every > 1 ? (size_t)c.compact_every : 1;
  return (j + 1) % every == 0 || j + 1 == n;
}

// Enqueue the whole chunk sequence on stream s: per chunk the tracking launch,
// the epilogue (passes + compaction) and the device-side turn advance.  The
// alive-list buffer alternates per compaction starting from `cur`.  Optional
// events bracket each tracking launch.
hipError_t enqueue_chunks(xtm_lattice_s* L, xtm_particles_s* P, const ChunkPlan& c, int32_t cur,
                          hipStream_t s, std::vector<hipEvent_t>* ev, int32_t* launches) {
  const SoA soa = soa_of(P);
  KernelRef kr = kref(L->ref, c.rad_mode, c.seed);
  kr.photon_table = c.photon_table;
  kr.rec = c.rec;
  kr.rec_turns = c.rec_turns;
  kr.rec_n = (int32_t)P->n;
  *launches = 0;
  if (P->alive_upper <= 0) return c.n_turns > 0 ? launch_advance(P->ctrl, c.backward ? -c.n_turns : c.n_turns, s) : hipSuccess;
  const std::vector<int32_t> sizes = chunk_sizes(c);
  for (size_t j = 0; j < sizes.size(); ++j) {
    const int32_t k = sizes[j];
    const bool compact_now = compacts_after(c, j, sizes.size());
    int32_t* in = P->idx[cur];
    int32_t* out = compact_now ? P->idx[1 - cur] : nullptr;
    hipError_t e;
    if (ev) {
      hipEvent_t a, b;
      if ((e = hipEventCreate(&a)) != hipSuccess) return e;
      if ((e = hipEventCreate(&b)) != hipSuccess) return e;
      ev->push_back(a);
      ev->push_back(b);
      if ((e = hipEventRecord(a, s)) != hipSuccess) return e;
    }
    if (c.batch && c.line)
      e = launch_line_batched(*c.line, L->n_el, soa, in, P->ctrl, P->alive_upper, k,
                              c.backward ? 1 : 0, kr, c.batch->first_d, s);
    else if (c.batch)
      e = launch_track_batched(c.batch->tabs_d, c.batch->first_d, (int32_t)c.batch->lats.size(),
                               L->n_el, soa, in, P->ctrl, P->alive_upper, c.block, k,
                               c.backward ? 1 : 0, kr, s);
    else if (c.line)
      e = launch_line(*c.line, L->n_el, soa, in, P->ctrl, P->alive_upper, c.block, k,
                      c.backward ? 1 : 0, kr, s);
    else
      e = launch_track(c.tab, L->n_el, soa, in, P->ctrl, P->alive_upper, c.block, k,
                       c.backward ? 1 : 0, kr, c.variant, s);
    if (e != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev->back(), s)) != hipSuccess) return e;
    ++*launches;
    // the interpreter keeps losses in registers and replays them; the
    // per-line kernels store a lost particle's coordinates as it is lost
    const bool replay = (c.variant == 4);
    e = launch_epilogue(in, out, replay ? P->lost : nullptr, P->alive_upper, soa, P->ctrl,
                        P->blockcnt, P->passes, L->n_el, k, c.backward ? 1 : 0, s);
    if (e != hipSuccess) return e;
    if (replay && c.batch) {
      e = launch_replay_batched(c.batch->tabs_d, c.batch->first_d, (int32_t)c.batch->lats.size(),
                                L->n_el, soa, P->lost, P->ctrl, P->alive_upper,
                                c.backward ? 1 : 0, kr, s);
      if (e != hipSuccess) return e;
    } else if (replay) {
      e = launch_replay(c.tab, L->n_el, soa, P->lost, P->ctrl, P->alive_upper, c.backward ? 1 : 0,
                        kr, s);
      if (e != hipSuccess) return e;
    }
    e = launch_advance(P->ctrl, c.backward ? -k : k, s);
    if (e != hipSuccess) return e;
    if (compact_now) cur = 1 - cur;
  }
  return hipSuccess;
}

int32_t flips(const ChunkPlan& c) {
  if (!c.compact || c.n_turns <= 0) return 0;
  const size_t n = chunk_sizes(c).size();
  int32_t f = 0;
  for (size_t j = 0; j < n; ++j) f += compacts_after(c, j, n) ? 1 : 0;
  return f;
}

xtm_status run_graph(xtm_lattice_s* L, xtm_particles_s* P, const ChunkPlan& c, hipStream_t s,
                     int32_t* launches) {
  GraphKey key{c.batch ? c.batch->id : L->id, c.n_turns, c.chunk, c.block, c.variant, c.backward ? 1 : 0, c.compact ? 1 : 0,
               c.compact_every, P->cur, c.rad_mode, P->alive_upper, c.seed, c.rec, c.rec_turns, c.ramp ? 1 : 0};
  for (const GraphEntry& g : P->graphs) {
    if (g.key == key) {
      HIP_TRY(hipGraphLaunch(g.exec, s), "graph launch");
      *launches = g.launches;
      return XTM_OK;
    }
  }
  if (!P->capture_stream)
    HIP_TRY(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking), "capture stream");
  HIP_TRY(hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal), "begin capture");
  int32_t n = 0;
  hipError_t e = enqueue_chunks(L, P, c, P->cur, P->capture_stream, nullptr, &n);
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(P->capture_stream, &graph);
  if (e != hipSuccess) { if (graph) hipGraphDestroy(graph); return hip_fail(e, "capture"); }
  if (e2 != hipSuccess) return hip_fail(e2, "end capture");
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "graph instantiate");
  if (P->graphs.size() >= 8) {  // keep the cache small
    hipGraphExecDestroy(P->graphs.front().exec);
    P->graphs.erase(P->graphs.begin());
  }
  P->graphs.push_back(GraphEntry{key, exec, n});
  HIP_TRY(hipGraphLaunch(exec, s), "graph launch");
  *launches = n;
  return XTM_OK;
}

void drop_graphs(xtm_particles_s* P) {
  for (GraphEntry& g : P->graphs) hipGraphExecDestroy(g.exec);
  P->graphs.clear();
}

xtm_status run_turns(xtm_lattice_s* L, xtm_particles_s* P, int32_t n_turns,
                     const xtm_track_opts* o, hipStream_t s, xtm_track_stats* stats,
                     bool backward, xtm_batch_s* B = nullptr) {
  if (!L || !P) return fail(XTM_E_ARG, "null handle");
  if (n_turns < 0) return fail(XTM_E_ARG, "n_turns must be >= 0");
  if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
  if (!same_ref(L->ref, P->ref))
    return fail(XTM_E_REFERENCE, "lattice and particle set have different references");
  if (backward && P->turn - n_turns < INT32_MIN / 2) return fail(XTM_E_ARG, "turn underflow");
  if (!backward && (int64_t)P->turn + n_turns > INT32_MAX / 2) return fail(XTM_E_ARG, "turn overflow");
  ChunkPlan c;
  c.batch = B;
  c.rad_mode = o ? o->radiation : 0;
  c.seed = o ? o->rng_seed : 0;
  c.rec = o ? o->record_buf : nullptr;
  c.rec_turns = (o && o->record_buf) ? o->record_turns : 0;
  if (c.rec && (c.rec_turns < 0 || backward))
    return fail(XTM_E_ARG, "the recorder needs record_turns >= 0 and forward tracking");
  if (c.rad_mode < 0 || c.rad_mode > 3) return fail(XTM_E_ARG, "radiation must be 0, 1, 2 or 3");
  c.photon_table = nullptr;
  if (c.rad_mode == 3) HIP_TRY(photon_table_device(&c.photon_table), "photon spectrum table");
  if (c.rad_mode && backward) return fail(XTM_E_ARG, "backward tracking with radiation is undefined");
  const bool use_plan = !(o && (o->block || o->variant));
  const int32_t plan_block = B ? B->plan_block : L->plan_block;
  c.block = (o && o->block) ? o->block : (use_plan && plan_block ? plan_block : 256);
  if (c.block < 64 || c.block > 256 || c.block % 64)
    return fail(XTM_E_ARG, "block must be 64, 128, 192 or 256");
  c.compact = !(o && o->no_compact) || backward;
  c.variant = (o && o->variant) ? o->variant
                                : (use_plan ? (B ? B->plan_variant : L->plan_variant) : 0);
  if (c.variant < 0 || (c.variant >= 1 && c.variant <= 3) || c.variant > 4 + kLineStyles)
    return fail(XTM_E_ARG, "kernel variant must be 0, 4 or 5.." + std::to_string(4 + kLineStyles));
  if (B) {
    if (backward) return fail(XTM_E_UNSUPPORTED, "batched tracking is forward only");
    if (c.variant != 0 && c.variant != 4 && !(c.variant >= 5 && line_block(c.variant - 5) == 64))
      return fail(XTM_E_UNSUPPORTED,
                  "batched tracking runs the interpreter (4) or a one-wave per-line form");
  }
  c.line = nullptr;
  if (c.variant == 0 || c.variant >= 5) {
    // the per-line kernel, compiled on first use; the default falls back to
    // the register-loss interpreter if the line has no compact cell structure
    // (a batch: if its variants differ in element structure)
    const int32_t want = c.variant ? c.variant : default_line_variant(P->alive_upper);
    const int32_t form = rad_form(L->radiates, c.rad_mode);
    LineKernel& lk = B ? B->line[form][want - 5]
                       : (backward ? L->bwd_line[want - 5] : L->fwd_line[form][want - 5]);
    if (!lk.tried && L->n_el > 0) {
      lk.tried = true;
      if (B) {
        std::vector<const std::vector<uint64_t>*> tabs;
        for (const xtm_lattice_s* l : B->lats) tabs.push_back(&l->fwd_h);
        build_line_kernel_multi(tabs, L->n_el, want - 5, true, form, &lk);
      } else {
        build_line_kernel(backward ? L->bwd_h : L->fwd_h, L->n_el, want - 5, form, &lk);
      }
    }
    if (lk.ok) {
      c.variant = want;
      c.line = &lk;
      c.block = line_block(want - 5);
    } else if (c.variant >= 5 && L->n_el > 0) {
      return fail(XTM_E_UNSUPPORTED, "per-line kernel unavailable: " + lk.error);
    } else {
      c.variant = 4;
    }
  }
  // turns per chunk: the caller's (a fixed length), else the plan's or the
  // automatic target, reached by a ramp from one turn
  const int32_t plan_chunk = B ? B->plan_chunk : L->plan_chunk;
  c.ramp = !(o && o->turns_per_chunk > 0);
  c.chunk = (o && o->turns_per_chunk > 0)
                ? o->turns_per_chunk
                : (plan_chunk > 0 ? std::min(plan_chunk, std::max(n_turns, 1))
                                  : auto_chunk(P->alive_upper, L->n_el, n_turns));
  if (o && o->compact_every < 0) return fail(XTM_E_ARG, "compact_every must be >= 0");
  const int32_t plan_every = B ? B->plan_compact_every : L->plan_compact_every;
  c.compact_every = (o && o->compact_every > 0) ? o->compact_every
                                                 : (plan_every > 0 ? plan_every : 1);
  if (c.chunk < 1) c.chunk = 1;
  if (L->n_el > 0 && (int64_t)c.chunk * L->n_el > INT32_MAX - 1)
    c.chunk = (int32_t)((INT32_MAX - 1) / L->n_el);
  c.n_turns = n_turns;
  c.backward = backward;
  c.tab = backward ? L->bwd_d : L->fwd_d;
  const bool graph = o && o->use_graph;
  const int64_t alive_before = P->alive_upper;
  if (stats) HIP_TRY(launch_fill_i64(P->passes, 0, s), "clear passes");
  const bool timing = stats && o && o->time_kernels;
  std::vector<hipEvent_t> ev;
  int32_t launches = 0;
  if (graph && n_turns > 0) {
    hipEvent_t a = nullptr, b = nullptr;
    if (timing) {
      HIP_TRY(hipEventCreate(&a), "event");
      HIP_TRY(hipEventCreate(&b), "event");
      ev.push_back(a);
      ev.push_back(b);
      HIP_TRY(hipEventRecord(a, s), "event record");
    }
    xtm_status st = run_graph(L, P, c, s, &launches);
    if (st != XTM_OK) return st;
    if (timing) HIP_TRY(hipEventRecord(b, s), "event record");
  } else if (n_turns > 0) {
    HIP_TRY(enqueue_chunks(L, P, c, P->cur, s, timing ? &ev : nullptr, &launches), "chunk launch");
  }
  // (an empty alive list enqueues no compaction, so the buffers do not swap)
  if (alive_before > 0 && (flips(c) & 1)) P->cur = 1 - P->cur;
  P->turn = backward ? P->turn - n_turns : P->turn + n_turns;
  if (stats) {
    int64_t alive = 0, passes = 0;
    xtm_status st = read_alive(P, s, &alive, &passes);
    double ms = 0.0;
    for (size_t j = 0; j + 1 < ev.size(); j += 2) {
      float dt = 0.f;
      if (st == XTM_OK && hipEventElapsedTime(&dt, ev[j], ev[j + 1]) == hipSuccess) ms += dt;
    }
    for (hipEvent_t e : ev) hipEventDestroy(e);
    if (st != XTM_OK) return st;
    stats->alive = alive;
    stats->passes = passes;
    stats->launches = launches;
    stats->variant = c.variant;
    stats->kernel_ms = ms;
  }
  return XTM_OK;
}

template <class F>
xtm_status guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return fail(XTM_E_NOMEM, "host allocation failed");
  } catch (const std::exception& ex) {
    return fail(XTM_E_ARG, ex.what());
  } catch (...) {
    return fail(XTM_E_ARG, "unknown exception");
  }
}

}  // namespace

extern "C" {

const char* xtm_last_error(void) { return g_err.c_str(); }
int32_t xtm_max_variant(void) { return 4 + xtm::kLineStyles; }

const char* xtm_version(void) { return "xtm 0.1 (gfx950, FP64 thin-lattice tracker)"; }

namespace {
// Thick elements as drift-kick-drift slices, kicks at the slice midpoints:
// d = L/N; DRIFT(d/2), then N times [kick, DRIFT(d)], the last drift d/2.
xtm_status expand_thick(const xtm_element_desc* el, int32_t n, std::vector<xtm_element_desc>* out,
                        std::vector<int32_t>* user) {
  for (int32_t i = 0; i < n; ++i) {
    const xtm_element_desc& e = el[i];
    if (e.type != XTM_QUADRUPOLE && e.type != XTM_SBEND) {
      out->push_back(e);
      user->push_back(i);
      continue;
    }
    const std::string where = "element " + std::to_string(i) + ": ";
    const double L = e.length, Nd = e.p[2];
    if (!(L > 0.0) || !std::isfinite(L))
      return fail(XTM_E_ELEMENT, where + "thick element needs a finite length > 0");
    if (!(Nd >= 1.0 && Nd <= 10000.0) || Nd != std::floor(Nd))
      return fail(XTM_E_ELEMENT, where + "slice count p[2] must be an integer in 1..10000");
    if (!std::isfinite(e.p[0]) || !std::isfinite(e.p[1]))
      return fail(XTM_E_ELEMENT, where + "non-finite strength");
    const int32_t N = (int32_t)Nd;
    const double d = L / (double)N;
    const double half = 0.5 * d;
    xtm_element_desc dr{};
    dr.type = XTM_DRIFT;
    xtm_element_desc k{};
    k.type = XTM_MULTIPOLE;
    k.order = 1;
    if (e.type == XTM_QUADRUPOLE) {
      k.knl[1] = e.p[0] * d;
      k.ksl[1] = e.p[1] * d;
    } else {
      const double a = e.p[0] / (double)N;
      k.knl[0] = a;
      k.hxl = a;
      k.length = d;
      k.knl[1] = e.p[1] * d;
    }
    dr.length = half;
    out->push_back(dr);
    user->push_back(i);
    for (int32_t j = 0; j < N; ++j) {
      out->push_back(k);
      user->push_back(i);
      dr.length = (j + 1 == N) ? half : d;
      out->push_back(dr);
      user->push_back(i);
    }
  }
  if (out->size() > (size_t)0x7fffffff) return fail(XTM_E_ELEMENT, "line too long");
  return XTM_OK;
}
}  // namespace

xtm_status xtm_lattice_create(const xtm_element_desc* el, int32_t n, const xtm_reference* ref,
                              xtm_lattice* out) {
  return guarded([&]() -> xtm_status {
    if (!out) return fail(XTM_E_ARG, "out is null");
    *out = nullptr;
    if (n < 0 || (n > 0 && !el)) return fail(XTM_E_ARG, "bad element array");
    RefQ r;
    if (!make_ref(ref, &r)) return fail(XTM_E_REFERENCE, "reference needs mass > 0 and p0c > 0");
    auto* L = new xtm_lattice_s();
    L->ref = r;
    {
      const xtm_status st = expand_thick(el, n, &L->desc_h, &L->user_h);
      if (st != XTM_OK) { delete L; return st; }
    }
    n = (int32_t)L->desc_h.size();
    L->n_el = n;
    for (int32_t i = 0; i < n; ++i) {
      xtm_status st = pack(L->desc_h[i], L->user_h[i], r, 1.0, L->fwd_h);
      if (st != XTM_OK) { delete L; return st; }
    }
    for (int32_t i = n - 1; i >= 0; --i) {
      xtm_status st = pack(L->desc_h[i], L->user_h[i], r, -1.0, L->bwd_h);
      if (st != XTM_OK) { delete L; return st; }
    }
    L->radiates = table_radiates(L->fwd_h, n);
    L->fwd_seg_h = segment(L->fwd_h, n);
    L->bwd_seg_h = segment(L->bwd_h, n);
    const size_t sbytes = L->fwd_seg_h.size() * sizeof(int32_t);
    if (hipMalloc(&L->fwd_seg_d, sbytes) != hipSuccess ||
        hipMalloc(&L->bwd_seg_d, L->bwd_seg_h.size() * sizeof(int32_t)) != hipSuccess ||
        hipMemcpy(L->fwd_seg_d, L->fwd_seg_h.data(), sbytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L->bwd_seg_d, L->bwd_seg_h.data(), L->bwd_seg_h.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(L->fwd_seg_d);
      hipFree(L->bwd_seg_d);
      delete L;
      return fail(XTM_E_NOMEM, "device allocation of the segment table failed");
    }
    const size_t bytes = (L->fwd_h.size() + 1) * sizeof(uint64_t);
    if (hipMalloc(&L->fwd_d, bytes) != hipSuccess || hipMalloc(&L->bwd_d, bytes) != hipSuccess) {
      hipFree(L->fwd_d);
      delete L;
      return fail(XTM_E_NOMEM, "device allocation of the element table failed");
    }
    L->fwd_h.push_back(0);
    L->bwd_h.push_back(0);
    if (hipMemcpy(L->fwd_d, L->fwd_h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(L->bwd_d, L->bwd_h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
      hipFree(L->fwd_d);
      hipFree(L->bwd_d);
      delete L;
      return fail(XTM_E_HIP, "copy of the element table failed");
    }
    *out = L;
    return XTM_OK;
  });
}

xtm_status xtm_lattice_destroy(xtm_lattice L) {
  if (!L) return XTM_OK;
  hipFree(L->fwd_d);
  hipFree(L->bwd_d);
  hipFree(L->fwd_seg_d);
  hipFree(L->bwd_seg_d);
  hipFree(L->refine_buf);
  for (int32_t k = 0; k < kLineStyles; ++k) {
    for (int32_t f = 0; f < kRadForms; ++f) free_line_kernel(&L->fwd_line[f][k]);
    free_line_kernel(&L->bwd_line[k]);
  }
  free_line_kernel(&L->rec_line);
  delete L;
  return XTM_OK;
}

xtm_status xtm_lattice_user_index(xtm_lattice L, int32_t* h_out) {
  return guarded([&]() -> xtm_status {
    if (!L || (!h_out && L->n_el > 0)) return fail(XTM_E_ARG, "null lattice or output");
    if (L->n_el > 0) std::memcpy(h_out, L->user_h.data(), L->n_el * sizeof(int32_t));
    return XTM_OK;
  });
}

xtm_status xtm_lattice_info(xtm_lattice L, int32_t* n_elements, int64_t* table_bytes) {
  if (!L) return fail(XTM_E_ARG, "null lattice");
  if (n_elements) *n_elements = L->n_el;
  if (table_bytes) *table_bytes = (int64_t)(L->fwd_h.size() * sizeof(uint64_t));
  return XTM_OK;
}

xtm_status xtm_particles_bind(const xtm_arrays* a, const xtm_reference* ref, xtm_particles* out) {
  return guarded([&]() -> xtm_status {
    if (!out) return fail(XTM_E_ARG, "out is null");
    *out = nullptr;
    if (!a || a->n < 0) return fail(XTM_E_ARG, "bad array descriptor");
    if (a->n > INT32_MAX - 1024) return fail(XTM_E_ARG, "at most 2^31 - 1025 particles per set");
    if (a->n > 0 && (!a->x || !a->px || !a->y || !a->py || !a->zeta || !a->delta || !a->ptau ||
                     !a->rpp || !a->rvv || !a->state || !a->at_element || !a->at_turn ||
                     !a->particle_id))
      return fail(XTM_E_ARG, "null particle array");
    RefQ r;
    if (!make_ref(ref, &r)) return fail(XTM_E_REFERENCE, "reference needs mass > 0 and p0c > 0");
    auto* P = new xtm_particles_s();
    P->a = *a;
    P->ref = r;
    P->n = a->n;
    const int64_t m = a->n > 0 ? a->n : 1;
    const int64_t nb = (m + kScanBlock - 1) / kScanBlock;
    bool ok = hipMalloc(&P->idx[0], m * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->idx[1], m * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->lost, m * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->ctrl, 4 * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->blockcnt, 2 * nb * sizeof(int32_t)) == hipSuccess &&
              hipMalloc(&P->passes, sizeof(int64_t)) == hipSuccess;
    if (!ok) {
      hipFree(P->idx[0]); hipFree(P->idx[1]); hipFree(P->lost); hipFree(P->ctrl);
      hipFree(P->blockcnt);
      hipFree(P->passes);
      delete P;
      return fail(XTM_E_NOMEM, "device allocation of particle work buffers failed");
    }
    *out = P;
    return XTM_OK;
  });
}

xtm_status xtm_particles_release(xtm_particles P) {
  if (!P) return XTM_OK;
  drop_graphs(P);
  if (P->capture_stream) hipStreamDestroy(P->capture_stream);
  hipFree(P->idx[0]);
  hipFree(P->idx[1]);
  hipFree(P->lost);
  hipFree(P->ctrl);
  hipFree(P->blockcnt);
  hipFree(P->passes);
  delete P;
  return XTM_OK;
}

xtm_status xtm_particles_init(xtm_particles P, const double* coords, int64_t first_id,
                              int32_t coords_on_device, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!P) return fail(XTM_E_ARG, "null particle set");
    if (P->n > 0 && !coords) return fail(XTM_E_ARG, "coords is null");
    hipStream_t s = (hipStream_t)stream;
    const double* dc = coords;
    double* tmp = nullptr;
    if (P->n > 0 && !coords_on_device) {
      const size_t bytes = (size_t)P->n * 6 * sizeof(double);
      if (hipMalloc(&tmp, bytes) != hipSuccess) return fail(XTM_E_NOMEM, "staging allocation failed");
      hipError_t e = hipMemcpyAsync(tmp, coords, bytes, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) { hipFree(tmp); return hip_fail(e, "upload of coordinates"); }
      dc = tmp;
    }
    hipError_t e = launch_init(dc, P->n, first_id, soa_of(P), kref(P->ref), s);
    if (e == hipSuccess) e = launch_iota(P->idx[0], P->n, P->ctrl, (int32_t)P->n, 0, s);
    if (e == hipSuccess) e = launch_fill_i64(P->passes, 0, s);
    if (tmp) {
      hipError_t e2 = hipStreamSynchronize(s);
      hipFree(tmp);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return hip_fail(e, "particle initialisation");
    P->cur = 0;
    P->turn = 0;
    P->alive_upper = P->n;
    P->initialised = true;
    return XTM_OK;
  });
}

xtm_status xtm_particles_reset(xtm_particles P, int32_t turn, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!P) return fail(XTM_E_ARG, "null particle set");
    hipStream_t s = (hipStream_t)stream;
    // all indices into the spare buffer, then one compaction into the live one
    hipError_t e = launch_iota(P->idx[1 - P->cur], P->n, P->ctrl, (int32_t)P->n, turn, s);
    if (e == hipSuccess)
      e = launch_epilogue(P->idx[1 - P->cur], P->idx[P->cur], nullptr, P->n > 0 ? P->n : 1,
                          soa_of(P), P->ctrl, P->blockcnt, P->passes, 0, 0, 0, s);
    if (e != hipSuccess) return hip_fail(e, "alive-list rebuild");
    P->turn = turn;
    P->alive_upper = P->n;
    P->initialised = true;
    return XTM_OK;
  });
}

xtm_status xtm_particles_turn(xtm_particles P, int32_t* turn) {
  if (!P || !turn) return fail(XTM_E_ARG, "null argument");
  *turn = P->turn;
  return XTM_OK;
}

xtm_status xtm_track(xtm_lattice L, xtm_particles P, int32_t n_turns, const xtm_track_opts* opts,
                     void* stream, xtm_track_stats* stats) {
  return guarded([&]() {
    return run_turns(L, P, n_turns, opts, (hipStream_t)stream, stats, false);
  });
}

xtm_status xtm_track_backward(xtm_lattice L, xtm_particles P, int32_t n_turns, void* stream,
                              xtm_track_stats* stats) {
  return guarded([&]() {
    return run_turns(L, P, n_turns, nullptr, (hipStream_t)stream, stats, true);
  });
}

xtm_status xtm_track_per_element(xtm_lattice L, xtm_particles P, int32_t n_turns, void* stream,
                                 xtm_track_stats* stats) {
  return guarded([&]() -> xtm_status {
    if (!L || !P) return fail(XTM_E_ARG, "null lattice or particle set");
    if (n_turns < 0) return fail(XTM_E_ARG, "n_turns must be >= 0");
    if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
    if (!same_ref(L->ref, P->ref)) return fail(XTM_E_REFERENCE, "reference mismatch");
    hipStream_t s = (hipStream_t)stream;
    std::vector<uint32_t> off, kt;  // word position and kernel type of each element's record
    off.reserve(L->n_el);
    kt.reserve(L->n_el);
    for (size_t w = 0; off.size() < (size_t)L->n_el && w < L->fwd_h.size();
         w += 1 + ((L->fwd_h[w] >> 16) & 0xffffu)) {
      off.push_back((uint32_t)w);
      kt.push_back((uint32_t)(L->fwd_h[w] & 0xffu));
    }
    if (off.size() != (size_t)L->n_el) return fail(XTM_E_STATE, "element table inconsistent");
    std::vector<int32_t> st0, at, ae, st1;
    if (stats) {  // passes are counted on the host from the states before and after
      st0.resize(P->n);
      if (P->n > 0)
        HIP_TRY(hipMemcpyAsync(st0.data(), P->a.state, P->n * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s), "copy state");
      HIP_TRY(hipStreamSynchronize(s), "synchronise");
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (stats) {
      HIP_TRY(hipEventCreate(&a), "event");
      HIP_TRY(hipEventCreate(&b), "event");
      HIP_TRY(hipEventRecord(a, s), "event record");
    }
    const KernelRef kr = kref(L->ref, 0, 0);
    HIP_TRY(launch_per_element(L->fwd_d, off.data(), kt.data(), L->n_el, soa_of(P), P->n, P->turn,
                               n_turns, kr, s), "per-element launch");
    if (stats) HIP_TRY(hipEventRecord(b, s), "event record");
    const int32_t t0 = P->turn;
    xtm_status rs = xtm_particles_reset(P, t0 + n_turns, stream);
    if (rs != XTM_OK) return rs;
    if (stats) {
      st1.resize(P->n);
      at.resize(P->n);
      ae.resize(P->n);
      const size_t bytes = P->n * sizeof(int32_t);
      if (P->n > 0) {
        HIP_TRY(hipMemcpyAsync(st1.data(), P->a.state, bytes, hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipMemcpyAsync(at.data(), P->a.at_turn, bytes, hipMemcpyDeviceToHost, s), "copy");
        HIP_TRY(hipMemcpyAsync(ae.data(), P->a.at_element, bytes, hipMemcpyDeviceToHost, s), "copy");
      }
      HIP_TRY(hipStreamSynchronize(s), "synchronise");
      int64_t passes = 0, alive = 0;
      for (int64_t i = 0; i < P->n; ++i) {
        if (st0[i] != 1) continue;
        if (st1[i] == 1) {
          passes += (int64_t)n_turns * L->n_el;
          ++alive;
        } else {
          passes += (int64_t)(at[i] - t0) * L->n_el + ae[i] + 1;
        }
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, a, b);
      hipEventDestroy(a);
      hipEventDestroy(b);
      stats->passes = passes;
      stats->alive = alive;
      stats->launches = n_turns * L->n_el;
      stats->variant = 0;
      stats->kernel_ms = ms;
    }
    return XTM_OK;
  });
}

// ------------------------------------------------------------ batches
xtm_status xtm_batch_create(const xtm_lattice* lattices, int32_t n_variants, xtm_batch* out) {
  return guarded([&]() -> xtm_status {
    if (!out) return fail(XTM_E_ARG, "out is null");
    *out = nullptr;
    if (!lattices || n_variants < 1) return fail(XTM_E_ARG, "need at least one lattice");
    for (int32_t v = 0; v < n_variants; ++v) {
      if (!lattices[v]) return fail(XTM_E_ARG, "null lattice " + std::to_string(v));
      if (lattices[v]->n_el != lattices[0]->n_el)
        return fail(XTM_E_ARG, "all lattices of a batch need the same element count");
      if (!same_ref(lattices[v]->ref, lattices[0]->ref))
        return fail(XTM_E_REFERENCE, "all lattices of a batch need the same reference");
    }
    auto* B = new xtm_batch_s();
    B->lats.assign(lattices, lattices + n_variants);
    B->n_el = lattices[0]->n_el;
    B->ref = lattices[0]->ref;
    std::vector<uint64_t*> t(n_variants);
    for (int32_t v = 0; v < n_variants; ++v) t[v] = lattices[v]->fwd_d;
    if (hipMalloc(&B->tabs_d, n_variants * sizeof(uint64_t*)) != hipSuccess ||
        hipMalloc(&B->first_d, (n_variants + 1) * sizeof(int32_t)) != hipSuccess ||
        hipMemcpy(B->tabs_d, t.data(), n_variants * sizeof(uint64_t*), hipMemcpyHostToDevice) !=
            hipSuccess) {
      hipFree(B->tabs_d);
      hipFree(B->first_d);
      delete B;
      return fail(XTM_E_NOMEM, "batch tables");
    }
    *out = B;
    return XTM_OK;
  });
}

xtm_status xtm_batch_destroy(xtm_batch B) {
  if (!B) return XTM_OK;
  for (int32_t f = 0; f < kRadForms; ++f)
    for (int32_t k = 0; k < kLineStyles; ++k) free_line_kernel(&B->line[f][k]);
  hipFree(B->tabs_d);
  hipFree(B->first_d);
  delete B;
  return XTM_OK;
}

namespace {
xtm_status set_partition(xtm_batch_s* B, xtm_particles_s* P, const int64_t* first_slot,
                         hipStream_t s) {
  const size_t nv = B->lats.size();
  if (!first_slot) return fail(XTM_E_ARG, "null slot partition");
  if (first_slot[0] != 0 || first_slot[nv] != P->n)
    return fail(XTM_E_ARG, "the slot partition must run from 0 to the set's size");
  for (size_t v = 0; v < nv; ++v)
    if (first_slot[v + 1] < first_slot[v]) return fail(XTM_E_ARG, "slot partition not ascending");
  std::vector<int64_t> f(first_slot, first_slot + nv + 1);
  if (f == B->first_h) return XTM_OK;
  std::vector<int32_t> f32(f.begin(), f.end());
  // the previous partition may still be read by queued kernels
  HIP_TRY(hipStreamSynchronize(s), "synchronise");
  HIP_TRY(hipMemcpy(B->first_d, f32.data(), f32.size() * sizeof(int32_t), hipMemcpyHostToDevice),
          "partition upload");
  B->first_h = f;
  return XTM_OK;
}
}  // namespace

xtm_status xtm_track_batched(xtm_batch B, xtm_particles P, const int64_t* first_slot,
                             int32_t n_turns, const xtm_track_opts* opts, void* stream,
                             xtm_track_stats* stats) {
  return guarded([&]() -> xtm_status {
    if (!B || !P) return fail(XTM_E_ARG, "null handle");
    xtm_status st = set_partition(B, P, first_slot, (hipStream_t)stream);
    if (st != XTM_OK) return st;
    return run_turns(B->lats[0], P, n_turns, opts, (hipStream_t)stream, stats, false, B);
  });
}

// ------------------------------------------------------------ autotuner
namespace {
// A scratch copy of a particle set: its own arrays, bound as a set.
struct Scratch {
  void* mem = nullptr;
  xtm_particles_s* P = nullptr;
  ~Scratch() {
    if (P) xtm_particles_release(P);
    hipFree(mem);
  }
};

xtm_status make_scratch_n(int64_t n, const RefQ& ref, Scratch* sc) {
  const int64_t m = n > 0 ? n : 1;
  const size_t bytes = (size_t)m * (9 * sizeof(double) + 3 * sizeof(int32_t) + sizeof(int64_t));
  HIP_TRY(hipMalloc(&sc->mem, bytes), "scratch particles");
  char* b = static_cast<char*>(sc->mem);
  xtm_arrays a{};
  double** f[9] = {&a.x, &a.px, &a.y, &a.py, &a.zeta, &a.delta, &a.ptau, &a.rpp, &a.rvv};
  for (int k = 0; k < 9; ++k) { *f[k] = reinterpret_cast<double*>(b); b += m * sizeof(double); }
  a.particle_id = reinterpret_cast<int64_t*>(b); b += m * sizeof(int64_t);
  int32_t** g[3] = {&a.state, &a.at_element, &a.at_turn};
  for (int k = 0; k < 3; ++k) { *g[k] = reinterpret_cast<int32_t*>(b); b += m * sizeof(int32_t); }
  a.n = n;
  xtm_reference r{ref.mass0, ref.charge0, ref.p0c};
  return xtm_particles_bind(&a, &r, &sc->P);
}

xtm_status make_scratch(const xtm_particles_s* src, Scratch* sc) {
  return make_scratch_n(src->n, src->ref, sc);
}

xtm_status copy_set(const xtm_particles_s* src, xtm_particles_s* dst, hipStream_t s) {
  const size_t nd = (size_t)src->n * sizeof(double), ni = (size_t)src->n * sizeof(int32_t);
  const xtm_arrays &a = src->a, &b = dst->a;
  const double* fs[9] = {a.x, a.px, a.y, a.py, a.zeta, a.delta, a.ptau, a.rpp, a.rvv};
  double* fd[9] = {b.x, b.px, b.y, b.py, b.zeta, b.delta, b.ptau, b.rpp, b.rvv};
  for (int k = 0; k < 9; ++k) HIP_TRY(hipMemcpyAsync(fd[k], fs[k], nd, hipMemcpyDeviceToDevice, s), "copy");
  const int32_t* is[3] = {a.state, a.at_element, a.at_turn};
  int32_t* id[3] = {b.state, b.at_element, b.at_turn};
  for (int k = 0; k < 3; ++k) HIP_TRY(hipMemcpyAsync(id[k], is[k], ni, hipMemcpyDeviceToDevice, s), "copy");
  HIP_TRY(hipMemcpyAsync(b.particle_id, a.particle_id, src->n * sizeof(int64_t),
                         hipMemcpyDeviceToDevice, s), "copy");
  HIP_TRY(launch_fill_i64(dst->passes, 0, s), "clear passes");
  return xtm_particles_reset(dst, src->turn, s);
}
}  // namespace

xtm_status xtm_autotune(xtm_lattice L, xtm_batch B, xtm_particles P, const int64_t* first_slot,
                        int32_t probe_turns, int32_t warm_turns, void* stream, xtm_plan* out) {
  return guarded([&]() -> xtm_status {
    if ((!L && !B) || (L && B) || !P) return fail(XTM_E_ARG, "give one of lattice or batch, and a set");
    if (probe_turns < 1) return fail(XTM_E_ARG, "probe_turns must be >= 1");
    if (warm_turns < 0) return fail(XTM_E_ARG, "warm_turns must be >= 0");
    if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
    hipStream_t s = (hipStream_t)stream;
    xtm_lattice_s* lat = B ? B->lats[0] : L;
    if (!same_ref(lat->ref, P->ref)) return fail(XTM_E_REFERENCE, "reference mismatch");
    if (B) {
      xtm_status st = set_partition(B, P, first_slot, s);
      if (st != XTM_OK) return st;
    }
    int32_t& pv = B ? B->plan_variant : L->plan_variant;
    int32_t& pb = B ? B->plan_block : L->plan_block;
    int32_t& pk = B ? B->plan_chunk : L->plan_chunk;
    int32_t& pc = B ? B->plan_compact_every : L->plan_compact_every;
    // the probes start from `base`: the set itself, or a copy of it tracked
    // warm_turns turns further (past the losses of its first turns, so the
    // probe sees the alive count and loss rate of the stretch it plans for)
    Scratch base_sc, sc;
    xtm_status st = make_scratch(P, &sc);
    if (st != XTM_OK) return st;
    const xtm_particles_s* base = P;
    if (warm_turns > 0) {
      st = make_scratch(P, &base_sc);
      if (st == XTM_OK) st = copy_set(P, base_sc.P, s);
      if (st == XTM_OK) st = run_turns(lat, base_sc.P, warm_turns, nullptr, s, nullptr, false, B);
      if (st == XTM_OK) {
        int64_t alive = 0;
        st = read_alive(base_sc.P, s, &alive, nullptr);
      }
      if (st != XTM_OK) return st;
      base = base_sc.P;
    }
    std::vector<int32_t> variants;
    if (lat->n_el > 0) {
      std::vector<const std::vector<uint64_t>*> tabs;
      if (B)
        for (const xtm_lattice_s* l : B->lats) tabs.push_back(&l->fwd_h);
      for (int32_t k = 0; k < kLineStyles; ++k) {
        if (B && line_block(k) != 64) continue;  // batches: the one-wave forms
        // the probes track without radiation
        LineKernel& lk = B ? B->line[0][k] : lat->fwd_line[0][k];
        if (!lk.tried) {
          lk.tried = true;
          if (B)
            build_line_kernel_multi(tabs, lat->n_el, k, true, 0, &lk);
          else
            build_line_kernel(lat->fwd_h, lat->n_el, k, 0, &lk);
        }
        if (lk.ok) variants.push_back(5 + k);
      }
    }
    variants.push_back(4);
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0), "event");
    HIP_TRY(hipEventCreate(&e1), "event");
    // one candidate plan: set it on the lattice (or batch), run the probe
    // through the plain tracking path (as later calls will), untimed then timed
    auto probe = [&](int32_t v, int32_t blk, int32_t k, int32_t every, double* rate) -> xtm_status {
      pv = v;
      pb = blk;
      pk = k;
      pc = every;
      for (int rep = 0; rep < 2; ++rep) {
        xtm_status r = copy_set(base, sc.P, s);
        if (r != XTM_OK) return r;
        if (hipEventRecord(e0, s) != hipSuccess) return fail(XTM_E_HIP, "event");
        r = run_turns(lat, sc.P, probe_turns, nullptr, s, nullptr, false, B);
        if (r != XTM_OK) return r;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
          return fail(XTM_E_HIP, "event");
        int64_t alive = 0, passes = 0;
        r = read_alive(sc.P, s, &alive, &passes);
        if (r != XTM_OK) return r;
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        *rate = ms > 0 ? (double)passes / (ms * 1e-3) : 0.0;
      }
      return XTM_OK;
    };
    xtm_plan best{};
    double best_rate = -1.0;
    auto consider = [&](int32_t v, int32_t blk, int32_t k, int32_t every) -> xtm_status {
      double rate = 0.0;
      xtm_status r = probe(v, blk, k, every, &rate);
      if (r == XTM_OK && rate > best_rate) {
        best_rate = rate;
        best = xtm_plan{v, blk, rate, k, every};
      }
      return r;
    };
    // 1. kernel form and block, automatic chunks compacted after each
    const int32_t blocks[3] = {64, 128, 256};
    for (int32_t v : variants) {
      for (int32_t blk : blocks) {
        if (v >= 5 && blk != line_block(v - 5)) continue;  // the per-line kernels' fixed shape
        if ((st = consider(v, blk, 0, 1)) != XTM_OK) break;
      }
      if (st != XTM_OK) break;
    }
    // 2. turns per chunk for that form (0 = automatic), up to the probe length
    if (st == XTM_OK) {
      const xtm_plan f = best;
      for (int32_t k : {1, 4, 16, 64, 256, 1024}) {
        if (k > probe_turns) break;
        if ((st = consider(f.variant, f.block, k, 1)) != XTM_OK) break;
      }
    }
    // 3. compaction period for that form and chunk length
    if (st == XTM_OK) {
      const xtm_plan f = best;
      for (int32_t every : {2, 4, 8}) {
        if ((st = consider(f.variant, f.block, f.turns_per_chunk, every)) != XTM_OK) break;
      }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != XTM_OK) {
      pv = pb = pk = pc = 0;
      return st;
    }
    pv = best.variant;
    pb = best.block;
    pk = best.turns_per_chunk;
    pc = best.compact_every;
    if (out) *out = best;
    return XTM_OK;
  });
}

xtm_status xtm_get_losses(xtm_particles P, int32_t* h_state, int32_t* h_at_turn,
                          int32_t* h_at_element, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!P) return fail(XTM_E_ARG, "null particle set");
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)P->n * sizeof(int32_t);
    if (P->n > 0) {
      if (h_state) HIP_TRY(hipMemcpyAsync(h_state, P->a.state, bytes, hipMemcpyDeviceToHost, s), "copy state");
      if (h_at_turn) HIP_TRY(hipMemcpyAsync(h_at_turn, P->a.at_turn, bytes, hipMemcpyDeviceToHost, s), "copy at_turn");
      if (h_at_element)
        HIP_TRY(hipMemcpyAsync(h_at_element, P->a.at_element, bytes, hipMemcpyDeviceToHost, s), "copy at_element");
    }
    HIP_TRY(hipStreamSynchronize(s), "synchronise");
    return XTM_OK;
  });
}

xtm_status xtm_philox4x32_10(uint64_t seed, const uint32_t ctr0[4], int64_t n_blocks,
                             uint32_t* d_out, void* stream) {
  if (n_blocks < 0 || !ctr0 || (n_blocks > 0 && !d_out)) return fail(XTM_E_ARG, "bad arguments");
  if (n_blocks > (int64_t)1 << 40) return fail(XTM_E_ARG, "too many blocks");
  hipError_t e = launch_philox(seed, ctr0, n_blocks, d_out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "philox launch");
  return XTM_OK;
}

// ------------------------------------------------------ learned early stop
namespace {
float2* g_twiddle = nullptr;  // (cos, sin)(2 pi k / 512), k < 256
float* g_window = nullptr;    // sin^2(pi n / 512)

xtm_status fft_tables() {
  if (g_twiddle) return XTM_OK;
  std::vector<float2> tw(256);
  std::vector<float> win(512);
  for (int k = 0; k < 256; ++k) {
    tw[k].x = (float)std::cos(2.0 * M_PI * k / 512.0);
    tw[k].y = (float)std::sin(2.0 * M_PI * k / 512.0);
  }
  for (int n = 0; n < 512; ++n) {
    const double sn = std::sin(M_PI * n / 512.0);
    win[n] = (float)(sn * sn);
  }
  float2* t = nullptr;
  float* w = nullptr;
  if (hipMalloc(&t, 256 * sizeof(float2)) != hipSuccess ||
      hipMalloc(&w, 512 * sizeof(float)) != hipSuccess) {
    hipFree(t);
    return fail(XTM_E_NOMEM, "feature tables");
  }
  HIP_TRY(hipMemcpy(t, tw.data(), 256 * sizeof(float2), hipMemcpyHostToDevice), "tables");
  HIP_TRY(hipMemcpy(w, win.data(), 512 * sizeof(float), hipMemcpyHostToDevice), "tables");
  g_twiddle = t;
  g_window = w;
  return XTM_OK;
}
}  // namespace

xtm_status xtm_features(const float* d_record, int64_t n, const double twiss4[4], double emit,
                        double r_aperture, float* d_feat, void* stream) {
  return guarded([&]() -> xtm_status {
    if (n < 0 || !twiss4 || (n > 0 && (!d_record || !d_feat)))
      return fail(XTM_E_ARG, "bad feature arguments");
    if (!(twiss4[0] > 0) || !(twiss4[2] > 0) || !(emit > 0) || !(r_aperture > 0))
      return fail(XTM_E_ARG, "beta, emittance and aperture must be positive");
    xtm_status st = fft_tables();
    if (st != XTM_OK) return st;
    hipError_t e = launch_features(d_record, n, twiss4, emit, r_aperture, g_twiddle, g_window,
                                   d_feat, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "features launch");
    return XTM_OK;
  });
}

xtm_status xtm_feature_stats(const float* d_feat, const int32_t* d_mask, int64_t n, float* d_norm,
                             void* stream) {
  if (n < 0 || !d_norm || (n > 0 && !d_feat)) return fail(XTM_E_ARG, "bad arguments");
  hipError_t e = launch_feature_stats(d_feat, d_mask, n, d_norm, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "feature stats launch");
  return XTM_OK;
}

xtm_status xtm_mlp_init(float* d_theta, uint64_t seed, void* stream) {
  if (!d_theta) return fail(XTM_E_ARG, "null parameters");
  hipError_t e = launch_mlp_init(d_theta, seed, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "mlp init launch");
  return XTM_OK;
}

xtm_status xtm_mlp_forward(const float* d_theta, const float* d_norm, const float* d_x, int64_t B,
                           float* d_logit, void* stream) {
  if (B < 0 || !d_theta || !d_norm || (B > 0 && (!d_x || !d_logit)))
    return fail(XTM_E_ARG, "bad arguments");
  hipError_t e = launch_mlp_forward(d_theta, d_norm, d_x, B, d_logit, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "mlp forward launch");
  return XTM_OK;
}

xtm_status xtm_mlp_workspace(int64_t B, int64_t* n_floats) {
  if (B < 0 || !n_floats) return fail(XTM_E_ARG, "bad arguments");
  *n_floats = mlp_workspace_floats(B);
  return XTM_OK;
}

xtm_status xtm_mlp_grad(const float* d_theta, const float* d_norm, const float* d_x,
                        const float* d_y, int64_t B, float pos_weight, float* d_grad,
                        float* d_loss, float* d_work, void* stream) {
  if (B <= 0 || !d_theta || !d_norm || !d_x || !d_y || !d_grad || !d_work)
    return fail(XTM_E_ARG, "bad arguments");
  hipError_t e = launch_mlp_grad(d_theta, d_norm, d_x, d_y, B, pos_weight, d_grad, d_loss, d_work,
                                 (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "mlp grad launch");
  return XTM_OK;
}

xtm_status xtm_mlp_grad_noalloc(const float* d_theta, const float* d_norm, const float* d_x,
                                const float* d_y, int64_t B, float pos_weight, float* d_grad,
                                float* d_loss, void* stream) {
  if (!d_theta || !d_norm || !d_x || !d_y || !d_grad) return fail(XTM_E_ARG, "bad arguments");
  if (B <= 0 || B > kMlpNoAllocMaxBatch)
    return fail(XTM_E_ARG, "batch must be 1.." + std::to_string(kMlpNoAllocMaxBatch) +
                               " rows for the allocation-free gradient");
  float* work = nullptr;
  hipError_t e = mlp_noalloc_workspace(&work);
  if (e != hipSuccess) return hip_fail(e, "fixed gradient workspace lookup");
  e = launch_mlp_grad(d_theta, d_norm, d_x, d_y, B, pos_weight, d_grad, d_loss, work,
                      (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "mlp grad launch");
  return XTM_OK;
}

xtm_status xtm_mlp_adam(float* d_theta, float* d_m, float* d_v, const float* d_grad, int32_t step,
                        float lr, void* stream) {
  if (!d_theta || !d_m || !d_v || !d_grad || step < 1) return fail(XTM_E_ARG, "bad arguments");
  hipError_t e = launch_adam(d_theta, d_m, d_v, d_grad, step, lr, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "adam launch");
  return XTM_OK;
}

xtm_status xtm_mlp_train(float* d_theta, float* d_m, float* d_v, const float* d_norm,
                         const float* d_x, const float* d_y, int64_t n, float pos_weight,
                         int32_t epochs, int32_t batch, float lr, uint64_t shuffle_seed,
                         int32_t* step, float* h_epoch_loss, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!d_theta || !d_m || !d_v || !d_norm || !d_x || !d_y || !step)
      return fail(XTM_E_ARG, "null argument");
    if (n < 1 || n > INT32_MAX || epochs < 0 || batch < 1 || *step < 0)
      return fail(XTM_E_ARG, "bad sizes");
    hipStream_t s = (hipStream_t)stream;
    const int64_t bmax = batch < n ? batch : n;
    const int64_t wf = mlp_workspace_floats(bmax);
    float *work = nullptr, *xb = nullptr, *yb = nullptr, *grad = nullptr, *loss = nullptr;
    int32_t* perm_d = nullptr;
    auto release = [&]() {
      hipFree(work); hipFree(xb); hipFree(yb); hipFree(grad); hipFree(loss); hipFree(perm_d);
    };
    if (hipMalloc(&work, wf * sizeof(float)) != hipSuccess ||
        hipMalloc(&xb, bmax * 16 * sizeof(float)) != hipSuccess ||
        hipMalloc(&yb, bmax * sizeof(float)) != hipSuccess ||
        hipMalloc(&grad, XTM_MLP_PARAMS * sizeof(float)) != hipSuccess ||
        hipMalloc(&loss, 4096 * sizeof(float)) != hipSuccess ||
        hipMalloc(&perm_d, n * sizeof(int32_t)) != hipSuccess) {
      release();
      return fail(XTM_E_NOMEM, "training buffers");
    }
    std::vector<int32_t> perm(n);
    std::mt19937_64 rng(shuffle_seed);
    const int64_t nb = (n + batch - 1) / batch;
    std::vector<float> lh;
    hipError_t e = hipSuccess;
    for (int32_t ep = 0; ep < epochs && e == hipSuccess; ++ep) {
      for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
      for (int64_t i = n - 1; i > 0; --i) {  // Fisher-Yates
        const int64_t j = (int64_t)(rng() % (uint64_t)(i + 1));
        std::swap(perm[i], perm[j]);
      }
      e = hipMemcpyAsync(perm_d, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s);
      for (int64_t b = 0; b < nb && e == hipSuccess; ++b) {
        const int64_t start = b * batch, B = (n - start < batch) ? n - start : batch;
        e = launch_gather_rows(d_x, d_y, perm_d + start, B, xb, yb, s);
        if (e == hipSuccess)
          e = launch_mlp_grad(d_theta, d_norm, xb, yb, B, pos_weight, grad,
                              loss + (b % 4096), work, s);
        if (e == hipSuccess) e = launch_adam(d_theta, d_m, d_v, grad, ++*step, lr, s);
      }
      // mean batch loss of the epoch (the permutation buffer is reused next epoch)
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess && h_epoch_loss) {
        const int64_t k = nb < 4096 ? nb : 4096;
        lh.resize(k);
        e = hipMemcpy(lh.data(), loss, k * sizeof(float), hipMemcpyDeviceToHost);
        double acc = 0.0;
        for (float v : lh) acc += v;
        h_epoch_loss[ep] = (float)(acc / (double)k);
      }
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) return hip_fail(e, "training");
    return XTM_OK;
  });
}

xtm_status xtm_select_threshold(const float* d_logit, const int32_t* d_label, int64_t n,
                                double max_false_rate, float* h_tau, double* h_false_rate,
                                int64_t* h_selected, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!h_tau || n < 0 || (n > 0 && (!d_logit || !d_label)))
      return fail(XTM_E_ARG, "bad arguments");
    std::vector<float> z(n);
    std::vector<int32_t> y(n);
    hipStream_t s = (hipStream_t)stream;
    if (n > 0) {
      HIP_TRY(hipMemcpyAsync(z.data(), d_logit, n * sizeof(float), hipMemcpyDeviceToHost, s), "copy");
      HIP_TRY(hipMemcpyAsync(y.data(), d_label, n * sizeof(int32_t), hipMemcpyDeviceToHost, s), "copy");
      HIP_TRY(hipStreamSynchronize(s), "synchronise");
    }
    std::vector<int64_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return z[a] > z[b]; });
    // walk thresholds downwards over distinct logits; keep the lowest that meets the budget
    float tau = INFINITY;
    double rate_at = 0.0;
    int64_t sel_at = 0, lost = 0;
    for (int64_t k = 0; k < n;) {
      int64_t j = k;
      while (j < n && z[order[j]] == z[order[k]]) {
        lost += (y[order[j]] == 0);
        ++j;
      }
      const double rate = (double)lost / (double)j;
      if (std::isfinite(z[order[k]]) && rate <= max_false_rate) {
        tau = z[order[k]];
        rate_at = rate;
        sel_at = j;
      }
      k = j;
    }
    *h_tau = tau;
    if (h_false_rate) *h_false_rate = rate_at;
    if (h_selected) *h_selected = sel_at;
    return XTM_OK;
  });
}

xtm_status xtm_dynamic_aperture(const int32_t* h_state, const double* h_radius, int32_t n_r,
                                int32_t n_theta, double* h_da) {
  if (!h_state || !h_radius || !h_da || n_r < 1 || n_theta < 1)
    return fail(XTM_E_ARG, "bad arguments");
  for (int32_t j = 0; j < n_theta; ++j) {
    double da = INFINITY;
    for (int32_t i = 0; i < n_r; ++i) {
      const int64_t k = (int64_t)j * n_r + i;
      if (h_state[k] <= 0 && h_radius[k] < da) da = h_radius[k];
    }
    h_da[j] = da;
  }
  return XTM_OK;
}

xtm_status xtm_retire(xtm_particles P, const float* d_logit, float logit_threshold,
                      uint64_t audit_seed, double audit_fraction, int32_t* d_audit_flags,
                      int64_t* h_retired, int64_t* h_audited, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!P || !d_logit) return fail(XTM_E_ARG, "null argument");
    if (!(audit_fraction >= 0.0) || audit_fraction > 1.0)
      return fail(XTM_E_ARG, "audit fraction must be in [0, 1]");
    if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
    hipStream_t s = (hipStream_t)stream;
    // audited iff word < ceil(fraction 2^32) (exact integer compare)
    const double th = std::ceil(audit_fraction * 4294967296.0);
    const unsigned int at = th >= 4294967295.0 ? 0xFFFFFFFFu : (unsigned int)th;
    unsigned int* counts = nullptr;
    if (hipMalloc(&counts, 2 * sizeof(unsigned int)) != hipSuccess)
      return fail(XTM_E_NOMEM, "retire counters");
    hipError_t e = hipMemsetAsync(counts, 0, 2 * sizeof(unsigned int), s);
    if (e == hipSuccess)
      e = launch_retire(soa_of(P), P->idx[P->cur], P->ctrl, P->alive_upper, d_logit,
                        logit_threshold, audit_seed, at, counts, d_audit_flags, s);
    // rebuild the alive list without the retired particles
    if (e == hipSuccess) e = launch_iota(P->idx[1 - P->cur], P->n, P->ctrl, (int32_t)P->n, P->turn, s);
    if (e == hipSuccess)
      e = launch_epilogue(P->idx[1 - P->cur], P->idx[P->cur], nullptr, P->n > 0 ? P->n : 1,
                          soa_of(P), P->ctrl, P->blockcnt, P->passes, 0, 0, 0, s);
    unsigned int hc[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hc, counts, sizeof hc, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(counts);
    if (e != hipSuccess) return hip_fail(e, "retire");
    if (h_retired) *h_retired = hc[0];
    if (h_audited) *h_audited = hc[1];
    int64_t alive = 0;
    return read_alive(P, s, &alive, nullptr);
  });
}

xtm_status xtm_photon_table(double* h_out, int32_t n) {
  return guarded([&]() -> xtm_status {
    if (!h_out || n != kPhotonTableNodes)
      return fail(XTM_E_ARG, "need an output of XTM_PHOTON_TABLE_NODES values");
    const std::vector<double>& t = photon_table_host();
    std::copy(t.begin(), t.end(), h_out);
    return XTM_OK;
  });
}

xtm_status xtm_rule_score(const float* d_feat, int64_t n, float* d_score, void* stream) {
  if (n < 0 || (n > 0 && (!d_feat || !d_score))) return fail(XTM_E_ARG, "bad arguments");
  hipError_t e = launch_rule_score(d_feat, n, d_score, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "rule score launch");
  return XTM_OK;
}

namespace {
// one-sided 95 % quantile of the standard normal distribution
constexpr double kAuditZ = 1.6448536269514722;

// Wilson's score interval, upper end: (p + z^2/2n + z sqrt(p(1-p)/n + z^2/4n^2)) / (1 + z^2/n)
double wilson_upper(int64_t k, int64_t n) {
  if (n <= 0) return 1.0;
  const double z2 = kAuditZ * kAuditZ, nn = (double)n;
  const double p = (double)k / nn;
  const double centre = p + z2 / (2.0 * nn);
  const double half = kAuditZ * std::sqrt(p * (1.0 - p) / nn + z2 / (4.0 * nn * nn));
  return std::min(1.0, (centre + half) / (1.0 + z2 / nn));
}
}  // namespace

xtm_status xtm_audit_upper_bound(int64_t n_lost, int64_t n_audited, double* out) {
  if (!out || n_lost < 0 || n_audited < 0 || n_lost > n_audited)
    return fail(XTM_E_ARG, "need 0 <= n_lost <= n_audited and an output");
  *out = wilson_upper(n_lost, n_audited);
  return XTM_OK;
}

xtm_status xtm_audit_verdict(xtm_particles P, const int32_t* d_audit_flags, double fallback_rate,
                             int64_t* h_audited, int64_t* h_lost, double* h_upper,
                             int32_t* h_fallback, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!P || (P->n > 0 && !d_audit_flags)) return fail(XTM_E_ARG, "null argument");
    if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> st((size_t)P->n), fl((size_t)P->n);
    if (P->n > 0) {
      HIP_TRY(hipMemcpyAsync(st.data(), P->a.state, P->n * sizeof(int32_t), hipMemcpyDeviceToHost,
                             s),
              "read states");
      HIP_TRY(hipMemcpyAsync(fl.data(), d_audit_flags, P->n * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s),
              "read audit flags");
    }
    HIP_TRY(hipStreamSynchronize(s), "synchronise");
    int64_t audited = 0, lost = 0, retired = 0;
    for (int64_t i = 0; i < P->n; ++i) {
      if (st[i] == 2) ++retired;
      if (fl[i] != 0) {
        ++audited;
        if (st[i] == 0 || st[i] == -1) ++lost;
      }
    }
    const double upper = wilson_upper(lost, audited);
    if (h_audited) *h_audited = audited;
    if (h_lost) *h_lost = lost;
    if (h_upper) *h_upper = upper;
    if (h_fallback) *h_fallback = (retired > 0 && upper > fallback_rate) ? 1 : 0;
    return XTM_OK;
  });
}

xtm_status xtm_resume_retired(xtm_lattice L, xtm_particles P, const xtm_track_opts* opts,
                              void* stream, xtm_track_stats* stats) {
  return guarded([&]() -> xtm_status {
    if (!L || !P) return fail(XTM_E_ARG, "null handle");
    if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
    if (opts && (opts->record_buf || opts->use_graph))
      return fail(XTM_E_ARG, "resuming retired particles takes no recorder and no graph");
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = P->n;
    const int32_t horizon = P->turn;
    std::vector<int32_t> st((size_t)n), at((size_t)n);
    if (n > 0) {
      HIP_TRY(hipMemcpyAsync(st.data(), P->a.state, n * sizeof(int32_t), hipMemcpyDeviceToHost, s),
              "read states");
      HIP_TRY(hipMemcpyAsync(at.data(), P->a.at_turn, n * sizeof(int32_t), hipMemcpyDeviceToHost,
                             s),
              "read turns");
    }
    HIP_TRY(hipStreamSynchronize(s), "synchronise");
    // retired slots ordered by the turn they were retired at, then by slot
    std::vector<std::pair<int32_t, int32_t>> ret;  // (turn, slot)
    for (int64_t i = 0; i < n; ++i)
      if (st[i] == 2) {
        if (at[i] > horizon) return fail(XTM_E_STATE, "a retired particle is ahead of the set");
        ret.push_back({at[i], (int32_t)i});
      }
    std::sort(ret.begin(), ret.end());
    xtm_track_opts o{};
    if (opts) o = *opts;
    int64_t passes = 0;
    int32_t launches = 0, variant = 0;
    double ms = 0.0;
    std::vector<int32_t> list;  // slots tracked together, ascending
    size_t g = 0;
    while (g < ret.size()) {
      const int32_t t = ret[g].first;
      // keep the resumed particles still alive, add this turn's group, in
      // slot order
      std::vector<int32_t> next;
      for (int32_t p : list)
        if (st[p] == 1) next.push_back(p);
      for (; g < ret.size() && ret[g].first == t; ++g) {
        st[ret[g].second] = 1;
        next.push_back(ret[g].second);
      }
      std::sort(next.begin(), next.end());
      list.swap(next);
      HIP_TRY(hipMemcpyAsync(P->a.state, st.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s),
              "write states");
      HIP_TRY(hipMemcpyAsync(P->idx[P->cur], list.data(), list.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, s),
              "write alive list");
      HIP_TRY(launch_iota(P->idx[P->cur], 0, P->ctrl, (int32_t)list.size(), t, s), "alive count");
      P->turn = t;
      P->alive_upper = (int64_t)list.size();
      const int32_t until = g < ret.size() ? ret[g].first : horizon;
      xtm_track_stats ts{};
      xtm_status r = run_turns(L, P, until - t, &o, s, &ts, false);
      if (r != XTM_OK) return r;
      passes += ts.passes;
      launches += ts.launches;
      variant = ts.variant;
      ms += ts.kernel_ms;
      if (n > 0)
        HIP_TRY(hipMemcpyAsync(st.data(), P->a.state, n * sizeof(int32_t), hipMemcpyDeviceToHost,
                               s),
                "read states");
      HIP_TRY(hipStreamSynchronize(s), "synchronise");
    }
    // every particle still alive is now at the horizon: rebuild the set's list
    HIP_TRY(launch_iota(P->idx[1 - P->cur], n, P->ctrl, (int32_t)n, horizon, s), "alive-list rebuild");
    HIP_TRY(launch_epilogue(P->idx[1 - P->cur], P->idx[P->cur], nullptr, n > 0 ? n : 1, soa_of(P),
                            P->ctrl, P->blockcnt, P->passes, 0, 0, 0, s),
            "alive-list rebuild");
    P->turn = horizon;
    P->alive_upper = n;
    int64_t alive = 0;
    xtm_status r = read_alive(P, s, &alive, nullptr);
    if (r != XTM_OK) return r;
    if (stats) {
      stats->passes = passes;
      stats->alive = alive;
      stats->launches = launches;
      stats->variant = variant;
      stats->kernel_ms = ms;
    }
    return XTM_OK;
  });
}

namespace {
bool is_ap_type(int32_t t) { return t == XTM_AP_CIRCLE || t == XTM_AP_ELLIPSE || t == XTM_AP_RECT; }
bool is_drift_type(int32_t t) { return t == XTM_DRIFT || t == XTM_DRIFT_EXPANDED; }

// Host geometry of the loss refinement: s of each element, the line frame of
// each element's entry coordinates (a shift d gives b += A d, a rotation by t
// gives A <- A R(t)^T), aperture polygons (rays from the aperture's origin at
// angles 2 pi k / M meeting its boundary, mapped to the line frame), table
// record positions, previous aperture and aperture ordinal of each element.
xtm_status build_refine_geometry(xtm_lattice_s* L, int32_t M) {
  const int32_t n = L->n_el;
  const auto& el = L->desc_h;
  std::vector<double> sv(n + 1), G(6 * (size_t)(n + 1));
  sv[0] = 0.0;
  G[0] = 1.0; G[1] = 0.0; G[2] = 0.0; G[3] = 1.0; G[4] = 0.0; G[5] = 0.0;
  for (int32_t e = 0; e < n; ++e) {
    sv[e + 1] = is_drift_type(el[e].type) ? sv[e] + el[e].length : sv[e];
    double a11 = G[6 * e], a12 = G[6 * e + 1], a21 = G[6 * e + 2], a22 = G[6 * e + 3];
    double b1 = G[6 * e + 4], b2 = G[6 * e + 5];
    if (el[e].type == XTM_XYSHIFT) {
      const double dx = el[e].p[0], dy = el[e].p[1];
      const double t1 = a11 * dx, t2 = a12 * dy, t3 = a21 * dx, t4 = a22 * dy;
      b1 = (t1 + t2) + b1;
      b2 = (t3 + t4) + b2;
    } else if (el[e].type == XTM_SROTATION) {
      const double c = std::cos(el[e].p[0]), sn = std::sin(el[e].p[0]);
      const double u11 = a11 * c, u12 = a12 * sn, u21 = a12 * c, u22 = a11 * sn;
      const double w11 = a21 * c, w12 = a22 * sn, w21 = a22 * c, w22 = a21 * sn;
      a11 = u11 + u12;
      a12 = u21 - u22;
      a21 = w11 + w12;
      a22 = w21 - w22;
    }
    double* g = &G[6 * (size_t)(e + 1)];
    g[0] = a11; g[1] = a12; g[2] = a21; g[3] = a22; g[4] = b1; g[5] = b2;
  }
  std::vector<int32_t> prev(n, -1), ord(n, -1), off_f(n), off_b(n);
  int32_t last = -1, n_ap = 0;
  for (int32_t e = 0; e < n; ++e)
    if (is_ap_type(el[e].type)) last = e;
  std::vector<double> poly;
  for (int32_t e = 0, pa = last; e < n; ++e) {
    if (!is_ap_type(el[e].type)) continue;
    prev[e] = pa;
    pa = e;
    ord[e] = n_ap++;
    const double* p = el[e].p;
    if (el[e].type == XTM_AP_RECT && !(p[0] < 0.0 && 0.0 < p[1] && p[2] < 0.0 && 0.0 < p[3]))
      return fail(XTM_E_UNSUPPORTED, "element " + std::to_string(e) +
                                         ": loss refinement needs the rectangle to contain its origin");
    const double* g = &G[6 * (size_t)e];
    for (int32_t k = 0; k < M; ++k) {
      const double ang = 2.0 * M_PI * (double)k / (double)M;
      const double c = std::cos(ang), sn = std::sin(ang);
      double rad;
      if (el[e].type == XTM_AP_CIRCLE) {
        rad = p[0];
      } else if (el[e].type == XTM_AP_ELLIPSE) {
        const double q = (c * c) / (p[0] * p[0]) + (sn * sn) / (p[1] * p[1]);
        rad = 1.0 / std::sqrt(q);
      } else {
        rad = INFINITY;
        if (c > 0.0) rad = std::fmin(rad, p[1] / c);
        if (c < 0.0) rad = std::fmin(rad, p[0] / c);
        if (sn > 0.0) rad = std::fmin(rad, p[3] / sn);
        if (sn < 0.0) rad = std::fmin(rad, p[2] / sn);
      }
      const double ux = rad * c, uy = rad * sn;
      const double t1 = g[0] * ux, t2 = g[1] * uy, t3 = g[2] * ux, t4 = g[3] * uy;
      poly.push_back((t1 + t2) + g[4]);
      poly.push_back((t3 + t4) + g[5]);
    }
  }
  // record positions: the backward table holds the elements in reverse order
  {
    size_t w = 0;
    for (int32_t e = 0; e < n; ++e) {
      off_f[e] = (int32_t)w;
      w += 1 + ((L->fwd_h[w] >> 16) & 0xffffu);
    }
    w = 0;
    for (int32_t j = 0; j < n; ++j) {
      off_b[n - 1 - j] = (int32_t)w;
      w += 1 + ((L->bwd_h[w] >> 16) & 0xffffu);
    }
  }
  const size_t nd = sv.size() + G.size() + poly.size();
  const size_t ni = 4 * (size_t)n;
  const size_t bytes = nd * sizeof(double) + ni * sizeof(int32_t);
  hipFree(L->refine_buf);
  L->refine_buf = nullptr;
  L->refine_M = 0;
  void* buf = nullptr;
  if (hipMalloc(&buf, bytes) != hipSuccess) return fail(XTM_E_NOMEM, "refinement geometry allocation");
  std::vector<unsigned char> h(bytes);
  unsigned char* q = h.data();
  auto put = [&](const void* src, size_t nb) { std::memcpy(q, src, nb); q += nb; };
  put(sv.data(), sv.size() * sizeof(double));
  put(G.data(), G.size() * sizeof(double));
  if (!poly.empty()) put(poly.data(), poly.size() * sizeof(double));
  put(off_f.data(), n * sizeof(int32_t));
  put(off_b.data(), n * sizeof(int32_t));
  put(prev.data(), n * sizeof(int32_t));
  put(ord.data(), n * sizeof(int32_t));
  if (hipMemcpy(buf, h.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    hipFree(buf);
    return fail(XTM_E_HIP, "refinement geometry copy");
  }
  RefineGeom& rg = L->refine;
  const double* d = (const double*)buf;
  rg.n_el = n;
  rg.M = M;
  rg.s = d;
  rg.G = d + sv.size();
  rg.poly = d + sv.size() + G.size();
  const int32_t* ip = (const int32_t*)(d + nd);
  rg.off_f = ip;
  rg.off_b = ip + n;
  rg.prev = ip + 2 * n;
  rg.ap_ord = ip + 3 * n;
  L->refine_buf = buf;
  L->refine_M = M;
  return XTM_OK;
}
}  // namespace

xtm_status xtm_refine_losses(xtm_lattice L, xtm_particles P, int32_t n_vertices, double ds,
                             int32_t n_bisect, double* d_s, double* d_x, double* d_y,
                             int32_t* d_tests, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L || !P) return fail(XTM_E_ARG, "null lattice or particle set");
    if (!P->initialised) return fail(XTM_E_STATE, "particle set not initialised");
    if (!same_ref(L->ref, P->ref)) return fail(XTM_E_REFERENCE, "reference mismatch");
    if (n_vertices < 4 || n_vertices > 4096) return fail(XTM_E_ARG, "n_vertices must be in 4..4096");
    if (!(ds > 0.0) || !std::isfinite(ds)) return fail(XTM_E_ARG, "ds must be finite and > 0");
    if (n_bisect < 0 || n_bisect > 60) return fail(XTM_E_ARG, "n_bisect must be in 0..60");
    if (P->n > 0 && (!d_s || !d_x || !d_y)) return fail(XTM_E_ARG, "null output array");
    if (L->n_el == 0) return fail(XTM_E_ARG, "empty lattice");
    for (int32_t e = 0; e < L->n_el; ++e)
      if (is_drift_type(L->desc_h[e].type) && std::fabs(L->desc_h[e].length) / ds > 1e8)
        return fail(XTM_E_ARG, "ds too small: more than 1e8 sub-steps in a drift");
    if (L->refine_M != n_vertices) {
      const xtm_status st = build_refine_geometry(L, n_vertices);
      if (st != XTM_OK) return st;
    }
    RefineGeom g = L->refine;
    g.ds = ds;
    g.n_bisect = n_bisect;
    HIP_TRY(launch_refine(L->fwd_d, L->bwd_d, g, soa_of(P), P->n, kref(L->ref, 0, 0), d_s, d_x,
                          d_y, d_tests, (hipStream_t)stream),
            "refinement launch");
    return XTM_OK;
  });
}

namespace {
// x = (I - A)^-1 b for a 4x4 A, Gaussian elimination with partial pivoting
bool solve_i_minus(const double A[4][4], const double b[4], double x[4]) {
  double m[4][5];
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) m[i][j] = (i == j ? 1.0 : 0.0) - A[i][j];
    m[i][4] = b[i];
  }
  for (int c = 0; c < 4; ++c) {
    int p = c;
    for (int i = c + 1; i < 4; ++i)
      if (std::fabs(m[i][c]) > std::fabs(m[p][c])) p = i;
    if (!(std::fabs(m[p][c]) > 0.0)) return false;
    if (p != c)
      for (int j = 0; j < 5; ++j) std::swap(m[p][j], m[c][j]);
    for (int i = c + 1; i < 4; ++i) {
      const double f = m[i][c] / m[c][c];
      for (int j = c; j < 5; ++j) m[i][j] -= f * m[c][j];
    }
  }
  for (int i = 3; i >= 0; --i) {
    double acc = m[i][4];
    for (int j = i + 1; j < 4; ++j) acc -= m[i][j] * x[j];
    x[i] = acc / m[i][i];
  }
  return true;
}
// One recorded turn (the coordinates at every element's entry and after the
// last): the generated recording kernel, compiled on the lattice's first
// call, or the element interpreter (k_record) for a line without a cell
// decomposition.  Both apply the same maps, so the records are the same.
// all_rows = false: only the row after the turn is needed (the generated
// kernel then stores only that row; the interpreter stores every row).
hipError_t record_turn(xtm_lattice_s* L, const double* d_in, int64_t n, double* d_out,
                       hipStream_t s, bool all_rows = true) {
  if (!L->rec_line.tried && L->n_el > 0) {
    L->rec_line.tried = true;
    build_record_kernel(L->fwd_h, L->n_el, &L->rec_line);
  }
  if (L->rec_line.ok)
    return launch_line_record(L->rec_line, L->n_el, d_in, n, d_out, all_rows,
                              kref(L->ref, 0, 0), s);
  return launch_record(L->fwd_d, L->fwd_seg_d, (int32_t)(L->fwd_seg_h.size() / 3), L->n_el, d_in,
                       n, d_out, kref(L->ref, 0, 0), s);
}
}  // namespace

xtm_status xtm_track_record(xtm_lattice L, const double* d_in, int64_t n, double* d_out,
                            void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L) return fail(XTM_E_ARG, "null lattice");
    if (n < 0 || n > 65536) return fail(XTM_E_ARG, "n must be in 0..65536");
    if (n > 0 && (!d_in || !d_out)) return fail(XTM_E_ARG, "null array");
    if (((uintptr_t)d_out & 15u) != 0) return fail(XTM_E_ARG, "d_out must be 16-byte aligned");
    HIP_TRY(record_turn(L, d_in, n, d_out, (hipStream_t)stream),
            "record launch");
    return XTM_OK;
  });
}

xtm_status xtm_twiss(xtm_lattice L, double delta0, double h, double hd, int32_t max_iter,
                     double tol, const double* co_guess, double* h_table,
                     xtm_twiss_summary* summary, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L) return fail(XTM_E_ARG, "null lattice");
    if (!h_table || !summary) return fail(XTM_E_ARG, "null output");
    if (!(h > 0.0) || !(hd > 0.0) || max_iter < 0 || !(tol >= 0.0) || !std::isfinite(delta0))
      return fail(XTM_E_ARG, "need h > 0, hd > 0, max_iter >= 0, tol >= 0, finite delta0");
    xtm_status st = XTM_OK;
    hipStream_t s = (hipStream_t)stream;
    const int32_t n_el = L->n_el;
    const int64_t np = 11;
    double* d_in = nullptr;
    double* d_out = nullptr;
    const size_t out_n = (size_t)(n_el + 1) * np * 6;
    if (hipMalloc(&d_in, np * 6 * sizeof(double)) != hipSuccess ||
        hipMalloc(&d_out, out_n * sizeof(double)) != hipSuccess) {
      hipFree(d_in);
      return fail(XTM_E_NOMEM, "twiss scratch allocation");
    }
    std::vector<double> out(out_n);
    auto run = [&](const double u[4], bool with_delta, bool all_rows) -> xtm_status {
      const int64_t m = with_delta ? 11 : 9;
      double c[11][6];
      for (int64_t r = 0; r < m; ++r) {
        for (int k = 0; k < 4; ++k) c[r][k] = u[k];
        c[r][4] = 0.0;
        c[r][5] = delta0;
      }
      for (int k = 0; k < 4; ++k) {
        c[1 + 2 * k][k] += h;
        c[2 + 2 * k][k] -= h;
      }
      if (with_delta) {
        c[9][5] = delta0 + hd;
        c[10][5] = delta0 - hd;
      }
      if (hipMemcpyAsync(d_in, c, m * 6 * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
        return fail(XTM_E_HIP, "twiss upload");
      if (record_turn(L, d_in, m, d_out, s, all_rows) != hipSuccess)
        return fail(XTM_E_HIP, "twiss record launch");
      const size_t first = all_rows ? 0 : (size_t)n_el * m * 6;
      const size_t cnt = (all_rows ? (size_t)(n_el + 1) : 1) * m * 6;
      if (hipMemcpyAsync(out.data() + first, d_out + first, cnt * sizeof(double),
                         hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return fail(XTM_E_HIP, "twiss download");
      return XTM_OK;
    };
    auto at = [&](int64_t m, int32_t e, int r, int k) {
      return out[((size_t)e * m + r) * 6 + k];
    };
    double u[4] = {0.0, 0.0, 0.0, 0.0};
    if (co_guess)
      for (int k = 0; k < 4; ++k) u[k] = co_guess[k];
    int32_t it = 0;
    double res = INFINITY, best = INFINITY;
    double J[4][4];
    for (;;) {
      st = run(u, false, false);
      if (st != XTM_OK) break;
      double F[4];
      for (int k = 0; k < 4; ++k)
        for (int i = 0; i < 4; ++i)
          J[i][k] = (at(9, n_el, 1 + 2 * k, i) - at(9, n_el, 2 + 2 * k, i)) / (2.0 * h);
      res = 0.0;
      for (int i = 0; i < 4; ++i) {
        F[i] = at(9, n_el, 0, i) - u[i];
        res = std::max(res, std::fabs(F[i]));
      }
      if (std::isnan(F[0] + F[1] + F[2] + F[3])) res = NAN;
      if (!(res > tol) || it >= max_iter || !(res < best)) break;
      best = res;
      double du[4];
      if (!solve_i_minus(J, F, du)) {
        st = fail(XTM_E_UNSUPPORTED, "closed orbit: singular I - J (integer tune)");
        break;
      }
      for (int k = 0; k < 4; ++k) u[k] = u[k] + du[k];
      ++it;
    }
    if (st == XTM_OK) st = run(u, true, true);
    if (st == XTM_OK) {
      // per-element maps, momentum columns, dispersion and uncoupled optics
      std::vector<double> M((size_t)(n_el + 1) * 16), md((size_t)(n_el + 1) * 4);
      for (int32_t e = 0; e <= n_el; ++e)
        for (int i = 0; i < 4; ++i) {
          for (int k = 0; k < 4; ++k)
            M[(size_t)e * 16 + i * 4 + k] =
                (at(11, e, 1 + 2 * k, i) - at(11, e, 2 + 2 * k, i)) / (2.0 * h);
          md[(size_t)e * 4 + i] = (at(11, e, 9, i) - at(11, e, 10, i)) / (2.0 * hd);
        }
      double Jt[4][4], eta0[4];
      for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k) Jt[i][k] = M[(size_t)n_el * 16 + i * 4 + k];
      if (!solve_i_minus(Jt, &md[(size_t)n_el * 4], eta0)) {
        st = fail(XTM_E_UNSUPPORTED, "dispersion: singular I - J (integer tune)");
      } else {
        double s_acc = 0.0;
        double q[2] = {0.0, 0.0};
        double b0[2], a0[2];
        for (int pl = 0; pl < 2 && st == XTM_OK; ++pl) {
          const int o = 2 * pl;
          const double a = Jt[o][o], b = Jt[o][o + 1], d = Jt[o + 1][o + 1];
          const double cmu = 0.5 * (a + d);
          if (!(1.0 - cmu * cmu > 0.0)) {
            st = fail(XTM_E_UNSUPPORTED, "unstable or half-integer/integer one-turn map");
            break;
          }
          const double smu = std::copysign(std::sqrt(1.0 - cmu * cmu), b);
          b0[pl] = b / smu;
          a0[pl] = (a - d) / (2.0 * smu);
        }
        if (st == XTM_OK) {
          double th_prev[2] = {0.0, 0.0}, mu[2] = {0.0, 0.0};
          for (int32_t e = 0; e <= n_el; ++e) {
            double* row = h_table + (size_t)e * 15;
            if (e > 0) {
              const auto& de = L->desc_h[e - 1];
              if (de.type == XTM_DRIFT || de.type == XTM_DRIFT_EXPANDED) s_acc = s_acc + de.length;
            }
            row[0] = s_acc;
            for (int k = 0; k < 4; ++k) row[1 + k] = at(11, e, 0, k);
            const double* Me = &M[(size_t)e * 16];
            for (int pl = 0; pl < 2; ++pl) {
              const int o = 2 * pl;
              const double p_ = Me[o * 4 + o], q_ = Me[o * 4 + o + 1];
              const double r_ = Me[(o + 1) * 4 + o], t_ = Me[(o + 1) * 4 + o + 1];
              const double bb = p_ * b0[pl] - q_ * a0[pl];
              const double beta = (bb * bb + q_ * q_) / b0[pl];
              const double alpha = -(bb * (r_ * b0[pl] - t_ * a0[pl]) + q_ * t_) / b0[pl];
              const double th = std::atan2(q_, bb);
              if (e > 0) {
                double dth = std::fmod(th - th_prev[pl], 2.0 * M_PI);
                if (dth < 0.0) dth += 2.0 * M_PI;
                mu[pl] = mu[pl] + dth;
              }
              th_prev[pl] = th;
              row[5 + 3 * pl] = beta;
              row[6 + 3 * pl] = alpha;
              row[7 + 3 * pl] = mu[pl];
            }
            for (int i = 0; i < 4; ++i) {
              double acc = 0.0;
              for (int j = 0; j < 4; ++j) acc += Me[i * 4 + j] * eta0[j];
              row[11 + i] = acc + md[(size_t)e * 4 + i];
            }
          }
          q[0] = mu[0] / (2.0 * M_PI);
          q[1] = mu[1] / (2.0 * M_PI);
          summary->qx = q[0];
          summary->qy = q[1];
          for (int k = 0; k < 4; ++k) summary->co[k] = u[k];
          summary->iterations = it;
          summary->residual = res;
        }
      }
    }
    hipFree(d_in);
    hipFree(d_out);
    return st;
  });
}

namespace {
using cplx = std::complex<double>;

cplx det3(const cplx m[3][3]) {
  return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
         m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
         m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

// a null vector of the (numerically) rank-3 matrix J - lambda I: the row of
// cofactors with the largest norm (a column of the adjugate)
void null_vector(const double J[4][4], cplx lam, cplx v[4]) {
  cplx A[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) A[i][j] = cplx(J[i][j], 0.0) - (i == j ? lam : cplx(0.0, 0.0));
  double best = -1.0;
  for (int r = 0; r < 4; ++r) {
    cplx c[4];
    double nrm = 0.0;
    for (int col = 0; col < 4; ++col) {
      cplx m[3][3];
      for (int i = 0, ii = 0; i < 4; ++i) {
        if (i == r) continue;
        for (int j = 0, jj = 0; j < 4; ++j) {
          if (j == col) continue;
          m[ii][jj++] = A[i][j];
        }
        ++ii;
      }
      c[col] = ((r + col) % 2 ? -1.0 : 1.0) * det3(m);
      nrm += std::norm(c[col]);
    }
    if (nrm > best) {
      best = nrm;
      for (int k = 0; k < 4; ++k) v[k] = c[k];
    }
  }
}
}  // namespace

xtm_status xtm_twiss_coupled(xtm_lattice L, double delta0, double h, double hd, int32_t max_iter,
                             double tol, double* h_table, double* out_q, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L || !h_table || !out_q) return fail(XTM_E_ARG, "null lattice or output");
    const int32_t n_el = L->n_el;
    std::vector<double> base((size_t)(n_el + 1) * 15);
    xtm_twiss_summary sm{};
    xtm_status st = xtm_twiss(L, delta0, h, hd, max_iter, tol, nullptr, base.data(), &sm, stream);
    if (st != XTM_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    // the 9 probes around the closed orbit, one recorded turn
    double c[9][6];
    for (int r = 0; r < 9; ++r) {
      for (int k = 0; k < 4; ++k) c[r][k] = base[1 + k];
      c[r][4] = 0.0;
      c[r][5] = delta0;
    }
    for (int k = 0; k < 4; ++k) {
      c[1 + 2 * k][k] += h;
      c[2 + 2 * k][k] -= h;
    }
    const size_t out_n = (size_t)(n_el + 1) * 9 * 6;
    double* d_in = nullptr;
    double* d_out = nullptr;
    if (hipMalloc(&d_in, sizeof c) != hipSuccess || hipMalloc(&d_out, out_n * sizeof(double)) != hipSuccess) {
      hipFree(d_in);
      return fail(XTM_E_NOMEM, "coupled optics scratch allocation");
    }
    std::vector<double> out(out_n);
    if (hipMemcpyAsync(d_in, c, sizeof c, hipMemcpyHostToDevice, s) != hipSuccess ||
        record_turn(L, d_in, 9, d_out, s) != hipSuccess ||
        hipMemcpyAsync(out.data(), d_out, out_n * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(XTM_E_HIP, "coupled optics record");
    hipFree(d_in);
    hipFree(d_out);
    if (st != XTM_OK) return st;
    auto at = [&](int32_t e, int r, int k) { return out[((size_t)e * 9 + r) * 6 + k]; };
    std::vector<double> M((size_t)(n_el + 1) * 16);
    for (int32_t e = 0; e <= n_el; ++e)
      for (int i = 0; i < 4; ++i)
        for (int k = 0; k < 4; ++k)
          M[(size_t)e * 16 + i * 4 + k] = (at(e, 1 + 2 * k, i) - at(e, 2 + 2 * k, i)) / (2.0 * h);
    double J[4][4];
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 4; ++k) J[i][k] = M[(size_t)n_el * 16 + i * 4 + k];
    // eigenvalues: lambda + 1/lambda = t, t^2 - tr(J) t + (m2 - 2) = 0, m2 the
    // sum of the principal 2x2 minors
    double tr = 0.0, tr2 = 0.0;
    for (int i = 0; i < 4; ++i) {
      tr += J[i][i];
      for (int k = 0; k < 4; ++k) tr2 += J[i][k] * J[k][i];
    }
    const double m2 = 0.5 * (tr * tr - tr2);
    const double disc = tr * tr - 4.0 * (m2 - 2.0);
    if (!(disc >= 0.0)) return fail(XTM_E_UNSUPPORTED, "coupled optics: unstable one-turn map");
    const double t[2] = {0.5 * (tr + std::sqrt(disc)), 0.5 * (tr - std::sqrt(disc))};
    cplx modes[2][4];
    for (int m = 0; m < 2; ++m) {
      if (!(std::fabs(t[m]) < 2.0))
        return fail(XTM_E_UNSUPPORTED, "coupled optics: unstable or integer/half-integer mode");
      const double cm = 0.5 * t[m];
      cplx lam(cm, std::sqrt(1.0 - cm * cm));
      cplx v[4];
      null_vector(J, lam, v);
      // v^H S v with S = [[0,1,0,0],[-1,0,0,0],[0,0,0,1],[0,0,-1,0]]
      cplx q = std::conj(v[0]) * v[1] - std::conj(v[1]) * v[0] + std::conj(v[2]) * v[3] -
               std::conj(v[3]) * v[2];
      if (q.imag() < 0.0) {
        for (int k = 0; k < 4; ++k) v[k] = std::conj(v[k]);
        q = std::conj(q);
      }
      if (!(q.imag() > 0.0)) return fail(XTM_E_UNSUPPORTED, "coupled optics: degenerate mode");
      const double f = std::sqrt(2.0 / q.imag());
      for (int k = 0; k < 4; ++k) modes[m][k] = v[k] * f;
    }
    // propagate, label (x-like mode first), phases
    std::vector<cplx> ve[2];
    double xlike[2] = {0.0, 0.0};
    for (int m = 0; m < 2; ++m) {
      ve[m].resize((size_t)(n_el + 1) * 4);
      for (int32_t e = 0; e <= n_el; ++e) {
        const double* Me = &M[(size_t)e * 16];
        for (int i = 0; i < 4; ++i) {
          cplx acc(0.0, 0.0);
          for (int j = 0; j < 4; ++j) acc += Me[i * 4 + j] * modes[m][j];
          ve[m][(size_t)e * 4 + i] = acc;
        }
        xlike[m] += std::norm(ve[m][(size_t)e * 4]) - std::norm(ve[m][(size_t)e * 4 + 2]);
      }
    }
    const int order[2] = {xlike[0] >= xlike[1] ? 0 : 1, xlike[0] >= xlike[1] ? 1 : 0};
    for (int slot = 0; slot < 2; ++slot) {
      const auto& w = ve[order[slot]];
      const int comp = slot == 0 ? 0 : 2;
      double mu = 0.0, th_prev = 0.0;
      for (int32_t e = 0; e <= n_el; ++e) {
        double* row = h_table + (size_t)e * 7;
        row[0] = base[(size_t)e * 15];
        row[1 + 2 * slot] = std::norm(w[(size_t)e * 4]);
        row[2 + 2 * slot] = std::norm(w[(size_t)e * 4 + 2]);
        const double th = std::arg(w[(size_t)e * 4 + comp]);
        if (e > 0) {
          double d = std::fmod(th - th_prev, 2.0 * M_PI);
          if (d < 0.0) d += 2.0 * M_PI;
          const auto& de = L->desc_h[e - 1];
          const bool drift = (de.type == XTM_DRIFT || de.type == XTM_DRIFT_EXPANDED) && de.length > 0.0;
          if (!drift && d > M_PI) d -= 2.0 * M_PI;
          mu += d;
        }
        th_prev = th;
        row[5 + slot] = mu;
      }
      out_q[slot] = mu / (2.0 * M_PI);
    }
    return XTM_OK;
  });
}

xtm_status xtm_twiss_open(xtm_lattice L, double delta0, double h, double hd, const double* init,
                          double* h_table, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L || !init || !h_table) return fail(XTM_E_ARG, "null lattice, initial values or output");
    if (!(h > 0.0) || !(hd > 0.0) || !std::isfinite(delta0))
      return fail(XTM_E_ARG, "need h > 0, hd > 0, finite delta0");
    if (!(init[4] > 0.0) || !(init[6] > 0.0)) return fail(XTM_E_ARG, "initial betas must be > 0");
    const int32_t n_el = L->n_el;
    hipStream_t s = (hipStream_t)stream;
    double c[11][6];
    for (int r = 0; r < 11; ++r) {
      for (int k = 0; k < 4; ++k) c[r][k] = init[k];
      c[r][4] = 0.0;
      c[r][5] = delta0;
    }
    for (int k = 0; k < 4; ++k) {
      c[1 + 2 * k][k] += h;
      c[2 + 2 * k][k] -= h;
    }
    c[9][5] = delta0 + hd;
    c[10][5] = delta0 - hd;
    const size_t out_n = (size_t)(n_el + 1) * 11 * 6;
    double* d_in = nullptr;
    double* d_out = nullptr;
    if (hipMalloc(&d_in, sizeof c) != hipSuccess || hipMalloc(&d_out, out_n * sizeof(double)) != hipSuccess) {
      hipFree(d_in);
      return fail(XTM_E_NOMEM, "open-line optics scratch allocation");
    }
    std::vector<double> out(out_n);
    xtm_status st = XTM_OK;
    if (hipMemcpyAsync(d_in, c, sizeof c, hipMemcpyHostToDevice, s) != hipSuccess ||
        record_turn(L, d_in, 11, d_out, s) != hipSuccess ||
        hipMemcpyAsync(out.data(), d_out, out_n * sizeof(double), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      st = fail(XTM_E_HIP, "open-line optics record");
    hipFree(d_in);
    hipFree(d_out);
    if (st != XTM_OK) return st;
    auto at = [&](int32_t e, int r, int k) { return out[((size_t)e * 11 + r) * 6 + k]; };
    const double b0[2] = {init[4], init[6]}, a0[2] = {init[5], init[7]};
    double s_acc = 0.0, th_prev[2] = {0.0, 0.0}, mu[2] = {0.0, 0.0};
    for (int32_t e = 0; e <= n_el; ++e) {
      double Me[4][4], md[4];
      for (int i = 0; i < 4; ++i) {
        for (int k = 0; k < 4; ++k) Me[i][k] = (at(e, 1 + 2 * k, i) - at(e, 2 + 2 * k, i)) / (2.0 * h);
        md[i] = (at(e, 9, i) - at(e, 10, i)) / (2.0 * hd);
      }
      double* row = h_table + (size_t)e * 15;
      if (e > 0) {
        const auto& de = L->desc_h[e - 1];
        if (de.type == XTM_DRIFT || de.type == XTM_DRIFT_EXPANDED) s_acc = s_acc + de.length;
      }
      row[0] = s_acc;
      for (int k = 0; k < 4; ++k) row[1 + k] = at(e, 0, k);
      for (int pl = 0; pl < 2; ++pl) {
        const int o = 2 * pl;
        const double p_ = Me[o][o], q_ = Me[o][o + 1], r_ = Me[o + 1][o], t_ = Me[o + 1][o + 1];
        const double bb = p_ * b0[pl] - q_ * a0[pl];
        row[5 + 3 * pl] = (bb * bb + q_ * q_) / b0[pl];
        row[6 + 3 * pl] = -(bb * (r_ * b0[pl] - t_ * a0[pl]) + q_ * t_) / b0[pl];
        const double th = std::atan2(q_, bb);
        if (e > 0) {
          double d = std::fmod(th - th_prev[pl], 2.0 * M_PI);
          if (d < 0.0) d += 2.0 * M_PI;
          mu[pl] = mu[pl] + d;
        }
        th_prev[pl] = th;
        row[7 + 3 * pl] = mu[pl];
      }
      for (int i = 0; i < 4; ++i) {
        double acc = 0.0;
        for (int j = 0; j < 4; ++j) acc += Me[i][j] * init[8 + j];
        row[11 + i] = acc + md[i];
      }
    }
    return XTM_OK;
  });
}

namespace {
// One turn of m particles given in canonical coordinates (x, px, y, py, zeta,
// pzeta = ptau / beta0) through the tracker (RF included; the mean energy
// loss of radiating multipoles when rad = 1); returns the same coordinates
// after the turn and each particle's state.
xtm_status track_turn_canonical(xtm_lattice_s* L, int32_t rad, const std::vector<double>& u,
                                std::vector<double>* out, std::vector<int32_t>* state,
                                hipStream_t s) {
  const int64_t m = (int64_t)(u.size() / 6);
  Scratch sc;
  xtm_status st = make_scratch_n(m, L->ref, &sc);
  if (st != XTM_OK) return st;
  const double b0 = L->ref.beta0;
  std::vector<double> c(u);
  for (int64_t i = 0; i < m; ++i) {
    const double ptau = b0 * u[6 * i + 5];
    const double w = ptau * (ptau + 2.0 / b0);
    c[6 * i + 5] = w / (1.0 + std::sqrt(1.0 + w));
  }
  st = xtm_particles_init(sc.P, c.data(), 0, 0, s);
  if (st != XTM_OK) return st;
  xtm_track_opts o{};
  o.radiation = rad;
  o.variant = 4;
  st = run_turns(L, sc.P, 1, &o, s, nullptr, false);
  if (st != XTM_OK) return st;
  const xtm_arrays& a = sc.P->a;
  std::vector<double> f[6];
  double* src[6] = {a.x, a.px, a.y, a.py, a.zeta, a.ptau};
  for (int k = 0; k < 6; ++k) {
    f[k].resize(m);
    HIP_TRY(hipMemcpyAsync(f[k].data(), src[k], m * sizeof(double), hipMemcpyDeviceToHost, s),
            "read coordinates");
  }
  state->resize(m);
  HIP_TRY(hipMemcpyAsync(state->data(), a.state, m * sizeof(int32_t), hipMemcpyDeviceToHost, s),
          "read states");
  HIP_TRY(hipStreamSynchronize(s), "synchronise");
  out->resize(6 * m);
  for (int64_t i = 0; i < m; ++i) {
    for (int k = 0; k < 5; ++k) (*out)[6 * i + k] = f[k][i];
    (*out)[6 * i + 5] = f[5][i] / b0;
  }
  return XTM_OK;
}

// T(u) and the central-difference Jacobian at u: 13 particles (u, u +- h_j
// e_j) in one turn; with Richardson, also the steps h/2 (25 particles) and
// J = (4 J(h/2) - J(h)) / 3.
xtm_status map_and_jacobian(xtm_lattice_s* L, int32_t rad, const double u[6], const double h[6],
                            bool richardson, double Tu[6], double J[36], hipStream_t s) {
  const int n_steps = richardson ? 2 : 1;
  std::vector<double> in;
  for (int k = 0; k < 6; ++k) in.push_back(u[k]);
  for (int r = 0; r < n_steps; ++r)
    for (int j = 0; j < 6; ++j)
      for (int sg = 0; sg < 2; ++sg) {
        for (int k = 0; k < 6; ++k) in.push_back(u[k]);
        in[in.size() - 6 + j] += (sg == 0 ? 1.0 : -1.0) * h[j] / (r == 0 ? 1.0 : 2.0);
      }
  std::vector<double> out;
  std::vector<int32_t> st;
  xtm_status e = track_turn_canonical(L, rad, in, &out, &st, s);
  if (e != XTM_OK) return e;
  for (int32_t v : st)
    if (v != 1) return fail(XTM_E_UNSUPPORTED, "a probe particle was lost in one turn");
  for (int k = 0; k < 6; ++k) Tu[k] = out[k];
  double Jr[2][36];
  for (int r = 0; r < n_steps; ++r)
    for (int j = 0; j < 6; ++j) {
      const double hh = h[j] / (r == 0 ? 1.0 : 2.0);
      const size_t p = 6 * (1 + 12 * r + 2 * j), m = p + 6;
      for (int i = 0; i < 6; ++i) Jr[r][6 * i + j] = (out[p + i] - out[m + i]) / (2.0 * hh);
    }
  for (int i = 0; i < 36; ++i) J[i] = richardson ? (4.0 * Jr[1][i] - Jr[0][i]) / 3.0 : Jr[0][i];
  return XTM_OK;
}

bool solve6(const double A[36], const double b[6], double x[6]) {
  double a[6][7];
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j < 6; ++j) a[i][j] = A[6 * i + j];
    a[i][6] = b[i];
  }
  for (int k = 0; k < 6; ++k) {
    int p = k;
    for (int i = k + 1; i < 6; ++i)
      if (std::fabs(a[i][k]) > std::fabs(a[p][k])) p = i;
    if (a[p][k] == 0.0) return false;
    for (int j = 0; j < 7; ++j) std::swap(a[k][j], a[p][j]);
    for (int i = k + 1; i < 6; ++i) {
      const double f = a[i][k] / a[k][k];
      for (int j = k; j < 7; ++j) a[i][j] -= f * a[k][j];
    }
  }
  for (int k = 5; k >= 0; --k) {
    double sum = a[k][6];
    for (int j = k + 1; j < 6; ++j) sum -= a[k][j] * x[j];
    x[k] = sum / a[k][k];
  }
  return true;
}
}  // namespace

xtm_status xtm_twiss6d(xtm_lattice L, int32_t radiation, const double* h_steps, int32_t max_iter,
                       double tol, xtm_normal_form6* out, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L || !out) return fail(XTM_E_ARG, "null argument");
    if (radiation < 0 || radiation > 1) return fail(XTM_E_ARG, "radiation must be 0 or 1");
    if (max_iter < 0 || !(tol >= 0.0)) return fail(XTM_E_ARG, "need max_iter >= 0, tol >= 0");
    double h[6] = {1e-7, 1e-9, 1e-7, 1e-9, 1e-6, 1e-8};
    if (h_steps)
      for (int k = 0; k < 6; ++k) {
        if (!(h_steps[k] > 0.0)) return fail(XTM_E_ARG, "steps must be positive");
        h[k] = h_steps[k];
      }
    hipStream_t s = (hipStream_t)stream;
    double u[6] = {0, 0, 0, 0, 0, 0}, Tu[6], J[36];
    double best = INFINITY, res = INFINITY;
    int32_t it = 0;
    for (;;) {
      xtm_status st = map_and_jacobian(L, radiation, u, h, false, Tu, J, s);
      if (st != XTM_OK) return st;
      double r[6];
      res = 0.0;
      for (int k = 0; k < 6; ++k) {
        r[k] = Tu[k] - u[k];
        res = std::max(res, std::fabs(r[k]));
      }
      if (res <= tol || res >= best || it >= max_iter) break;
      best = res;
      double A[36], du[6];
      for (int i = 0; i < 36; ++i) A[i] = (i % 7 == 0 ? 1.0 : 0.0) - J[i];
      if (!solve6(A, r, du)) return fail(XTM_E_UNSUPPORTED, "I - J is singular (integer tune)");
      for (int k = 0; k < 6; ++k) u[k] += du[k];
      ++it;
    }
    xtm_status st = map_and_jacobian(L, radiation, u, h, true, Tu, J, s);
    if (st != XTM_OK) return st;
    NormalForm6 nf{};
    for (int k = 0; k < 6; ++k) nf.co[k] = u[k];
    if (!normal_form6(J, &nf))
      return fail(XTM_E_UNSUPPORTED, "the one-turn map has a real eigenvalue (unstable plane)");
    std::memcpy(out->co, nf.co, sizeof out->co);
    std::memcpy(out->J, J, sizeof out->J);
    std::memcpy(out->lam_re, nf.lam_re, sizeof out->lam_re);
    std::memcpy(out->lam_im, nf.lam_im, sizeof out->lam_im);
    std::memcpy(out->q, nf.q, sizeof out->q);
    std::memcpy(out->damping, nf.damping, sizeof out->damping);
    std::memcpy(out->v_re, nf.v_re, sizeof out->v_re);
    std::memcpy(out->v_im, nf.v_im, sizeof out->v_im);
    out->iterations = it;
    out->pad = 0;
    out->residual = res;
    return XTM_OK;
  });
}

xtm_status xtm_normal_form_of_map(const double* J, xtm_normal_form6* out) {
  return guarded([&]() -> xtm_status {
    if (!J || !out) return fail(XTM_E_ARG, "null argument");
    NormalForm6 nf{};
    if (!normal_form6(J, &nf))
      return fail(XTM_E_UNSUPPORTED, "the map has a real eigenvalue (unstable plane)");
    std::memset(out, 0, sizeof *out);
    std::memcpy(out->J, J, sizeof out->J);
    std::memcpy(out->lam_re, nf.lam_re, sizeof out->lam_re);
    std::memcpy(out->lam_im, nf.lam_im, sizeof out->lam_im);
    std::memcpy(out->q, nf.q, sizeof out->q);
    std::memcpy(out->damping, nf.damping, sizeof out->damping);
    std::memcpy(out->v_re, nf.v_re, sizeof out->v_re);
    std::memcpy(out->v_im, nf.v_im, sizeof out->v_im);
    return XTM_OK;
  });
}

xtm_status xtm_matched_gaussian(const xtm_normal_form6* nf, const xtm_reference* ref,
                                const double eps[3], const double* h_gauss, int64_t n,
                                double* h_out) {
  return guarded([&]() -> xtm_status {
    if (!nf || !ref || !eps || n < 0 || (n > 0 && (!h_gauss || !h_out)))
      return fail(XTM_E_ARG, "null argument or negative count");
    for (int k = 0; k < 3; ++k)
      if (!(eps[k] >= 0.0)) return fail(XTM_E_ARG, "emittances must be >= 0");
    RefQ r;
    if (!make_ref(ref, &r)) return fail(XTM_E_REFERENCE, "mass and p0c must be positive");
    NormalForm6 f{};
    std::memcpy(f.co, nf->co, sizeof f.co);
    std::memcpy(f.v_re, nf->v_re, sizeof f.v_re);
    std::memcpy(f.v_im, nf->v_im, sizeof f.v_im);
    matched_gaussian(f, r.beta0, eps, h_gauss, n, h_out);
    return XTM_OK;
  });
}

xtm_status xtm_chromaticity(xtm_lattice L, double delta0, double eps, double h, double hd,
                            int32_t max_iter, double tol, double* out_dq, void* stream) {
  return guarded([&]() -> xtm_status {
    if (!L || !out_dq) return fail(XTM_E_ARG, "null lattice or output");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(XTM_E_ARG, "eps must be finite and > 0");
    std::vector<double> table((size_t)(L->n_el + 1) * 15);
    xtm_twiss_summary sp{}, sm{};
    xtm_status st = xtm_twiss(L, delta0 + eps, h, hd, max_iter, tol, nullptr, table.data(), &sp,
                              stream);
    if (st != XTM_OK) return st;
    st = xtm_twiss(L, delta0 - eps, h, hd, max_iter, tol, nullptr, table.data(), &sm, stream);
    if (st != XTM_OK) return st;
    out_dq[0] = (sp.qx - sm.qx) / (2.0 * eps);
    out_dq[1] = (sp.qy - sm.qy) / (2.0 * eps);
    return XTM_OK;
  });
}

xtm_status xtm_sync(void* stream) {
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "stream synchronise");
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "device error");
  return XTM_OK;
}

}  // extern "C"
