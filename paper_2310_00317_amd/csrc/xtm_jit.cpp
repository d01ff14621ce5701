// xtm_jit.cpp -- per-line tracking kernels generated and compiled at run time.
//
// The paper's tracker assembles and compiles one kernel that tracks the whole
// beam line.  On gfx950 the reason to do so is sharper than on a CPU: with
// one particle per lane and often fewer than two waves per SIMD, a generic
// element interpreter spends more issue slots on scalar dispatch (type
// decode, compare tree, loop control, register shuffling between switch arms)
// than on the FP64 maps.  Here the element-type sequence is cut into cells of
// a fixed period; each distinct cell signature ("kind") becomes one
// straight-line block of map calls with compile-time parameter offsets, and
// the kernel loops over the cells of a turn with one scalar branch per cell.
// Element parameters stay data (one array, read with scalar loads), so all
// lattices with the same structure share one compiled kernel.
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "xtm_internal.h"

namespace xtm {

static const char* kMapsSource =
#include "xtm_maps_src.inc"
    ;

namespace {

struct Compiled {
  hipModule_t module = nullptr;
  hipFunction_t fn = nullptr;
  std::string error;
};

std::mutex g_mu;
std::map<std::string, Compiled> g_cache;  // schedule + generated source -> compiled kernel

uint32_t sig_of(uint64_t h) { return (uint32_t)(h & 0xffffu); }  // kernel type | order << 8

struct Decomp {
  std::vector<std::vector<uint32_t>> kinds;  // element signatures of each kind
  std::vector<int32_t> cell_kind;            // kind of each cell, in line order
  std::vector<int32_t> cell_start;           // first element index of each cell
};

// Cover the line with cells: a repeating unit U of P elements wherever it
// matches, and the stretches in between ("gaps", e.g. a lone RF cavity or a
// cell whose sextupole slot holds a cavity) as further kinds, split into
// pieces of at most max_unit elements.  Among all units (P <= max_unit,
// every phase) keep the cover with the fewest cells whose distinct kinds
// need at most max_code elements of generated code.
constexpr int kMaxUnit = 24;
constexpr int kMaxCode = 48;
// the long-cell forms
constexpr int kLongUnit = 40;
constexpr int kLongCode = 64;
// the recording kernel buffers a cell's rows in LDS: at most 16 elements a
// cell (16 x 64 lanes x 48 bytes)
constexpr int kMaxRecordUnit = 16;

bool decompose(const std::vector<uint32_t>& sig, Decomp* out, int32_t max_unit = kMaxUnit,
               int32_t max_code = kMaxCode) {
  const int32_t E = (int32_t)sig.size();
  if (E == 0) return false;
  size_t best_cells = 0;
  int32_t best_code = 0;
  for (int32_t P = 1; P <= max_unit && P <= E; ++P) {
    for (int32_t o = 0; o < P && o + P <= E; ++o) {
      const uint32_t* U = &sig[o];
      std::map<std::vector<uint32_t>, int32_t> kinds;
      kinds.emplace(std::vector<uint32_t>(U, U + P), 0);
      int32_t code = P;
      Decomp d;
      d.kinds.push_back(std::vector<uint32_t>(U, U + P));
      bool ok = true;
      auto add = [&](int32_t start, int32_t len) {
        std::vector<uint32_t> t(sig.begin() + start, sig.begin() + start + len);
        auto it = kinds.find(t);
        if (it == kinds.end()) {
          code += len;
          it = kinds.emplace(t, (int32_t)d.kinds.size()).first;
          d.kinds.push_back(t);
        }
        d.cell_kind.push_back(it->second);
        d.cell_start.push_back(start);
      };
      auto flush = [&](int32_t g0, int32_t g1) {  // gap [g0, g1)
        for (int32_t s = g0; s < g1; s += max_unit) add(s, std::min(max_unit, g1 - s));
      };
      int32_t i = 0, gap = -1;
      while (i < E && ok) {
        if (i + P <= E && std::memcmp(&sig[i], U, P * sizeof(uint32_t)) == 0) {
          if (gap >= 0) flush(gap, i), gap = -1;
          d.cell_kind.push_back(0);
          d.cell_start.push_back(i);
          i += P;
        } else {
          if (gap < 0) gap = i;
          ++i;
        }
        if (code > max_code) ok = false;
      }
      if (ok && gap >= 0) flush(gap, E);
      if (!ok || code > max_code) continue;
      if (best_cells == 0 || d.cell_kind.size() < best_cells ||
          (d.cell_kind.size() == best_cells && code < best_code)) {
        best_cells = d.cell_kind.size();
        best_code = code;
        *out = d;
      }
    }
  }
  return best_cells > 0;
}

int32_t n_words(uint32_t s) {
  const uint32_t kt = s & 0xffu, order = (s >> 8) & 0xffu;
  switch (kt) {
    case K_DRIFT: case K_DRIFT_EXP: case K_AP_CIRC: return 1;
    case K_MULT: return 2 * ((int32_t)order + 1);
    case K_MULT_CURV: return 2 * ((int32_t)order + 1) + 3;
    case K_MULT_LR: return 2 * ((int32_t)order + 1) + 1;
    case K_RF: return 3;
    case K_SHIFT: case K_SROT: case K_AP_ELL: return 2;
    case K_AP_RECT: return 4;
    default: return 0;
  }
}

// C++ statement applying one element whose parameters are P[0..] where P is
// the expression `arr` (an LDS pointer "p + o" or a local array name); `j` is
// the expression of its position in the cell (the loss code is e0 + j).
// Loss handling (`mode`): kSaveAtLoss stores a failing lane's entry
// coordinates at the element; kMarkOnly only records the loss code (the cell
// is replayed for lanes lost in it, see generate); kReplay applies the map
// alone (the replay itself).
// kRecord: the maps for optics by tracking (apertures not applied; a lane
// whose drift finds no real longitudinal momentum keeps its entry
// coordinates and applies no further maps).
enum EmitMode { kSaveAtLoss = 0, kMarkOnly = 1, kReplay = 2, kRecord = 3 };

std::string emit(uint32_t s, const std::string& arr, const std::string& j, bool far_rf,
                 EmitMode mode) {
  const uint32_t kt = s & 0xffu, order = (s >> 8) & 0xffu;
  auto P = [&](int32_t m) { return "(" + arr + ")[" + std::to_string(m) + "]"; };
  std::ostringstream c;
  switch (kt) {
    case K_DRIFT: {
      // the drift record's order: the length's class for the short sequences
      const std::string any = std::to_string(order);
      if (mode == kReplay)
        c << "(void)xtmm::drift_exact(q, " << P(0) << ", " << any << ");";
      else if (mode == kRecord)
        c << "{ const xtmm::Pt q0_ = q; if (!xtmm::drift_exact(q, " << P(0) << ", " << any
          << ")) { q = q0_; alive = false; } }";
      else if (mode == kMarkOnly)
        c << "xtmm::mark(xtmm::drift_exact(q, " << P(0) << ", " << any << "), code, st, e0 + "
          << j << ", -1);";
      else
        // one rare branch per drift: operands outside the window take the
        // generic operations, and a lane lost here stores its entry state
        c << "{ const xtmm::DriftIn d_ = xtmm::drift_in(q); double lp_, dq_; bool f_; "
          << "xtmm::drift_quotients(" << P(0) << ", d_, " << any << ", lp_, dq_, f_); "
          << "if (!f_) { if (!(d_.pz2 > 0.0) && live) { SAVE(); code = e0 + " << j
          << "; st = -1; live = false; } xtmm::drift_generic(" << P(0)
          << ", d_, lp_, dq_); } xtmm::drift_apply(q, lp_, dq_); }";
      break;
    }
    case K_DRIFT_EXP:
      c << "xtmm::drift_expanded(q, " << P(0) << ");";
      break;
    case K_MULT:
      c << "{ double kx, ky; xtmm::multipole<" << order << ">(q, " << arr << ", kx, ky); }";
      break;
    case K_MULT_CURV: {
      const int32_t v = 2 * ((int32_t)order + 1);
      c << "{ double kx, ky; xtmm::multipole<" << order << ">(q, " << arr
        << ", kx, ky); xtmm::curvature(q, " << P(v) << ", " << P(v + 1) << ", " << P(v + 2)
        << "); RAD(kx, ky, " << P(v + 2) << ", " << j << "); }";
      break;
    }
    case K_MULT_LR: {
      const int32_t v = 2 * ((int32_t)order + 1);
      c << "{ double kx, ky; xtmm::multipole<" << order << ">(q, " << arr
        << ", kx, ky); RAD(kx, ky, " << P(v) << ", " << j << "); }";
      break;
    }
    case K_RF:
      c << (far_rf ? "xtmm::rf_far(q, " : "xtmm::rf(q, ") << P(0) << ", " << P(1) << ", " << P(2)
        << ", beta0, two_over_beta0);";
      break;
    case K_SHIFT:
      c << "xtmm::xyshift(q, " << P(0) << ", " << P(1) << ");";
      break;
    case K_SROT:
      c << "xtmm::srotation(q, " << P(0) << ", " << P(1) << ");";
      break;
    case K_AP_CIRC:
    case K_AP_ELL:
    case K_AP_RECT: {
      if (mode == kReplay || mode == kRecord) break;  // a test, no change of coordinates
      std::string test;
      if (kt == K_AP_CIRC) test = "xtmm::in_circle(q, " + P(0) + ")";
      else if (kt == K_AP_ELL) test = "xtmm::in_ellipse(q, " + P(0) + ", " + P(1) + ")";
      else test = "xtmm::in_rect(q, " + P(0) + ", " + P(1) + ", " + P(2) + ", " + P(3) + ")";
      c << "{ const bool ok = " << test << "; ";
      if (mode == kSaveAtLoss)
        c << "if (!ok && live) { SAVE(); code = e0 + " << j << "; st = 0; live = false; } }";
      else
        c << "xtmm::mark(ok, code, st, e0 + " << j << ", 0); }";
      break;
    }
    default:
      break;  // marker
  }
  return c.str();
}

int32_t kind_words(const std::vector<uint32_t>& k) {
  int32_t w = 0;
  for (uint32_t s : k) w += n_words(s);
  return w;
}

// Generated kernel.  Per cell the workgroup holds the cell's parameters in
// one of two LDS slots: while the waves compute cell g from slot g&1, each
// thread has already loaded its share of cell g+1's parameters from global
// memory and writes it to the other slot before the cell barrier.  Element
// code then reads its parameters as broadcast LDS reads at compile-time
// offsets.
std::string generate(const Decomp& d, int32_t style, bool batched, int32_t rad_form) {
  int32_t maxw = 1;
  for (const auto& k : d.kinds) maxw = std::max(maxw, kind_words(k));
  // the lanes of a workgroup share one LDS slot pair, filled by all of them
  // and fenced by workgroup barriers (line_block: 256 lanes, or one wave)
  const int32_t lanes = line_block(style);
  // how element code reads its parameters from the slot (line_fetch):
  // 0 = at each use (the compiler interleaves the reads with the arithmetic),
  // 1 = all of an element's words in one group before its arithmetic,
  // 2 = the next element's group issued before the current element's
  //     arithmetic, so the read latency overlaps one element of work
  const int32_t fetch = line_fetch(style);
  // loss handling: at each loss test (a divergent store per test), or once
  // per cell (line_deferred: the tests only record the loss code; lanes lost
  // in the cell replay it afterwards)
  const bool deferred = line_deferred(style);
  // particles per lane (line_ppt): one, or two whose maps interleave
  const int32_t ppt = line_ppt(style);
  std::vector<uint32_t> sigs;  // distinct element signatures of the line
  std::string replay_tables;   // per kind: first entry; per entry: signature, offset
  if (deferred) {
    std::ostringstream kf, es, eo;
    int32_t n = 0;
    for (const auto& k : d.kinds) {
      kf << n << ", ";
      int32_t o = 0;
      for (uint32_t e : k) {
        size_t g = 0;
        while (g < sigs.size() && sigs[g] != e) ++g;
        if (g == sigs.size()) sigs.push_back(e);
        es << g << ", ";
        eo << o << ", ";
        o += n_words(e);
        ++n;
      }
    }
    kf << n;
    replay_tables = "__constant__ int kind_first[] = {" + kf.str() + "};\n"
                    "__constant__ int elem_sig[] = {" + es.str() + "};\n"
                    "__constant__ int elem_off[] = {" + eo.str() + "};\n";
  }
  // a kernel with radiation steps calls its RF sine out of line
  bool far_rf = false;
  if (rad_form != 0)
    for (const auto& k : d.kinds)
      for (uint32_t e : k) far_rf |= ((e & 0xffu) == K_MULT_CURV || (e & 0xffu) == K_MULT_LR);
  // the radiation step after a radiating multipole (rad_form): none; the
  // mean and Gaussian models with the mode read at run time; photon by photon
  std::string rad_macro;
  if (rad_form == 0)
    rad_macro = "#define RAD(kx, ky, lr, j) ((void)0)\n";
  else
    rad_macro = std::string("#define RAD(kx, ky, lr, j) xtmm::radiate_at<true, ") +
                (rad_form == 2 ? "true>(q, kx, ky, lr, 3, " : "false>(q, kx, ky, lr, r.rad_mode, ") +
                "r.seed, pid, \\\n"
                "    t0 + t, ec + (j), r.gamma0, r.c_mean, r.c_quant, r.p0c, beta0, two_over_beta0, "
                "\\\n"
                "    r.photon_table, r.c_nphot, r.c_ucrit)\n";
  const int32_t per_thread = (maxw + lanes - 1) / lanes;
  std::ostringstream s;
  s << "#include \"xtm_maps.h\"\n"
       "struct SoA { double *x, *px, *y, *py, *zeta, *delta, *ptau, *rpp, *rvv;\n"
       "             int *state, *at_element, *at_turn; long long* pid; };\n"
       "struct KRef { double beta0, two_over_beta0, gamma0, c_mean, c_quant, p0c;\n"
       "              unsigned long long seed; int rad_mode; int pad;\n"
       "              float* rec; int rec_turns; int rec_n;\n"
       "              const double* photon_table; double c_nphot, c_ucrit; };\n"
    << rad_macro <<
       "// a lane that fails a loss test stores the coordinates it entered the\n"
       "// element with (a rare, divergent store); the loss record follows at the end\n"
       "// (its slot index passes through a register move, so the nine store\n"
       "// addresses are formed on this rare path instead of held in registers)\n"
       "#define SAVE() do { int pj_; asm volatile(\"v_mov_b32 %0, %1\" : \"=v\"(pj_) : \"v\"(pi)); \\\n"
       "    P.x[pj_] = q.x; P.px[pj_] = q.px; P.y[pj_] = q.y; P.py[pj_] = q.py; \\\n"
       "    P.zeta[pj_] = q.zeta; P.delta[pj_] = q.delta; P.ptau[pj_] = q.ptau; \\\n"
       "    P.rpp[pj_] = q.rpp; P.rvv[pj_] = q.rvv; } while (0)\n"
       "#define MAXW " << maxw << "\n"
       "#define PER_THREAD " << per_thread << "\n"
       "#define LANES " << lanes << "\n"
       "#define PPT " << ppt << "\n"
       << replay_tables <<
       "extern \"C\" __global__ void __launch_bounds__(" << lanes << ")\n"
       "xtm_line(const double* __restrict__ " << (batched ? "prm_all" : "prm")
    << ", const int* __restrict__ cells, int n_cells,\n"
       "         int n_el, SoA P, const int* __restrict__ idx, const int* __restrict__ ctrl,\n"
       "         int n_turns, int backward, KRef r"
    << (batched ? ",\n         const int* __restrict__ first_slot, int nv, long long prm_stride"
                : "")
    << ") {\n";
  s << "  __shared__ double slot[2 * MAXW];\n"
       "  const int lane = threadIdx.x;\n";
  // a batch of lattice variants with one cell structure: each slot belongs
  // to the variant whose slot range holds it; the wave makes one pass per
  // variant among its lanes (smallest first), reading that variant's
  // parameters, with the lanes of the other variants idle
  const std::string exit_stmt = batched ? "break;" : "return;";
  if (ppt == 1) {
    s << "  const int t0 = ctrl[1];\n"
         "  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;\n"
         "  const bool in_range = i < ctrl[0];\n"
         "  const int pi = in_range ? idx[i] : 0;\n";
    if (batched)
      s << "  const bool tracked0 = in_range && P.state[pi] == 1;\n"
           "  int v = 0x7fffffff;\n"
           "  if (tracked0) {\n"
           "    int lo = 0, hi = nv;\n"
           "    while (hi - lo > 1) { const int mid = (lo + hi) >> 1; "
           "if (first_slot[mid] <= pi) lo = mid; else hi = mid; }\n"
           "    v = lo;\n"
           "  }\n"
           "  bool pending = tracked0;\n"
           "  while (__any(pending)) {\n"
           "  int m_ = pending ? v : 0x7fffffff;\n"
           "  for (int o_ = 32; o_ > 0; o_ >>= 1) m_ = min(m_, __shfl_xor(m_, o_, 64));\n"
           "  const int vu = __builtin_amdgcn_readfirstlane(m_);\n"
           "  const bool tracked = pending && v == vu;\n"
           "  pending = pending && !tracked;\n"
           "  const double* __restrict__ prm = prm_all + (long long)vu * prm_stride;\n"
           "  do {\n";
    else
      s << "  const bool tracked = in_range && P.state[pi] == 1;\n";
    s << "  int code = tracked ? 0 : 1;\n"
         "  int st = 1;\n"
         "  bool live = tracked;\n";
    s << "  if (__syncthreads_and(code != 0)) " << exit_stmt << "\n";
    s << "  xtmm::Pt q;\n"
         "  q.x = P.x[pi]; q.px = P.px[pi]; q.y = P.y[pi]; q.py = P.py[pi]; q.zeta = P.zeta[pi];\n"
         "  q.delta = P.delta[pi]; q.ptau = P.ptau[pi]; q.rpp = P.rpp[pi]; q.rvv = P.rvv[pi];\n"
         "  const double beta0 = r.beta0, two_over_beta0 = r.two_over_beta0;\n"
         "  const long long pid = P.pid[pi];\n"
         "  xtmm::refresh(q, beta0);\n";
  } else {
    // two particles per lane: slots i0 and i0 + LANES of the workgroup's range
    s << "  const int t0 = ctrl[1];\n"
         "  const long long i0 = (long long)blockIdx.x * (PPT * LANES) + threadIdx.x;\n"
         "  bool in_range_[PPT];\n"
         "  int pi_[PPT];\n"
         "#pragma unroll\n"
         "  for (int k_ = 0; k_ < PPT; ++k_) {\n"
         "    in_range_[k_] = i0 + k_ * LANES < ctrl[0];\n"
         "    pi_[k_] = in_range_[k_] ? idx[i0 + k_ * LANES] : 0;\n"
         "  }\n"
         "  bool tracked_[PPT];\n";
    if (batched)
      s << "  int v_[PPT];\n"
           "  bool pending_[PPT];\n"
           "#pragma unroll\n"
           "  for (int k_ = 0; k_ < PPT; ++k_) {\n"
           "    const int pi = pi_[k_];\n"
           "    pending_[k_] = in_range_[k_] && P.state[pi] == 1;\n"
           "    v_[k_] = 0x7fffffff;\n"
           "    if (pending_[k_]) {\n"
           "      int lo = 0, hi = nv;\n"
           "      while (hi - lo > 1) { const int mid = (lo + hi) >> 1; "
           "if (first_slot[mid] <= pi) lo = mid; else hi = mid; }\n"
           "      v_[k_] = lo;\n"
           "    }\n"
           "  }\n"
           "  while (__any(pending_[0] || pending_[1])) {\n"
           "  int m_ = min(pending_[0] ? v_[0] : 0x7fffffff, pending_[1] ? v_[1] : 0x7fffffff);\n"
           "  for (int o_ = 32; o_ > 0; o_ >>= 1) m_ = min(m_, __shfl_xor(m_, o_, 64));\n"
           "  const int vu = __builtin_amdgcn_readfirstlane(m_);\n"
           "#pragma unroll\n"
           "  for (int k_ = 0; k_ < PPT; ++k_) {\n"
           "    tracked_[k_] = pending_[k_] && v_[k_] == vu;\n"
           "    pending_[k_] = pending_[k_] && !tracked_[k_];\n"
           "  }\n"
           "  const double* __restrict__ prm = prm_all + (long long)vu * prm_stride;\n"
           "  do {\n";
    else
      s << "#pragma unroll\n"
           "  for (int k_ = 0; k_ < PPT; ++k_) tracked_[k_] = in_range_[k_] && P.state[pi_[k_]] == 1;\n";
    s << "  int code_[PPT], st_[PPT];\n"
         "  bool live_[PPT];\n"
         "#pragma unroll\n"
         "  for (int k_ = 0; k_ < PPT; ++k_) {\n"
         "    code_[k_] = tracked_[k_] ? 0 : 1; st_[k_] = 1; live_[k_] = tracked_[k_];\n"
         "  }\n"
         "  if (__syncthreads_and(code_[0] != 0 && code_[1] != 0)) " << exit_stmt << "\n"
         "  const double beta0 = r.beta0, two_over_beta0 = r.two_over_beta0;\n"
         "  xtmm::Pt q_[PPT];\n"
         "  long long pid_[PPT];\n"
         "#pragma unroll\n"
         "  for (int k_ = 0; k_ < PPT; ++k_) {\n"
         "    xtmm::Pt& q = q_[k_];\n"
         "    const int pi = pi_[k_];\n"
         "    q.x = P.x[pi]; q.px = P.px[pi]; q.y = P.y[pi]; q.py = P.py[pi]; q.zeta = P.zeta[pi];\n"
         "    q.delta = P.delta[pi]; q.ptau = P.ptau[pi]; q.rpp = P.rpp[pi]; q.rvv = P.rvv[pi];\n"
         "    pid_[k_] = P.pid[pi];\n"
         "    xtmm::refresh(q, beta0);\n"
         "  }\n";
  }
  s <<        "  {\n"
       "    const int off0 = cells[1], nw0 = cells[3];\n"
       "    for (int w = lane; w < nw0; w += LANES) slot[w] = prm[off0 + w];\n"
       "  }\n";
  s << "  __syncthreads();\n";
  // the cell table read one record (kind, first word, first element, words)
  // at a time, one cell ahead: the current cell's record came with the
  // previous cell's, so a cell starts with one scalar load, not three in
  // sequence
  s << "  int b = 0;\n"
       "  const int4* __restrict__ cells4 = reinterpret_cast<const int4*>(cells);\n"
       "  int4 rc = cells4[0];\n"
       "  for (int t = 0; t < n_turns; ++t) {\n"
       "    const int enc_t = t * n_el + 1;\n";
  const std::string rec_body =
       "    if (r.rec && t0 + t < r.rec_turns && code == 0) {\n"
       "      const unsigned long long base = (unsigned long long)(t0 + t) * 4 * r.rec_n + pi;\n"
       "      r.rec[base] = (float)q.x;\n"
       "      r.rec[base + r.rec_n] = (float)q.px;\n"
       "      r.rec[base + 2ull * r.rec_n] = (float)q.y;\n"
       "      r.rec[base + 3ull * r.rec_n] = (float)q.py;\n"
       "    }\n";
  if (ppt == 1)
    s << rec_body;
  else
    s << "#pragma unroll\n"
         "    for (int k_ = 0; k_ < PPT; ++k_) {\n"
         "    const xtmm::Pt& q = q_[k_];\n"
         "    const int pi = pi_[k_], code = code_[k_];\n"
      << rec_body << "    }\n";
  s <<
       "    for (int c = 0; c < n_cells; ++c) {\n"
       "      const int cn = (c + 1 == n_cells) ? 0 : c + 1;\n"
       "      const int4 rn = cells4[cn];\n"
       "      const int offn = rn.y, nwn = rn.w;\n"
       "      // every lane loads (past the cell's words, its first word; the\n"
       "      // parameter array ends in a pad word): no branch around the loads\n"
       "      double pre[PER_THREAD];\n"
       "#pragma unroll\n"
       "      for (int k = 0; k < PER_THREAD; ++k) {\n"
       "        const int w = lane + k * LANES;\n"
       "        const double v_ = prm[offn + (w < nwn ? w : 0)];\n"
       "        pre[k] = (w < nwn) ? v_ : 0.0;\n"
       "      }\n"
       "      const int kind = rc.x;\n"
       "      const int ec = rc.z;\n"
       "      // slot base hidden behind a register move: element reads become\n"
       "      // base + immediate-offset LDS loads instead of hoisted constant selects\n"
       "      int base;\n"
       "      asm volatile(\"v_mov_b32 %0, %1\" : \"=v\"(base) : \"s\"(b * MAXW));\n"
       "      // (the mask tells the compiler the base is small and non-negative, which\n"
       "      // lets it fold the element offsets into the LDS instructions)\n"
       "      const double* p = &slot[base & 0x3fff];\n"
       "      // the cell's loss-code base lives in a VGPR so the per-element codes\n"
       "      // e0 + j are vector adds of literals, not hoisted scalar constants\n"
       "      int e0;\n"
       "      asm volatile(\"v_mov_b32 %0, %1\" : \"=v\"(e0) : \"s\"(enc_t + ec));\n";
  if (deferred)
    s << "      const int code_in = code;\n"
         "      const xtmm::Pt qc = q;\n";
  for (size_t k = 0; k < d.kinds.size(); ++k) {
    s << "      " << (k ? "else if" : "if") << " (kind == " << k << ") {\n";
    const auto& kd = d.kinds[k];
    std::vector<int32_t> off(kd.size() + 1, 0);
    for (size_t j = 0; j < kd.size(); ++j) off[j + 1] = off[j] + n_words(kd[j]);
    // registers of element j's parameters, loaded from the slot in one group
    auto load = [&](size_t j) {
      const int32_t nw = n_words(kd[j]);
      if (nw == 0) return;
      s << "        double w" << j << "[" << nw << "];\n"
        << "#pragma unroll\n"
        << "        for (int m = 0; m < " << nw << "; ++m) w" << j << "[m] = p[" << off[j]
        << " + m];\n";
    };
    // fetch 2: element m's words are read before element m - 1's arithmetic,
    // or, for an element of many words (a high-order multipole) after a
    // short test or frame change, before element m - 2's: the aperture's few
    // operations would not cover the multipole's reads.  (Reading a drift's
    // one word that early costs the saturated rings more registers than it
    // saves.)
    std::vector<size_t> read_before(kd.size(), 0);
    for (size_t m = 1; m < kd.size(); ++m) {
      const uint32_t kp = kd[m - 1] & 0xffu;
      const bool short_prev = kp == K_AP_CIRC || kp == K_AP_ELL || kp == K_AP_RECT ||
                              kp == K_SHIFT || kp == K_SROT || kp == K_MARKER;
      read_before[m] = (short_prev && m >= 2 && n_words(kd[m]) >= 8) ? m - 2 : m - 1;
    }
    if (fetch == 2 && !kd.empty()) load(0);
    for (size_t j = 0; j < kd.size(); ++j) {
      std::string arr = "p + " + std::to_string(off[j]);
      if (fetch == 1) {
        load(j);
        s << "        __builtin_amdgcn_sched_barrier(0);\n";
      } else if (fetch == 2) {
        for (size_t m = j + 1; m < kd.size() && m <= j + 2; ++m)
          if (read_before[m] == j) load(m);
        s << "        __builtin_amdgcn_sched_barrier(0);\n";
      }
      if (fetch != 0 && n_words(kd[j]) > 0) arr = "w" + std::to_string(j);
      const std::string stmt =
          emit(kd[j], arr, std::to_string(j), far_rf, deferred ? kMarkOnly : kSaveAtLoss);
      if (stmt.empty()) continue;
      if (ppt == 1) {
        s << "        " << stmt << "\n";
      } else {
        // the same element for each particle of the lane, through references
        // that give each copy the one-particle names
        for (int32_t k = 0; k < ppt; ++k)
          s << "        { xtmm::Pt& q = q_[" << k << "]; int& code = code_[" << k
            << "]; int& st = st_[" << k << "]; bool& live = live_[" << k
            << "]; (void)live; const int pi = pi_[" << k
            << "]; const long long pid = pid_[" << k << "]; (void)pid; (void)pi; " << stmt
            << " }\n";
      }
    }
    s << "      }\n";
  }
  if (deferred) {
    // one wave-uniform test per cell; a lane lost in the cell re-applies the
    // cell's maps up to its lost element from the cell-entry copy (the same
    // operations, so the same values) and stores those entry coordinates.
    // The replay walks the cell's element list with one switch over the
    // line's element signatures, so this rare path adds little code.
    s << "      if (__any(code != code_in)) {\n"
         "        if (code != code_in) {\n"
         "          const int jl = code - e0;\n"
         "          xtmm::Pt q = qc;\n"
         "          for (int j = kind_first[kind]; j < kind_first[kind] + jl; ++j) {\n"
         "            const double* pe = p + elem_off[j];\n"
         "            switch (elem_sig[j]) {\n";
    for (size_t g = 0; g < sigs.size(); ++g) {
      const std::string stmt = emit(sigs[g], "pe", "(j - kind_first[kind])", far_rf, kReplay);
      if (!stmt.empty()) s << "              case " << g << ": " << stmt << " break;\n";
    }
    s << "              default: break;\n"
         "            }\n"
         "          }\n"
         "          SAVE();\n"
         "        }\n"
         "      }\n";
  }
  s << "#pragma unroll\n"
       "      for (int k = 0; k < PER_THREAD; ++k) {\n"
       "        const int w = lane + k * LANES;\n"
       "        if (w < nwn) slot[(b ^ 1) * MAXW + w] = pre[k];\n"
       "      }\n"
       "      b ^= 1;\n"
       "      rc = rn;\n";
  s << "      __syncthreads();\n";
  s << "    }\n";
  if (ppt == 1)
    s << "    if (__syncthreads_and(code != 0)) break;\n";
  else
    s << "    if (__syncthreads_and(code_[0] != 0 && code_[1] != 0)) break;\n";
  const std::string store_body =
       "  if (code == 0) {\n"
       "    P.x[pi] = q.x; P.px[pi] = q.px; P.y[pi] = q.y; P.py[pi] = q.py; P.zeta[pi] = q.zeta;\n"
       "    P.delta[pi] = q.delta; P.ptau[pi] = q.ptau; P.rpp[pi] = q.rpp; P.rvv[pi] = q.rvv;\n"
       "    P.at_turn[pi] = backward ? t0 - n_turns : t0 + n_turns;\n"
       "    P.at_element[pi] = 0;\n"
       "  } else {\n"
       "    const int tl = (code - 1) / n_el, el = (code - 1) - tl * n_el;\n"
       "    P.state[pi] = st;\n"
       "    P.at_element[pi] = backward ? n_el - 1 - el : el;\n"
       "    P.at_turn[pi] = backward ? t0 - 1 - tl : t0 + tl;\n"
       "  }\n";
  s << "  }\n";
  if (ppt == 1)
    s << "  if (!tracked) " << exit_stmt << "\n" << store_body;
  else
    s << "#pragma unroll\n"
         "  for (int k_ = 0; k_ < PPT; ++k_) {\n"
         "  if (!tracked_[k_]) continue;\n"
         "  const xtmm::Pt& q = q_[k_];\n"
         "  const int pi = pi_[k_], code = code_[k_], st = st_[k_];\n"
      << store_body << "  }\n";
  if (batched)
    s << "  } while (0);\n"
         "  }\n";
  s << "}\n";
  return s.str();
}

// Generated recording kernel for optics by tracking: one turn of a few
// particles from their (x, px, y, py, zeta, delta), the coordinates stored at
// the entry of every element and after the last.  The cell structure,
// parameter staging (two LDS slots, the next cell's words loaded during the
// current cell) and element code are those of the tracking kernel's
// one-wave form with the next element's parameters read ahead; apertures are
// not applied, and a lane whose drift finds no real longitudinal momentum
// keeps its entry coordinates and applies no further maps.  The rows of a
// cell go to an LDS buffer and leave for global memory together at the
// cell's end, as contiguous runs written by all lanes.
std::string generate_record(const Decomp& d) {
  int32_t maxw = 1, maxk = 1;
  for (const auto& k : d.kinds) {
    maxw = std::max(maxw, kind_words(k));
    maxk = std::max(maxk, (int32_t)k.size());
  }
  constexpr int32_t lanes = 64;
  const int32_t per_thread = (maxw + lanes - 1) / lanes;
  std::ostringstream s;
  s << "#include \"xtm_maps.h\"\n"
       "struct KRef { double beta0, two_over_beta0, gamma0, c_mean, c_quant, p0c;\n"
       "              unsigned long long seed; int rad_mode; int pad;\n"
       "              float* rec; int rec_turns; int rec_n;\n"
       "              const double* photon_table; double c_nphot, c_ucrit; };\n"
       "#define RAD(kx, ky, lr, j) ((void)0)\n"
       "#define MAXW " << maxw << "\n"
       "#define MAXK " << maxk << "\n"
       "#define PER_THREAD " << per_thread << "\n"
       "#define LANES " << lanes << "\n"
       "// row j of the cell in the LDS buffer (every lane writes its own)\n"
       "#define REC(j) do { if (ALL) { double2* r_ = rows + ((j) * LANES + lane) * 3; \\\n"
       "    r_[0] = make_double2(q.x, q.px); r_[1] = make_double2(q.y, q.py); \\\n"
       "    r_[2] = make_double2(q.zeta, q.delta); } } while (0)\n"
       "// ALL: every row, else only the row after the turn (one kernel for both,\n"
       "// each body specialised)\n"
       "template <bool ALL>\n"
       "__device__ __forceinline__ void record_body(const double* __restrict__ prm,\n"
       "    const int* __restrict__ cells, int n_cells, int n_el, const double* __restrict__ c6,\n"
       "    long long n, double* __restrict__ out, const KRef& r, double* slot, double2* rows) {\n"
       "  const int lane = threadIdx.x;\n"
       "  const long long i0 = (long long)blockIdx.x * LANES;\n"
       "  const long long i = i0 + lane;\n"
       "  const bool act = i < n;\n"
       "  // the block's particles: its rows of one element are nb_ consecutive 48-byte rows\n"
       "  const int nb_ = (int)(n - i0 < LANES ? n - i0 : LANES);\n"
       "  double2* __restrict__ out2 = reinterpret_cast<double2*>(out);\n"
       "  const double beta0 = r.beta0, two_over_beta0 = r.two_over_beta0;\n"
       "  (void)two_over_beta0;\n"
       "  xtmm::Pt q{};\n"
       "  if (act) {\n"
       "    const double* c = c6 + 6 * i;\n"
       "    const double dl = c[5];\n"
       "    const double u = dl * (2.0 + dl);\n"
       "    q.x = c[0]; q.px = c[1]; q.y = c[2]; q.py = c[3]; q.zeta = c[4]; q.delta = dl;\n"
       "    q.ptau = beta0 * u / (1.0 + sqrt(1.0 + beta0 * beta0 * u));\n"
       "    q.rpp = 1.0 / (1.0 + dl);\n"
       "    q.rvv = (1.0 + dl) / (1.0 + beta0 * q.ptau);\n"
       "    xtmm::refresh(q, beta0);\n"
       "  }\n"
       "  bool alive = act;\n"
       "  // the coordinates have arrived before the cell loop: otherwise the\n"
       "  // loop's first uses of them would carry a wait for every load in\n"
       "  // flight, the next cell's parameters included, on every cell\n"
       "  __builtin_amdgcn_s_waitcnt(0);\n"
       "  {\n"
       "    const int off0 = cells[1], nw0 = cells[3];\n"
       "    for (int w = lane; w < nw0; w += LANES) slot[w] = prm[off0 + w];\n"
       "  }\n"
       "  // parameters two cells ahead: the words of cell c + 1 arrived during\n"
       "  // cell c - 1 (a lone wave reads each cell's words once, from beyond the\n"
       "  // L2, and one cell of work does not cover that latency).  Two register\n"
       "  // sets take turns, the loop body holding two cells, so no set is copied\n"
       "  // (a copy would wait for the loads in flight).\n"
       "  double preA[PER_THREAD], preB[PER_THREAD];\n"
       "  {\n"
       "    const int c1 = n_cells > 1 ? 1 : 0;\n"
       "    const int off1 = cells[4 * c1 + 1], nw1 = cells[4 * c1 + 3];\n"
       "#pragma unroll\n"
       "    for (int k = 0; k < PER_THREAD; ++k) {\n"
       "      const int w = lane + k * LANES;\n"
       "      preA[k] = (w < nw1) ? prm[off1 + w] : 0.0;\n"
       "    }\n"
       "  }\n"
       "  __syncthreads();\n"
       "  int b = 0;\n"
       "  for (int c = 0; c < n_cells; c += 2) {\n";
  // one cell cc = c + half: its words in slot b, the next cell's in `cur`,
  // the cell after that loaded into `nxt`
  auto cell = [&](int half, const char* cur, const char* nxt) {
    s << "  {\n"
         "    const int cc = c + " << half << ";\n"
         "    const int cn = (cc + 1 == n_cells) ? cc : cc + 1;\n"
         "    const int nwn = cells[4 * cn + 3];\n"
         "    const int c2 = (cc + 2 < n_cells) ? cc + 2 : n_cells - 1;\n"
         "    const int off2 = cells[4 * c2 + 1], nw2 = cells[4 * c2 + 3];\n"
         "    // every lane loads (a lane past the cell's words reads its first\n"
         "    // word, the parameter array ends in a pad word), so the loads are\n"
         "    // not under a branch and the waits for them can count\n"
         "#pragma unroll\n"
         "    for (int k = 0; k < PER_THREAD; ++k) {\n"
         "      const int w = lane + k * LANES;\n"
         "      const double v_ = prm[off2 + (w < nw2 ? w : 0)];\n"
         "      " << nxt << "[k] = (w < nw2) ? v_ : 0.0;\n"
         "    }\n"
         "    const int kind = cells[4 * cc];\n"
         "    const int ec = cells[4 * cc + 2];\n"
         "    const int len = (cc + 1 == n_cells ? n_el : cells[4 * (cc + 1) + 2]) - ec;\n"
         "    int base;\n"
         "    asm volatile(\"v_mov_b32 %0, %1\" : \"=v\"(base) : \"s\"(b * MAXW));\n"
         "    const double* p = &slot[base & 0x3fff];\n";
    for (size_t k = 0; k < d.kinds.size(); ++k) {
      s << "    " << (k ? "else if" : "if") << " (kind == " << k << ") {\n";
      const auto& kd = d.kinds[k];
      std::vector<int32_t> off(kd.size() + 1, 0);
      for (size_t j = 0; j < kd.size(); ++j) off[j + 1] = off[j] + n_words(kd[j]);
      auto load = [&](size_t j) {
        const int32_t nw = n_words(kd[j]);
        if (nw == 0) return;
        s << "      double w" << j << "[" << nw << "];\n"
          << "#pragma unroll\n"
          << "      for (int m = 0; m < " << nw << "; ++m) w" << j << "[m] = p[" << off[j]
          << " + m];\n";
      };
      if (!kd.empty()) load(0);
      for (size_t j = 0; j < kd.size(); ++j) {
        if (j + 1 < kd.size()) load(j + 1);
        s << "      __builtin_amdgcn_sched_barrier(0);\n";
        const std::string arr =
            n_words(kd[j]) > 0 ? "w" + std::to_string(j) : "p + " + std::to_string(off[j]);
        s << "      REC(" << j << ");\n";
        const std::string stmt = emit(kd[j], arr, std::to_string(j), false, kRecord);
        if (!stmt.empty()) s << "      if (alive) { " << stmt << " }\n";
      }
      s << "    }\n";
    }
    s << "#pragma unroll\n"
         "    for (int k = 0; k < PER_THREAD; ++k) {\n"
         "      const int w = lane + k * LANES;\n"
         "      if (w < nwn) slot[(b ^ 1) * MAXW + w] = " << cur << "[k];\n"
         "    }\n"
         "    b ^= 1;\n"
         "    __syncthreads();\n"
         "    if (ALL) {\n"
         "      // the cell's rows, element-major: len runs of nb_ rows of three\n"
         "      // 16-byte words, each run contiguous in the output\n"
         "      const int per = nb_ * 3;\n"
         "      for (int t = lane; t < len * per; t += LANES) {\n"
         "        const int er = t / per, rem = t - er * per;\n"
         "        const int pp = rem / 3, kk = rem - pp * 3;\n"
         "        out2[((unsigned long long)(ec + er) * n + i0 + pp) * 3 + kk] =\n"
         "            rows[(er * LANES + pp) * 3 + kk];\n"
         "      }\n"
         "      __syncthreads();\n"
         "    }\n"
         "  }\n";
  };
  cell(0, "preA", "preB");
  s << "  if (c + 1 < n_cells)\n";
  cell(1, "preB", "preA");
  s << "  }\n"
       "  if (act) {\n"
       "    double2* o_ = out2 + ((unsigned long long)n_el * n + i) * 3;\n"
       "    o_[0] = make_double2(q.x, q.px); o_[1] = make_double2(q.y, q.py);\n"
       "    o_[2] = make_double2(q.zeta, q.delta);\n"
       "  }\n"
       "}\n"
       "extern \"C\" __global__ void __launch_bounds__(64)\n"
       "xtm_record(const double* __restrict__ prm, const int* __restrict__ cells, int n_cells,\n"
       "           int n_el, const double* __restrict__ c6, long long n,\n"
       "           double* __restrict__ out, int all_rows, KRef r) {\n"
       "  __shared__ double slot[2 * MAXW];\n"
       "  __shared__ double2 rows[MAXK * LANES * 3];\n"
       "  if (all_rows) record_body<true>(prm, cells, n_cells, n_el, c6, n, out, r, slot, rows);\n"
       "  else record_body<false>(prm, cells, n_cells, n_el, c6, n, out, r, slot, rows);\n"
       "}\n";
  return s.str();
}

// ilp_sched: LLVM's instruction-level-parallelism scheduling strategy instead
// of the default occupancy-first one.  A particle's element chain is one
// dependent sequence and, in the tail of a dynamic-aperture scan, a wave is
// alone on its SIMD and waits on each result; the ILP schedule interleaves
// more of each element's independent operations at the cost of registers
// (the DA-ring kernel: 205 VGPRs against 175).
Compiled compile(const std::string& src, const char* name, bool ilp_sched) {
  Compiled out;
  hiprtcProgram prog;
  const char* hdr = kMapsSource;
  const char* hname = "xtm_maps.h";
  if (hiprtcCreateProgram(&prog, src.c_str(), "xtm_line.hip", 1, &hdr, &hname) != HIPRTC_SUCCESS) {
    out.error = "hiprtcCreateProgram failed";
    return out;
  }
  std::vector<const char*> opts = {"--offload-arch=gfx950", "-O3", "-std=c++17",
                                   "-ffp-contract=off", "-fno-fast-math", "-Xclang",
                                   "-target-feature", "-Xclang", "-packed-fp32-ops"};
  if (ilp_sched) {
    opts.push_back("-mllvm");
    opts.push_back("-amdgpu-sched-strategy=max-ilp");
  }
  hiprtcResult r = hiprtcCompileProgram(prog, (int)opts.size(), opts.data());
  if (r != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    out.error = "hiprtc: " + log;
    hiprtcDestroyProgram(&prog);
    return out;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  std::vector<char> code(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  if (hipModuleLoadData(&out.module, code.data()) != hipSuccess) {
    out.error = "hipModuleLoadData failed";
    return out;
  }
  if (hipModuleGetFunction(&out.fn, out.module, name) != hipSuccess) {
    out.error = "hipModuleGetFunction failed";
    out.fn = nullptr;
  }
  return out;
}

}  // namespace

namespace {
// Signature, parameter-word position and parameter words of each element of
// a host element table.
void split_table(const std::vector<uint64_t>& tab, int32_t n_el, std::vector<uint32_t>* sig,
                 std::vector<int32_t>* word_of, std::vector<double>* prm) {
  size_t off = 0;
  for (int32_t e = 0; e < n_el; ++e) {
    const uint64_t h = tab[off];
    const uint32_t nw = (uint32_t)((h >> 16) & 0xffffu);
    sig->push_back(sig_of(h));
    word_of->push_back((int32_t)prm->size());
    for (uint32_t w = 0; w < nw; ++w) {
      double d;
      std::memcpy(&d, &tab[off + 1 + w], 8);
      prm->push_back(d);
    }
    off += 1 + nw;
  }
}
}  // namespace

bool table_radiates(const std::vector<uint64_t>& tab, int32_t n_el) {
  size_t off = 0;
  for (int32_t e = 0; e < n_el && off < tab.size(); ++e) {
    const uint32_t kt = (uint32_t)(tab[off] & 0xffu);
    if (kt == K_MULT_CURV || kt == K_MULT_LR) return true;
    off += 1 + (size_t)((tab[off] >> 16) & 0xffffu);
  }
  return false;
}

bool build_line_kernel(const std::vector<uint64_t>& tab, int32_t n_el, int32_t style,
                       int32_t rad_form, LineKernel* k) {
  return build_line_kernel_multi({&tab}, n_el, style, false, rad_form, k);
}

namespace {
// Compile (or take from the cache) a generated kernel and upload its
// parameter array and cell table.
bool finish_kernel(const Decomp& d, const std::string& source, const char* name,
                   bool ilp_sched, const std::vector<int32_t>& word_of,
                   const std::vector<double>& prm, LineKernel* k) {
  k->source = source;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    const std::string key = (ilp_sched ? "ilp\n" : "default\n") + k->source;
    auto it = g_cache.find(key);
    if (it == g_cache.end()) it = g_cache.emplace(key, compile(k->source, name, ilp_sched)).first;
    if (!it->second.fn) {
      k->error = it->second.error;
      return false;
    }
    k->fn = it->second.fn;
  }
  std::vector<int32_t> cells;  // per cell: kind, first parameter word, first element, words
  for (size_t c = 0; c < d.cell_kind.size(); ++c) {
    cells.push_back(d.cell_kind[c]);
    cells.push_back(word_of[d.cell_start[c]]);
    cells.push_back(d.cell_start[c]);
    cells.push_back(kind_words(d.kinds[d.cell_kind[c]]));
  }
  k->period = (int32_t)d.kinds[0].size();
  k->n_cells = (int32_t)d.cell_kind.size();
  k->n_kinds = (int32_t)d.kinds.size();
  if (hipMalloc(&k->prm_d, prm.size() * sizeof(double)) != hipSuccess ||
      hipMalloc(&k->cells_d, cells.size() * sizeof(int32_t)) != hipSuccess ||
      hipMemcpy(k->prm_d, prm.data(), prm.size() * sizeof(double), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(k->cells_d, cells.data(), cells.size() * sizeof(int32_t),
                hipMemcpyHostToDevice) != hipSuccess) {
    k->error = "device allocation for the line kernel failed";
    free_line_kernel(k);
    return false;
  }
  k->ok = true;
  return true;
}
}  // namespace

bool build_line_kernel_multi(const std::vector<const std::vector<uint64_t>*>& tabs, int32_t n_el,
                             int32_t style, bool batched, int32_t rad_form, LineKernel* k) {
  std::vector<uint32_t> sig;
  std::vector<int32_t> word_of;  // parameter-array offset of each element
  std::vector<double> prm;
  sig.reserve(n_el);
  split_table(*tabs[0], n_el, &sig, &word_of, &prm);
  if (prm.empty()) prm.push_back(0.0);
  const size_t stride = prm.size();
  for (size_t v = 1; v < tabs.size(); ++v) {
    std::vector<uint32_t> sv;
    std::vector<int32_t> wv;
    std::vector<double> pv;
    split_table(*tabs[v], n_el, &sv, &wv, &pv);
    if (pv.empty()) pv.push_back(0.0);
    if (sv != sig || pv.size() != stride) {
      k->error = "lattice variant " + std::to_string(v) + " differs in element structure";
      return false;
    }
    prm.insert(prm.end(), pv.begin(), pv.end());
  }
  prm.push_back(0.0);  // pad word: the first word of a cell without words
  if (batched && line_block(style) != 64) {
    k->error = "batched per-line kernels use one-wave workgroups";
    return false;
  }
  Decomp d;
  if (!decompose(sig, &d, line_long(style) ? kLongUnit : kMaxUnit,
                 line_long(style) ? kLongCode : kMaxCode)) {
    k->error = "no cell decomposition within the code budget";
    return false;
  }
  k->style = style;
  k->batched = batched;
  k->nv = (int32_t)tabs.size();
  k->stride = (int64_t)stride;
  // single-lattice kernels take the ILP schedule (measured 2-4 % faster on
  // the DA ring and with the mean and Gaussian radiation, 1 % slower on a
  // saturated FODO ring); the batched ones (0.7 % slower with it on 64
  // variants) and the photon form (4 % slower) keep the default
  const bool ilp = !batched && rad_form != 2;
  return finish_kernel(d, generate(d, style, batched, rad_form), "xtm_line", ilp, word_of, prm,
                       k);
}

bool build_record_kernel(const std::vector<uint64_t>& tab, int32_t n_el, LineKernel* k) {
  std::vector<uint32_t> sig;
  std::vector<int32_t> word_of;
  std::vector<double> prm;
  split_table(tab, n_el, &sig, &word_of, &prm);
  prm.push_back(0.0);  // pad word: the first word of a cell without words
  Decomp d;
  if (!decompose(sig, &d, kMaxRecordUnit)) {
    k->error = "no cell decomposition within the code budget";
    return false;
  }
  k->style = 5;  // one-wave workgroups, the next element's parameters read ahead
  k->stride = (int64_t)prm.size();
  return finish_kernel(d, generate_record(d), "xtm_record", true, word_of, prm, k);
}

void free_line_kernel(LineKernel* k) {
  hipFree(k->prm_d);
  hipFree(k->cells_d);
  k->prm_d = nullptr;
  k->cells_d = nullptr;
  k->ok = false;
}

hipError_t launch_line(const LineKernel& k, int32_t n_el, SoA P, const int32_t* idx,
                       const int32_t* ctrl, int64_t grid_upper, int32_t block, int32_t n_turns,
                       int32_t backward, KernelRef r, hipStream_t s) {
  if (grid_upper <= 0 || n_turns <= 0) return hipSuccess;
  const double* prm = k.prm_d;
  const int32_t* cells = k.cells_d;
  int32_t n_cells = k.n_cells;
  void* args[] = {(void*)&prm, (void*)&cells, (void*)&n_cells, (void*)&n_el, (void*)&P,
                  (void*)&idx, (void*)&ctrl, (void*)&n_turns, (void*)&backward, (void*)&r};
  // the generated kernel stages each cell's parameters with the stride of
  // its style's fixed workgroup size (line_block)
  (void)block;
  const int32_t wg = line_block(k.style);
  const int64_t per_wg = (int64_t)wg * line_ppt(k.style);  // particles per workgroup
  const unsigned grid = (unsigned)((grid_upper + per_wg - 1) / per_wg);
  return hipModuleLaunchKernel(k.fn, grid, 1, 1, (unsigned)wg, 1, 1, 0, s, args, nullptr);
}

hipError_t launch_line_record(const LineKernel& k, int32_t n_el, const double* c6, int64_t n,
                              double* out, bool all_rows, KernelRef r, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const double* prm = k.prm_d;
  const int32_t* cells = k.cells_d;
  int32_t n_cells = k.n_cells;
  long long nn = (long long)n;
  int32_t all = all_rows ? 1 : 0;
  void* args[] = {(void*)&prm, (void*)&cells, (void*)&n_cells, (void*)&n_el, (void*)&c6,
                  (void*)&nn,  (void*)&out,   (void*)&all,     (void*)&r};
  const unsigned grid = (unsigned)((n + 63) / 64);
  return hipModuleLaunchKernel(k.fn, grid, 1, 1, 64, 1, 1, 0, s, args, nullptr);
}

hipError_t launch_line_batched(const LineKernel& k, int32_t n_el, SoA P, const int32_t* idx,
                               const int32_t* ctrl, int64_t grid_upper, int32_t n_turns,
                               int32_t backward, KernelRef r, const int32_t* first_slot,
                               hipStream_t s) {
  if (grid_upper <= 0 || n_turns <= 0) return hipSuccess;
  if (!k.batched) return hipErrorInvalidValue;
  const double* prm = k.prm_d;
  const int32_t* cells = k.cells_d;
  int32_t n_cells = k.n_cells, nv = k.nv;
  long long stride = (long long)k.stride;
  void* args[] = {(void*)&prm,  (void*)&cells, (void*)&n_cells, (void*)&n_el,
                  (void*)&P,    (void*)&idx,   (void*)&ctrl,    (void*)&n_turns,
                  (void*)&backward, (void*)&r, (void*)&first_slot, (void*)&nv, (void*)&stride};
  const int32_t wg = line_block(k.style);
  const int64_t per_wg = (int64_t)wg * line_ppt(k.style);  // particles per workgroup
  const unsigned grid = (unsigned)((grid_upper + per_wg - 1) / per_wg);
  return hipModuleLaunchKernel(k.fn, grid, 1, 1, (unsigned)wg, 1, 1, 0, s, args, nullptr);
}

}  // namespace xtm
