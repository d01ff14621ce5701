// xtm_kernels.hip -- gfx950 kernels of the thin-lattice FP64 tracker.
//
// One thread owns one particle.  Its nine FP64 coordinates live in VGPRs for
// the whole chunk of turns; the element table is walked with wave-uniform
// (scalar) loads, so element parameters land in SGPRs and the element switch
// is a scalar branch.  HBM is touched only at chunk boundaries (one
// coalesced-by-index load and store of the particle state).
//
// Maps (paper section "Lattice modelling and single particle tracking": thin
// elements, multipolar errors, tilts and misalignments as reference-frame
// changes; aperture checks stop lost particles, section "Particle-matter
// interaction and collimation studies").  Every fused multiply-add is an
// explicit fma(); everything else is a correctly rounded IEEE operation, and
// the library is built with -ffp-contract=off, so the operation order below
// is the rounding contract:
//   exact drift    pz = sqrt((1+d)^2 - px^2 - py^2), lp = L (1/pz),
//                  x = fma(px, lp, x), y = fma(py, lp, y),
//                  zeta = fma(lp, (d(2+d) - px^2 - py^2) (1/(1+pz)) - beta0 ptau, zeta)
//   expanded drift x = fma(px, L rpp, x), ...,
//                  zeta = fma(L, (d - beta0 ptau) rpp - 0.5 (px^2+py^2) rpp^3 (1+beta0 ptau), zeta)
//   multipole      Horner from the top order: b <- b z + c_n with
//                  re = fma(br, x, fma(-bi, y, cr)), im = fma(br, y, fma(bi, x, ci));
//                  px -= re, py += im  (c_n = (knl_n + i ksl_n)/n!)
//   RF             ptau += amp sin(phase - k zeta); delta = v/(1+sqrt(1+v)),
//                  v = ptau (ptau + 2/beta0); rpp = 1/(1+delta); rvv = (1+delta)/(1+beta0 ptau)
//   apertures      lost iff !(inside), so NaN is lost and the boundary survives
#include <mutex>

#include "xtm_internal.h"
#include "xtm_maps.h"

namespace xtm {

// ------------------------------------------------------------- particle init
__global__ void __launch_bounds__(256) k_init(const double* __restrict__ c6, int64_t n,
                                              int64_t first_id, SoA P, KernelRef r) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double* c = c6 + 6 * i;
  double d = c[5];
  // ptau from delta without cancellation: u = d(2+d), ptau = b0 u / (1 + sqrt(1 + b0^2 u))
  double u = d * (2.0 + d);
  double ptau = r.beta0 * u / (1.0 + sqrt(1.0 + r.beta0 * r.beta0 * u));
  P.x[i] = c[0];
  P.px[i] = c[1];
  P.y[i] = c[2];
  P.py[i] = c[3];
  P.zeta[i] = c[4];
  P.delta[i] = d;
  P.ptau[i] = ptau;
  P.rpp[i] = 1.0 / (1.0 + d);
  P.rvv[i] = (1.0 + d) / (1.0 + r.beta0 * ptau);
  P.state[i] = 1;
  P.at_element[i] = 0;
  P.at_turn[i] = 0;
  P.pid[i] = first_id + i;
}

__global__ void __launch_bounds__(256) k_iota(int32_t* idx, int64_t n, int32_t* ctrl,
                                              int32_t n_alive, int32_t turn) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) idx[i] = (int32_t)i;
  if (i == 0) {
    ctrl[0] = n_alive;
    ctrl[1] = turn;
    ctrl[2] = n_alive;
  }
}

// end of a chunk: the alive particles are dk turns further
__global__ void k_advance(int32_t* ctrl, int32_t dk) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctrl[1] += dk;
}

__global__ void k_fill_i64(int64_t* p, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ------------------------------------------------ track kernel, variant 4
// Branch-free loss handling.  A lane never stores while tracking: a failed
// check only records, in registers, the first loss (state and the position
// (turn, element) in the chunk), and the lane keeps computing on whatever its
// coordinates become.  At the end survivors store their state; lost
// particles store only the loss record, their coordinates stay at the chunk
// start, and k_replay re-tracks them to the loss point (the maps are
// deterministic, so the replayed coordinates are bitwise the ones the lane had
// when it was lost).  The element loop thus has no divergent control flow.
__device__ __forceinline__ void multipole_n(xtmm::Pt& q, const double* __restrict__ prm,
                                            uint32_t order, double& kx, double& ky) {
  switch (order) {
    case 0: xtmm::multipole<0>(q, prm, kx, ky); break;
    case 1: xtmm::multipole<1>(q, prm, kx, ky); break;
    case 2: xtmm::multipole<2>(q, prm, kx, ky); break;
    case 3: xtmm::multipole<3>(q, prm, kx, ky); break;
    case 4: xtmm::multipole<4>(q, prm, kx, ky); break;
    case 5: xtmm::multipole<5>(q, prm, kx, ky); break;
    case 6: xtmm::multipole<6>(q, prm, kx, ky); break;
    case 7: xtmm::multipole<7>(q, prm, kx, ky); break;
    case 8: xtmm::multipole<8>(q, prm, kx, ky); break;
    case 9: xtmm::multipole<9>(q, prm, kx, ky); break;
    default: xtmm::multipole<10>(q, prm, kx, ky); break;
  }
}

// radiation after a multipole of length lr (identity of the deviate: particle
// id, absolute turn, element index of the line as tracked, thick elements sliced)
__device__ __forceinline__ void maybe_radiate(xtmm::Pt& q, double kx, double ky, double lr,
                                              const KernelRef& r, long long pid, int turn,
                                              int element) {
  xtmm::radiate_at<true>(q, kx, ky, lr, r.rad_mode, r.seed, pid, turn, element, r.gamma0, r.c_mean,
                   r.c_quant, r.p0c, r.beta0, r.two_over_beta0, r.photon_table, r.c_nphot,
                   r.c_ucrit);
}

// kRad = false compiles the radiation step out, for kernels that always run
// with radiation off (optics by tracking, loss refinement): the photon
// emitter is an out-of-line call whose register and stack cost would
// otherwise be paid across their whole element loop.
template <bool kRad = true>
__device__ __forceinline__ void apply_elem(xtmm::Pt& q, uint32_t ktype, uint32_t order,
                                           const double* __restrict__ prm, const KernelRef& r,
                                           bool& ok, int& lost_state, long long pid, int turn,
                                           int element) {
  double kx, ky;
  ok = true;
  lost_state = 0;
  if (ktype == K_MULT_LR) {
    multipole_n(q, prm, order, kx, ky);
    if (kRad) maybe_radiate(q, kx, ky, prm[2 * (order + 1)], r, pid, turn, element);
    return;
  }
  if (ktype == K_MULT) {
    switch (order) {
      case 0: xtmm::multipole<0>(q, prm, kx, ky); break;
      case 1: xtmm::multipole<1>(q, prm, kx, ky); break;
      case 2: xtmm::multipole<2>(q, prm, kx, ky); break;
      case 3: xtmm::multipole<3>(q, prm, kx, ky); break;
      case 4: xtmm::multipole<4>(q, prm, kx, ky); break;
      case 5: xtmm::multipole<5>(q, prm, kx, ky); break;
      case 6: xtmm::multipole<6>(q, prm, kx, ky); break;
      case 7: xtmm::multipole<7>(q, prm, kx, ky); break;
      case 8: xtmm::multipole<8>(q, prm, kx, ky); break;
      case 9: xtmm::multipole<9>(q, prm, kx, ky); break;
      default: xtmm::multipole<10>(q, prm, kx, ky); break;
    }
    return;
  }
  switch (ktype) {
    case K_DRIFT:
      ok = xtmm::drift_exact(q, prm[0], (int)order);
      lost_state = -1;
      break;
    case K_AP_CIRC:
      ok = xtmm::in_circle(q, prm[0]);
      break;
    case K_DRIFT_EXP:
      xtmm::drift_expanded(q, prm[0]);
      break;
    case K_MULT_CURV: {
      multipole_n(q, prm, order, kx, ky);
      const double* cv = prm + 2 * (order + 1);
      xtmm::curvature(q, cv[0], cv[1], cv[2]);
      if (kRad) maybe_radiate(q, kx, ky, cv[2], r, pid, turn, element);
      break;
    }
    case K_RF:
      xtmm::rf(q, prm[0], prm[1], prm[2], r.beta0, r.two_over_beta0);
      break;
    case K_SHIFT:
      xtmm::xyshift(q, prm[0], prm[1]);
      break;
    case K_SROT:
      xtmm::srotation(q, prm[0], prm[1]);
      break;
    case K_AP_ELL:
      ok = xtmm::in_ellipse(q, prm[0], prm[1]);
      break;
    case K_AP_RECT:
      ok = xtmm::in_rect(q, prm[0], prm[1], prm[2], prm[3]);
      break;
    default:
      break;
  }
}

__device__ __forceinline__ void load_pt(const SoA& P, int32_t p, xtmm::Pt& q, double beta0) {
  q.x = P.x[p]; q.px = P.px[p]; q.y = P.y[p]; q.py = P.py[p]; q.zeta = P.zeta[p];
  q.delta = P.delta[p]; q.ptau = P.ptau[p]; q.rpp = P.rpp[p]; q.rvv = P.rvv[p];
  xtmm::refresh(q, beta0);
}

__device__ __forceinline__ void store_pt(const SoA& P, int32_t p, const xtmm::Pt& q) {
  P.x[p] = q.x; P.px[p] = q.px; P.y[p] = q.y; P.py[p] = q.py; P.zeta[p] = q.zeta;
  P.delta[p] = q.delta; P.ptau[p] = q.ptau; P.rpp[p] = q.rpp; P.rvv[p] = q.rvv;
}

// One chunk of n_turns for the lanes with `active` set (the others idle):
// element parameters through scalar loads (the table pointer is wave-uniform),
// a loss recorded in registers (code = turn * n_el + element + 1) and the
// coordinates at the lost element's entry restored afterwards by k_replay.
__device__ __forceinline__ void track_lanes(const uint64_t* __restrict__ tab, int32_t n_el,
                                            SoA P, int32_t p, bool active, int32_t t0,
                                            int32_t n_turns, int32_t backward,
                                            const KernelRef& r) {
  int code = active ? 0 : 1;
  int st = 1;
  if (__all(code != 0)) return;
  xtmm::Pt q;
  load_pt(P, p, q, r.beta0);
  const long long pid = P.pid[p];
  for (int32_t t = 0; t < n_turns; ++t) {
    uint32_t off = 0;
    const int enc0 = t * n_el + 1;
    if (r.rec && t0 + t < r.rec_turns && code == 0) {
      const size_t base = (size_t)(t0 + t) * 4 * r.rec_n + p;
      r.rec[base] = (float)q.x;
      r.rec[base + r.rec_n] = (float)q.px;
      r.rec[base + 2 * (size_t)r.rec_n] = (float)q.y;
      r.rec[base + 3 * (size_t)r.rec_n] = (float)q.py;
    }
    for (int32_t e = 0; e < n_el; ++e) {
      off = __builtin_amdgcn_readfirstlane(off);
      const uint64_t* w = tab + off;
      const uint64_t h = w[0];
      const double* __restrict__ prm = reinterpret_cast<const double*>(w + 1);
      bool ok;
      int ls;
      apply_elem(q, (uint32_t)(h & 0xffu), (uint32_t)((h >> 8) & 0xffu), prm, r, ok, ls, pid,
                 t0 + t, e);
      xtmm::mark(ok, code, st, enc0 + e, ls);
      off += 1 + (uint32_t)((h >> 16) & 0xffffu);
    }
    if (__all(code != 0)) break;
  }
  if (!active) return;
  if (code == 0) {
    store_pt(P, p, q);
    P.at_turn[p] = backward ? t0 - n_turns : t0 + n_turns;
    P.at_element[p] = 0;
  } else {
    const int32_t tl = (code - 1) / n_el, el = (code - 1) - tl * n_el;
    P.state[p] = st;
    P.at_element[p] = backward ? n_el - 1 - el : el;
    P.at_turn[p] = backward ? t0 - 1 - tl : t0 + tl;
  }
}

__global__ void __launch_bounds__(256) k_track4(const uint64_t* __restrict__ tab, int32_t n_el,
                                                SoA P, const int32_t* __restrict__ idx,
                                                const int32_t* __restrict__ ctrl, int32_t n_turns,
                                                int32_t backward, KernelRef r) {
  const int32_t t0 = ctrl[1];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in_range = i < ctrl[0];
  const int32_t p = in_range ? idx[i] : 0;
  const bool tracked = in_range && P.state[p] == 1;
  track_lanes(tab, n_el, P, p, tracked, t0, n_turns, backward, r);
}

// Variant of the slot: the v with first_slot[v] <= p < first_slot[v + 1].
__device__ __forceinline__ int32_t variant_of(const int32_t* __restrict__ first_slot, int32_t nv,
                                              int32_t p) {
  int32_t lo = 0, hi = nv;  // first_slot[lo] <= p < first_slot[hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (first_slot[mid] <= p) lo = mid; else hi = mid;
  }
  return lo;
}

// Batched form: the set's slots are split into nv contiguous variant ranges,
// each tracked through its own element table.  A wave whose lanes span k
// variants makes k passes, one per variant in ascending order, each with the
// other lanes idle; with order-preserving compaction only waves at a range
// boundary have k > 1.
__global__ void __launch_bounds__(256) k_track4_batched(const uint64_t* const* __restrict__ tabs,
                                                        const int32_t* __restrict__ first_slot,
                                                        int32_t nv, int32_t n_el, SoA P,
                                                        const int32_t* __restrict__ idx,
                                                        const int32_t* __restrict__ ctrl,
                                                        int32_t n_turns, int32_t backward,
                                                        KernelRef r) {
  const int32_t t0 = ctrl[1];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in_range = i < ctrl[0];
  const int32_t p = in_range ? idx[i] : 0;
  bool pending = in_range && P.state[p] == 1;
  const int32_t v = pending ? variant_of(first_slot, nv, p) : 0x7fffffff;
  while (__any(pending)) {
    // smallest pending variant of the wave
    int32_t m = pending ? v : 0x7fffffff;
    for (int off = 32; off > 0; off >>= 1) m = min(m, __shfl_xor(m, off, 64));
    const int32_t vu = __builtin_amdgcn_readfirstlane(m);
    const bool active = pending && v == vu;
    const uint64_t* tab = tabs[vu];
    track_lanes(tab, n_el, P, p, active, t0, n_turns, backward, r);
    pending = pending && !active;
  }
}

// Re-track particles lost during the chunk from their chunk-start state up to
// (not including) the element that lost them, and store those coordinates.
__device__ __forceinline__ void replay_one(const uint64_t* __restrict__ tab, int32_t n_el, SoA P,
                                           int32_t p, int32_t t0, int32_t backward,
                                           const KernelRef& r) {
  const int32_t at = P.at_turn[p], ae = P.at_element[p];
  const int32_t tl = backward ? t0 - 1 - at : at - t0;
  const int32_t el = backward ? n_el - 1 - ae : ae;
  int64_t remaining = (int64_t)tl * n_el + el;
  xtmm::Pt q;
  load_pt(P, p, q, r.beta0);
  const long long pid = P.pid[p];
  for (int32_t t = 0; t <= tl && remaining > 0; ++t) {
    uint32_t off = 0;
    for (int32_t e = 0; e < n_el && remaining > 0; ++e, --remaining) {
      const uint64_t* w = tab + off;
      const uint64_t h = w[0];
      bool ok;
      int ls;
      apply_elem(q, (uint32_t)(h & 0xffu), (uint32_t)((h >> 8) & 0xffu),
                 reinterpret_cast<const double*>(w + 1), r, ok, ls, pid,
                 backward ? t0 - 1 - t : t0 + t, e);
      off += 1 + (uint32_t)((h >> 16) & 0xffffu);
    }
  }
  store_pt(P, p, q);
}

// Every lane of a wave walks the same (turn, element) sequence from the
// chunk start, so the walk position is wave-uniform and the element records
// come through scalar loads; each lane applies the maps only until its own
// loss point, and the wave runs to the furthest loss point among its lanes.
__global__ void __launch_bounds__(256) k_replay(const uint64_t* __restrict__ tab, int32_t n_el,
                                                SoA P, const int32_t* __restrict__ lost,
                                                const int32_t* __restrict__ ctrl,
                                                int32_t backward, KernelRef r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < ctrl[3];
  if (__all(!act)) return;
  const int32_t t0 = ctrl[1];
  const int32_t p = act ? lost[i] : 0;
  int64_t remaining = 0;
  xtmm::Pt q;
  long long pid = 0;
  if (act) {
    const int32_t at = P.at_turn[p], ae = P.at_element[p];
    const int32_t tl = backward ? t0 - 1 - at : at - t0;
    const int32_t el = backward ? n_el - 1 - ae : ae;
    remaining = (int64_t)tl * n_el + el;
    load_pt(P, p, q, r.beta0);
    pid = P.pid[p];
  }
  int64_t m = remaining;
  for (int s = 32; s > 0; s >>= 1) {
    const int64_t o = __shfl_xor(m, s, 64);
    m = o > m ? o : m;
  }
  const uint32_t m_lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)m);
  const uint32_t m_hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)m >> 32));
  const int64_t wave_max = (int64_t)(((uint64_t)m_hi << 32) | m_lo);
  uint32_t off = 0;
  int32_t t = 0, e = 0;
  for (int64_t k = 0; k < wave_max; ++k) {
    off = __builtin_amdgcn_readfirstlane(off);
    const uint64_t* w = tab + off;
    const uint64_t h = w[0];
    if (k < remaining) {
      bool ok;
      int ls;
      apply_elem(q, (uint32_t)(h & 0xffu), (uint32_t)((h >> 8) & 0xffu),
                 reinterpret_cast<const double*>(w + 1), r, ok, ls, pid,
                 backward ? t0 - 1 - t : t0 + t, e);
    }
    off += 1 + (uint32_t)((h >> 16) & 0xffffu);
    if (++e == n_el) {
      e = 0;
      ++t;
      off = 0;
    }
  }
  if (act) store_pt(P, p, q);
}

__global__ void __launch_bounds__(256) k_replay_batched(const uint64_t* const* __restrict__ tabs,
                                                        const int32_t* __restrict__ first_slot,
                                                        int32_t nv, int32_t n_el, SoA P,
                                                        const int32_t* __restrict__ lost,
                                                        const int32_t* __restrict__ ctrl,
                                                        int32_t backward, KernelRef r) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ctrl[3]) return;
  const int32_t p = lost[i];
  replay_one(tabs[variant_of(first_slot, nv, p)], n_el, P, p, ctrl[1], backward, r);
}

// -------------------------------------------------------- chunk epilogue
// Block-wide exclusive scan of a 0/1 flag over kScanBlock threads (16 wave64s).
__device__ __forceinline__ int32_t block_rank(bool flag, int32_t* s_wave, int32_t* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const uint64_t m = __ballot(flag);
  const int32_t in_wave = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
  if (lane == 0) s_wave[wave] = __popcll(m);
  __syncthreads();
  int32_t before = 0, all = 0;
  const int nw = blockDim.x >> 6;
  for (int k = 0; k < nw; ++k) {
    const int32_t c = s_wave[k];
    before += (k < wave) ? c : 0;
    all += c;
  }
  *total = all;
  return before + in_wave;
}

// Pass 1: per-block counts of (alive, lost during this chunk) and the
// chunk's pass count.
__device__ __forceinline__ bool lost_in_chunk(int32_t at, int32_t t0, int32_t chunk_turns,
                                              int32_t backward) {
  return backward ? (at <= t0 - 1 && at >= t0 - chunk_turns) : (at >= t0 && at < t0 + chunk_turns);
}

__global__ void __launch_bounds__(kScanBlock) k_count(const int32_t* __restrict__ idx, SoA P,
                                                      int32_t* ctrl, int32_t* blockcnt,
                                                      unsigned long long* passes, int32_t n_el,
                                                      int32_t chunk_turns, int32_t backward) {
  const int32_t t0 = ctrl[1];
  __shared__ int32_t s_wave[kScanBlock / 64];
  __shared__ unsigned long long s_pass[kScanBlock / 64];
  const int32_t n_alive = ctrl[0];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool alive = false, gone = false;
  int64_t np = 0;
  if (i < n_alive) {
    const int32_t p = idx[i];
    const int32_t st = P.state[p];
    alive = (st == 1);
    if (alive) {
      np = (int64_t)chunk_turns * n_el;
    } else {
      const int32_t at = P.at_turn[p], ae = P.at_element[p];
      gone = lost_in_chunk(at, t0, chunk_turns, backward);
      if (gone)
        np = backward ? (int64_t)(t0 - 1 - at) * n_el + (n_el - ae)
                      : (int64_t)(at - t0) * n_el + ae + 1;
    }
  }
  int32_t total_alive, total_gone;
  block_rank(alive, s_wave, &total_alive);
  __syncthreads();
  block_rank(gone, s_wave, &total_gone);
  unsigned long long v = (unsigned long long)np;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) s_pass[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long sum = 0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) sum += s_pass[k];
    if (sum) atomicAdd(passes, sum);
    blockcnt[2 * blockIdx.x] = total_alive;
    blockcnt[2 * blockIdx.x + 1] = total_gone;
    if (blockIdx.x == 0) ctrl[2] = n_alive;  // count this epilogue scanned
  }
}

// Pass 2: order-preserving scatter of the alive entries (into idx_out, if
// given) and of the entries lost during the chunk (into lost_out); the last
// block writes the new alive count (ctrl[0]) and the lost count (ctrl[3]).
// It reads the old count from ctrl[2] (set by pass 1), so writing ctrl[0]
// cannot race with a reader of this launch.
__global__ void __launch_bounds__(kScanBlock) k_scatter(const int32_t* __restrict__ idx_in,
                                                        int32_t* __restrict__ idx_out,
                                                        int32_t* __restrict__ lost_out, SoA P,
                                                        int32_t* ctrl,
                                                        const int32_t* __restrict__ blockcnt,
                                                        int32_t chunk_turns, int32_t backward) {
  __shared__ int32_t s_wave[kScanBlock / 64];
  __shared__ int32_t s_red[2][kScanBlock / 64];
  const int32_t n_old = ctrl[2];
  const int32_t t0 = ctrl[1];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int32_t part_a = 0, part_g = 0;
  for (int32_t b = threadIdx.x; b < (int32_t)blockIdx.x; b += blockDim.x) {
    part_a += blockcnt[2 * b];
    part_g += blockcnt[2 * b + 1];
  }
  for (int off = 32; off > 0; off >>= 1) {
    part_a += __shfl_down(part_a, off, 64);
    part_g += __shfl_down(part_g, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    s_red[0][threadIdx.x >> 6] = part_a;
    s_red[1][threadIdx.x >> 6] = part_g;
  }
  __syncthreads();
  int32_t off_a = 0, off_g = 0;
  for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
    off_a += s_red[0][k];
    off_g += s_red[1][k];
  }
  bool alive = false, gone = false;
  int32_t p = 0;
  if (i < n_old) {
    p = idx_in[i];
    const int32_t st = P.state[p];
    alive = (st == 1);
    gone = !alive && lost_in_chunk(P.at_turn[p], t0, chunk_turns, backward);
  }
  int32_t total_a, total_g;
  const int32_t rank_a = block_rank(alive, s_wave, &total_a);
  __syncthreads();
  const int32_t rank_g = block_rank(gone, s_wave, &total_g);
  // either list is optional (the store-on-loss kernels keep no lost list)
  if (alive && idx_out) idx_out[off_a + rank_a] = p;
  if (gone && lost_out) lost_out[off_g + rank_g] = p;
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    if (idx_out) ctrl[0] = off_a + total_a;
    ctrl[3] = lost_out ? off_g + total_g : 0;
  }
}

// Raw Philox4x32-10 blocks: block j uses counter ctr0 + j (128-bit carry),
// key = (seed_lo, seed_hi).
__global__ void __launch_bounds__(256) k_philox(unsigned long long seed, uint32_t c0,
                                                uint32_t c1, uint32_t c2, uint32_t c3,
                                                int64_t n_blocks, uint32_t* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_blocks) return;
  const unsigned long long lo0 = ((unsigned long long)c1 << 32) | c0;
  const unsigned long long lo = lo0 + (unsigned long long)j;
  const unsigned long long hi = (((unsigned long long)c3 << 32) | c2) + (lo < lo0 ? 1ull : 0ull);
  xtmm::U4 c{(unsigned int)lo, (unsigned int)(lo >> 32), (unsigned int)hi,
             (unsigned int)(hi >> 32)};
  const xtmm::U4 w = xtmm::philox4x32_10(c, (unsigned int)seed, (unsigned int)(seed >> 32));
  out[4 * j] = w.a;
  out[4 * j + 1] = w.b;
  out[4 * j + 2] = w.c;
  out[4 * j + 3] = w.d;
}

// ------------------------------------------------ photon spectrum table
// The inverse photon spectrum of the photon-by-photon radiation model,
// uploaded from the host table at the first use on each device.  In host code
// `photon_table_dev` names a host-side stand-in: kernels receive the device
// address looked up with hipGetSymbolAddress.
static __device__ __align__(256) double photon_table_dev[kPhotonTableNodes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_photon_mu;
const double* g_photon_addr[kMaxDevices] = {};
}  // namespace

hipError_t photon_table_device(const double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  const std::vector<double>& host = photon_table_host();
  std::lock_guard<std::mutex> lock(g_photon_mu);
  if (!g_photon_addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(photon_table_dev));
    if (e != hipSuccess) return e;
    e = hipMemcpy(p, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return e;
    g_photon_addr[dev] = static_cast<const double*>(p);
  }
  *out = g_photon_addr[dev];
  return hipSuccess;
}

// ------------------------------------------------------------- launchers
hipError_t launch_philox(unsigned long long seed, const uint32_t ctr0[4], int64_t n_blocks,
                         uint32_t* out, hipStream_t s) {
  if (n_blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((n_blocks + 255) / 256)), dim3(256), 0, s, seed,
                     ctr0[0], ctr0[1], ctr0[2], ctr0[3], n_blocks, out);
  return hipGetLastError();
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

hipError_t launch_init(const double* coords6, int64_t n, int64_t first_id, SoA P, KernelRef r,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init, dim3(blocks_for(n, 256)), dim3(256), 0, s, coords6, n, first_id, P, r);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* idx, int64_t n, int32_t* ctrl, int32_t n_alive, int32_t turn,
                       hipStream_t s) {
  int64_t m = n > 0 ? n : 1;
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(m, 256)), dim3(256), 0, s, idx, n, ctrl, n_alive,
                     turn);
  return hipGetLastError();
}

hipError_t launch_advance(int32_t* ctrl, int32_t dk, hipStream_t s) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, s, ctrl, dk);
  return hipGetLastError();
}

hipError_t launch_fill_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

// ------------------------------------------------------ one launch per element
// Baseline for the persistent kernels, kept for measurement: element `e`
// (its record at word `off` of the table) is applied to every alive particle
// by a launch of its own, which reads from HBM the fields of the particle's
// state that the element's map uses and writes back the ones it changes
// (drift: reads x, px, y, py, zeta, delta, ptau, writes x, y, zeta;
// multipole: reads x, y, px, py, writes px, py; aperture: reads x, y; RF:
// reads zeta, ptau, writes ptau, delta, rpp, rvv; shift: x, y; rotation: x,
// px, y, py), plus the state word.  Other elements (bends with curvature,
// radiating multipoles, expanded drifts) read and write the whole state.  A
// particle failing the element's loss test keeps the coordinates it entered
// with (they are not written) and records the element and the turn.
__device__ __forceinline__ void elem_lost(const SoA& P, int64_t p, int st, int32_t e, int32_t turn) {
  P.state[p] = st;
  P.at_element[p] = e;
  P.at_turn[p] = turn;
}

template <uint32_t KT>
__global__ void __launch_bounds__(256) k_elem(const uint64_t* __restrict__ tab, uint32_t off,
                                              int32_t e, SoA P, int64_t n, int32_t turn,
                                              KernelRef r) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || P.state[p] != 1) return;
  const uint64_t h = tab[off];
  const uint32_t order = (uint32_t)((h >> 8) & 0xffu);
  const double* __restrict__ prm = reinterpret_cast<const double*>(tab + off + 1);
  xtmm::Pt q;
  if constexpr (KT == K_DRIFT) {
    q.x = P.x[p]; q.px = P.px[p]; q.y = P.y[p]; q.py = P.py[p]; q.zeta = P.zeta[p];
    q.delta = P.delta[p]; q.ptau = P.ptau[p];
    xtmm::refresh(q, r.beta0);
    if (!xtmm::drift_exact(q, prm[0], (int)order)) return elem_lost(P, p, -1, e, turn);
    P.x[p] = q.x; P.y[p] = q.y; P.zeta[p] = q.zeta;
  } else if constexpr (KT == K_MULT) {
    q.x = P.x[p]; q.y = P.y[p]; q.px = P.px[p]; q.py = P.py[p];
    double kx, ky;
    multipole_n(q, prm, order, kx, ky);
    P.px[p] = q.px; P.py[p] = q.py;
  } else if constexpr (KT == K_AP_CIRC || KT == K_AP_ELL || KT == K_AP_RECT) {
    q.x = P.x[p]; q.y = P.y[p];
    bool ok;
    if constexpr (KT == K_AP_CIRC) ok = xtmm::in_circle(q, prm[0]);
    else if constexpr (KT == K_AP_ELL) ok = xtmm::in_ellipse(q, prm[0], prm[1]);
    else ok = xtmm::in_rect(q, prm[0], prm[1], prm[2], prm[3]);
    if (!ok) elem_lost(P, p, 0, e, turn);
  } else if constexpr (KT == K_RF) {
    q.zeta = P.zeta[p]; q.ptau = P.ptau[p];
    xtmm::rf(q, prm[0], prm[1], prm[2], r.beta0, r.two_over_beta0);
    P.ptau[p] = q.ptau; P.delta[p] = q.delta; P.rpp[p] = q.rpp; P.rvv[p] = q.rvv;
  } else if constexpr (KT == K_SHIFT) {
    q.x = P.x[p]; q.y = P.y[p];
    xtmm::xyshift(q, prm[0], prm[1]);
    P.x[p] = q.x; P.y[p] = q.y;
  } else if constexpr (KT == K_SROT) {
    q.x = P.x[p]; q.px = P.px[p]; q.y = P.y[p]; q.py = P.py[p];
    xtmm::srotation(q, prm[0], prm[1]);
    P.x[p] = q.x; P.px[p] = q.px; P.y[p] = q.y; P.py[p] = q.py;
  } else if constexpr (KT == K_MARKER) {
    (void)prm;
  } else {
    load_pt(P, (int32_t)p, q, r.beta0);
    bool ok;
    int ls;
    apply_elem(q, (uint32_t)(h & 0xffu), order, prm, r, ok, ls, 0, turn, e);
    if (!ok) return elem_lost(P, p, ls, e, turn);
    store_pt(P, (int32_t)p, q);
  }
}

// After the last turn: survivors stand at element 0 of turn `turn`.
__global__ void __launch_bounds__(256) k_elem_finish(SoA P, int64_t n, int32_t turn) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || P.state[p] != 1) return;
  P.at_turn[p] = turn;
  P.at_element[p] = 0;
}

hipError_t launch_per_element(const uint64_t* tab, const uint32_t* offsets, const uint32_t* ktypes,
                              int32_t n_el, SoA P, int64_t n, int32_t t0, int32_t n_turns,
                              KernelRef r, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned nb = blocks_for(n, 256);
  for (int32_t t = 0; t < n_turns; ++t) {
    for (int32_t e = 0; e < n_el; ++e) {
      const uint32_t o = offsets[e];
      const int32_t tt = t0 + t;
#define XTM_ELEM(KT) hipLaunchKernelGGL(k_elem<KT>, dim3(nb), dim3(256), 0, s, tab, o, e, P, n, tt, r)
      switch (ktypes[e]) {
        case K_DRIFT: XTM_ELEM(K_DRIFT); break;
        case K_MULT: XTM_ELEM(K_MULT); break;
        case K_AP_CIRC: XTM_ELEM(K_AP_CIRC); break;
        case K_AP_ELL: XTM_ELEM(K_AP_ELL); break;
        case K_AP_RECT: XTM_ELEM(K_AP_RECT); break;
        case K_RF: XTM_ELEM(K_RF); break;
        case K_SHIFT: XTM_ELEM(K_SHIFT); break;
        case K_SROT: XTM_ELEM(K_SROT); break;
        case K_MARKER: XTM_ELEM(K_MARKER); break;
        default: XTM_ELEM(K_MULT_CURV); break;  // whole state through apply_elem
      }
#undef XTM_ELEM
      const hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
  }
  hipLaunchKernelGGL(k_elem_finish, dim3(nb), dim3(256), 0, s, P, n, t0 + n_turns);
  return hipGetLastError();
}

hipError_t launch_track(const uint64_t* tab, int32_t n_el, SoA P, const int32_t* idx, const int32_t* ctrl, int64_t grid_upper,
                        int32_t block, int32_t n_turns, int32_t backward, KernelRef r,
                        int32_t variant, hipStream_t s) {
  if (grid_upper <= 0 || n_turns <= 0) return hipSuccess;
  if (variant != 4) return hipErrorInvalidValue;  // the interpreter is variant 4
  hipLaunchKernelGGL(k_track4, dim3(blocks_for(grid_upper, block)), dim3(block), 0, s, tab, n_el,
                     P, idx, ctrl, n_turns, backward, r);
  return hipGetLastError();
}

hipError_t launch_epilogue(const int32_t* idx_in, int32_t* idx_out, int32_t* lost_out,
                           int64_t grid_upper, SoA P, int32_t* ctrl, int32_t* blockcnt,
                           int64_t* passes, int32_t n_el, int32_t chunk_turns, int32_t backward,
                           hipStream_t s) {
  if (grid_upper <= 0) return hipSuccess;
  const unsigned nb = blocks_for(grid_upper, kScanBlock);
  hipLaunchKernelGGL(k_count, dim3(nb), dim3(kScanBlock), 0, s, idx_in, P, ctrl, blockcnt,
                     reinterpret_cast<unsigned long long*>(passes), n_el, chunk_turns, backward);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || (idx_out == nullptr && lost_out == nullptr)) return e;
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kScanBlock), 0, s, idx_in, idx_out, lost_out, P,
                     ctrl, blockcnt, chunk_turns, backward);
  return hipGetLastError();
}

hipError_t launch_track_batched(const uint64_t* const* tabs, const int32_t* first_slot, int32_t nv,
                                int32_t n_el, SoA P, const int32_t* idx, const int32_t* ctrl,
                                int64_t grid_upper, int32_t block, int32_t n_turns,
                                int32_t backward, KernelRef r, hipStream_t s) {
  if (grid_upper <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_track4_batched, dim3(blocks_for(grid_upper, block)), dim3(block), 0, s, tabs,
                     first_slot, nv, n_el, P, idx, ctrl, n_turns, backward, r);
  return hipGetLastError();
}

hipError_t launch_replay_batched(const uint64_t* const* tabs, const int32_t* first_slot, int32_t nv,
                                 int32_t n_el, SoA P, const int32_t* lost, const int32_t* ctrl,
                                 int64_t grid_upper, int32_t backward, KernelRef r,
                                 hipStream_t s) {
  if (grid_upper <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_replay_batched, dim3(blocks_for(grid_upper, 256)), dim3(256), 0, s, tabs,
                     first_slot, nv, n_el, P, lost, ctrl, backward, r);
  return hipGetLastError();
}

hipError_t launch_replay(const uint64_t* tab, int32_t n_el, SoA P, const int32_t* lost,
                         const int32_t* ctrl, int64_t grid_upper, int32_t backward, KernelRef r,
                         hipStream_t s) {
  if (grid_upper <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_replay, dim3(blocks_for(grid_upper, 256)), dim3(256), 0, s, tab, n_el, P,
                     lost, ctrl, backward, r);
  return hipGetLastError();
}

}  // namespace xtm

// ------------------------------------------------ optics by tracking
// One turn of a few particles from the line start, the coordinates recorded
// at the entry of every element and after the last (apertures not checked;
// a particle whose longitudinal momentum becomes imaginary in a drift keeps
// the coordinates it entered that drift with).  One thread per particle, 64 per
// workgroup; the element table passes through LDS segment by segment (the
// table's segments of at most kSegWords words), so an element costs LDS
// reads, not two dependent global loads.  The set-up from
// (x, px, y, py, zeta, delta) is the one of particle initialisation.
namespace xtm {
namespace {
__global__ void __launch_bounds__(64)
k_record(const uint64_t* __restrict__ fwd, const int32_t* __restrict__ seg, int32_t n_seg,
         int32_t n_el, const double* __restrict__ c6, int64_t n, double* __restrict__ out,
         KernelRef r) {
  __shared__ uint64_t lds[kSegWords];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = i < n;
  xtmm::Pt q{};
  if (act) {
    const double* c = c6 + 6 * i;
    const double d = c[5];
    const double u = d * (2.0 + d);
    q.x = c[0];
    q.px = c[1];
    q.y = c[2];
    q.py = c[3];
    q.zeta = c[4];
    q.delta = d;
    q.ptau = r.beta0 * u / (1.0 + sqrt(1.0 + r.beta0 * r.beta0 * u));
    q.rpp = 1.0 / (1.0 + d);
    q.rvv = (1.0 + d) / (1.0 + r.beta0 * q.ptau);
    xtmm::refresh(q, r.beta0);
  }
  bool alive = true;
  auto record = [&](int32_t e) {
    double* o = out + ((size_t)e * (size_t)n + (size_t)i) * 6;
    o[0] = q.x; o[1] = q.px; o[2] = q.y; o[3] = q.py; o[4] = q.zeta; o[5] = q.delta;
  };
  int32_t e = 0;
  for (int32_t sgi = 0; sgi < n_seg; ++sgi) {
    const int32_t w0 = seg[3 * sgi], nwords = seg[3 * sgi + 1], n_here = seg[3 * sgi + 2];
    __syncthreads();
    for (int32_t k = threadIdx.x; k < nwords; k += blockDim.x) lds[k] = fwd[w0 + k];
    __syncthreads();
    uint32_t off = 0;
    for (int32_t k = 0; k < n_here; ++k, ++e) {
      const uint64_t h = lds[off];
      const uint32_t kt = (uint32_t)(h & 0xffu);
      const uint32_t nw = (uint32_t)((h >> 16) & 0xffffu);
      const double* prm = reinterpret_cast<const double*>(&lds[off + 1]);
      off += 1 + nw;
      if (!act) continue;
      record(e);
      if (!alive || kt == K_AP_CIRC || kt == K_AP_ELL || kt == K_AP_RECT) continue;
      const xtmm::Pt q0 = q;
      bool ok;
      int lost_state;
      apply_elem<false>(q, kt, (uint32_t)((h >> 8) & 0xffu), prm, r, ok, lost_state, 0, 0, e);
      if (!ok) {
        q = q0;
        alive = false;
      }
    }
  }
  if (act) record(n_el);
}
}  // namespace

hipError_t launch_record(const uint64_t* fwd, const int32_t* seg, int32_t n_seg, int32_t n_el,
                         const double* c6, int64_t n, double* out, KernelRef r, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 63) / 64;
  hipLaunchKernelGGL(k_record, dim3((unsigned)blocks), dim3(64), 0, s, fwd, seg, n_seg, n_el, c6,
                     n, out, r);
  return hipGetLastError();
}
}  // namespace xtm

// ------------------------------------------------ loss-location refinement
// One wave per particle.  A particle lost on an aperture is backtracked
// through the inverse maps to the exit of the previous aperture, then tracked
// forward again (every lane carries the same particle); inside each drift its
// line-frame position runs on the segment between the drift's entry and exit,
// and the ends of the drift's sub-steps are tested against the aperture
// interpolated vertex by vertex between the two polygons.  The scan tests 64
// consecutive sub-steps at once, lane l the sub-step base + 1 + l against the
// whole polygon staged in LDS, the first failing one being the lowest set bit
// of the wave's ballot (polygons above the LDS limit: one sub-step at a time,
// one edge per lane).  The first failing sub-step is bisected with one edge
// per lane: lane k tests edge (k, k+1) and the even-odd parity is the parity
// of the wave's ballot (the exclusive-or of the same per-edge tests in any
// order).  Every operation is the one written in the refinement definition
// (explicit fma for interpolation, separate products and sums elsewhere).
namespace xtm {
namespace {

__device__ __forceinline__ double lerp_f(double a, double b, double f) { return fma(f, b - a, a); }

__device__ __forceinline__ void to_line(const double* __restrict__ g, double ux, double uy,
                                        double& lx, double& ly) {
  const double t1 = g[0] * ux;
  const double t2 = g[1] * uy;
  const double t3 = g[2] * ux;
  const double t4 = g[3] * uy;
  lx = (t1 + t2) + g[4];
  ly = (t3 + t4) + g[5];
}

// crossing of the horizontal ray from (px, py) with the edge from vertex i to
// vertex j of the polygon A + w (B - A)
__device__ __forceinline__ bool edge_toggle(double px, double py, double axi, double ayi,
                                            double bxi, double byi, double axj, double ayj,
                                            double bxj, double byj, double w) {
  const double xi = lerp_f(axi, bxi, w), yi = lerp_f(ayi, byi, w);
  const double xj = lerp_f(axj, bxj, w), yj = lerp_f(ayj, byj, w);
  if ((yi > py) == (yj > py)) return false;
  const double t1 = (xj - xi) * (py - yi);
  const double t2 = (px - xi) * (yj - yi);
  const double cr = t1 - t2;
  return yj > yi ? cr > 0.0 : cr < 0.0;
}

// the lane's edge of a polygon of at most 64 vertices, held in registers
struct Edge {
  bool on;
  double axi, ayi, bxi, byi, axj, ayj, bxj, byj;
};

__device__ __forceinline__ bool in_poly_wave(double px, double py, const Edge& e,
                                             const double* __restrict__ A,
                                             const double* __restrict__ B, int32_t M, double w) {
  bool t = false;
  if (M <= 64) {
    t = e.on && edge_toggle(px, py, e.axi, e.ayi, e.bxi, e.byi, e.axj, e.ayj, e.bxj, e.byj, w);
  } else {
    for (int32_t k = threadIdx.x; k < M; k += 64) {
      const int32_t kn = (k + 1 == M) ? 0 : k + 1;
      t ^= edge_toggle(px, py, A[2 * k], A[2 * k + 1], B[2 * k], B[2 * k + 1], A[2 * kn],
                       A[2 * kn + 1], B[2 * kn], B[2 * kn + 1], w);
    }
  }
  return (__popcll(__ballot(t)) & 1) != 0;
}

// the whole polygon A + w (B - A) for one lane's point, vertices from LDS
// ((x, y) pairs of A and of the differences D = B - A, rounded once: the
// same values lerp forms), each vertex interpolated once and carried to the
// next edge
__device__ __forceinline__ bool in_poly_lane(double px, double py, const double2* A,
                                             const double2* D, int32_t M, double w) {
  bool in = false;
  const double2 a0 = A[0], d0 = D[0];
  const double x0 = fma(w, d0.x, a0.x), y0 = fma(w, d0.y, a0.y);
  double xi = x0, yi = y0;
  for (int32_t k = 0; k < M; ++k) {
    double xj, yj;
    if (k + 1 == M) {
      xj = x0;
      yj = y0;
    } else {
      const double2 a = A[k + 1], d = D[k + 1];
      xj = fma(w, d.x, a.x);
      yj = fma(w, d.y, a.y);
    }
    if ((yi > py) != (yj > py)) {
      const double t1 = (xj - xi) * (py - yi);
      const double t2 = (px - xi) * (yj - yi);
      const double cr = t1 - t2;
      if (yj > yi ? cr > 0.0 : cr < 0.0) in = !in;
    }
    xi = xj;
    yi = yj;
  }
  return in;
}

__device__ __forceinline__ bool is_drift_k(uint32_t kt) { return kt == K_DRIFT || kt == K_DRIFT_EXP; }

// polygons of up to this many vertices are staged in LDS and the drift scan
// tests 64 consecutive sub-steps at once (one per lane)
constexpr int32_t kRefineLdsVerts = 256;

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 4)))
k_refine(const uint64_t* __restrict__ fwd, const uint64_t* __restrict__ bwd, RefineGeom g, SoA P,
         int64_t n, KernelRef r, double* __restrict__ s_out, double* __restrict__ x_out,
         double* __restrict__ y_out, int32_t* __restrict__ tests) {
  const int64_t i = blockIdx.x;
  if (i >= n) return;
  const double nan = __builtin_nan("");
  double so = nan, xo = nan, yo = nan;
  int32_t nt = 0;
  const int32_t eL = P.at_element[i];
  const int32_t n_el = g.n_el;
  if (P.state[i] == 0 && eL >= 0 && eL < n_el && g.ap_ord[eL] >= 0) {
    const int32_t eP = g.prev[eL];
    const double sL = g.s[eL];
    const double sP = eP < eL ? g.s[eP] : g.s[eP] - g.s[n_el];
    xtmm::Pt q;
    load_pt(P, (int32_t)i, q, r.beta0);
    to_line(g.G + 6 * eL, q.x, q.y, xo, yo);
    so = sL;
    const long long pid = P.pid[i];
    if (sL - sP > 0.0) {
      bool ok = true;
      for (int32_t j = (eL + n_el - 1) % n_el; j != eP; j = (j + n_el - 1) % n_el) {
        const uint64_t h = bwd[g.off_b[j]];
        const double* prm = reinterpret_cast<const double*>(bwd + g.off_b[j] + 1);
        bool okj;
        int lost_state;
        apply_elem<false>(q, (uint32_t)(h & 0xffu), (uint32_t)((h >> 8) & 0xffu), prm, r, okj,
                          lost_state, pid, 0, j);
        if (!okj) { ok = false; break; }
      }
      if (ok) {
        const int32_t M = g.M;
        const double* A = g.poly + (size_t)g.ap_ord[eP] * 2 * M;
        const double* B = g.poly + (size_t)g.ap_ord[eL] * 2 * M;
        __shared__ double2 polyA[kRefineLdsVerts], polyD[kRefineLdsVerts];
        const bool lds = M <= kRefineLdsVerts;
        if (lds) {
          for (int32_t v = threadIdx.x; v < M; v += 64) {
            polyA[v] = make_double2(A[2 * v], A[2 * v + 1]);
            polyD[v] = make_double2(B[2 * v] - A[2 * v], B[2 * v + 1] - A[2 * v + 1]);
          }
          __syncthreads();
        }
        Edge e{};
        const int32_t k = threadIdx.x;
        e.on = M <= 64 && k < M;
        if (e.on) {
          const int32_t kn = (k + 1 == M) ? 0 : k + 1;
          e.axi = A[2 * k]; e.ayi = A[2 * k + 1]; e.bxi = B[2 * k]; e.byi = B[2 * k + 1];
          e.axj = A[2 * kn]; e.ayj = A[2 * kn + 1]; e.bxj = B[2 * kn]; e.byj = B[2 * kn + 1];
        }
        double sc = sP;
        for (int32_t j = (eP + 1) % n_el; j != eL; j = (j + 1) % n_el) {
          const uint64_t h = fwd[g.off_f[j]];
          const uint32_t kt = (uint32_t)(h & 0xffu);
          const double* prm = reinterpret_cast<const double*>(fwd + g.off_f[j] + 1);
          bool okj;
          int lost_state;
          if (!is_drift_k(kt)) {
            apply_elem<false>(q, kt, (uint32_t)((h >> 8) & 0xffu), prm, r, okj, lost_state, pid,
                              0, j);
            continue;
          }
          const double L = prm[0];
          double v0x, v0y, v1x, v1y;
          to_line(g.G + 6 * j, q.x, q.y, v0x, v0y);
          apply_elem<false>(q, kt, (uint32_t)((h >> 8) & 0xffu), prm, r, okj, lost_state, pid, 0,
                            j);
          if (!okj) break;
          to_line(g.G + 6 * j, q.x, q.y, v1x, v1y);
          bool found = false;
          if (L > 0.0) {
            long long K = (long long)ceil(L / g.ds);
            if (K < 1) K = 1;
            long long kf = 0;  // first sub-step whose end is outside (0: none)
            if (lds) {
              // 64 sub-steps per pass, lane l testing sub-step base + 1 + l
              for (long long base = 0; base < K && kf == 0; base += 64) {
                const long long kk = base + 1 + threadIdx.x;
                bool out = false;
                if (kk <= K) {
                  const double f = (double)kk / (double)K;
                  const double sf = sc + L * f;
                  const double w = (sf - sP) / (sL - sP);
                  out = !in_poly_lane(lerp_f(v0x, v1x, f), lerp_f(v0y, v1y, f), polyA, polyD,
                                      M, w);
                }
                const unsigned long long mask = __ballot(out);
                if (mask) {
                  const int first = __ffsll((long long)mask) - 1;
                  kf = base + 1 + first;
                  nt += first + 1;
                } else {
                  nt += (int32_t)((K - base) < 64 ? (K - base) : 64);
                }
              }
            } else {
              for (long long kk = 1; kk <= K; ++kk) {
                const double f = (double)kk / (double)K;
                const double sf = sc + L * f;
                const double w = (sf - sP) / (sL - sP);
                ++nt;
                if (!in_poly_wave(lerp_f(v0x, v1x, f), lerp_f(v0y, v1y, f), e, A, B, M, w)) {
                  kf = kk;
                  break;
                }
              }
            }
            if (kf > 0) {
              const long long kk = kf;
              const double f = (double)kk / (double)K;
              double lo = (double)(kk - 1) / (double)K, hi = f;
              for (int32_t b = 0; b < g.n_bisect; ++b) {
                const double m = 0.5 * (lo + hi);
                const double sm = sc + L * m;
                const double wm = (sm - sP) / (sL - sP);
                ++nt;
                if (in_poly_wave(lerp_f(v0x, v1x, m), lerp_f(v0y, v1y, m), e, A, B, M, wm))
                  lo = m;
                else
                  hi = m;
              }
              so = sc + L * hi;
              xo = lerp_f(v0x, v1x, hi);
              yo = lerp_f(v0y, v1y, hi);
              found = true;
            }
          }
          if (found) break;
          sc = sc + L;
        }
      }
    }
  }
  if (threadIdx.x == 0) {
    s_out[i] = so;
    x_out[i] = xo;
    y_out[i] = yo;
    if (tests) tests[i] = nt;
  }
}

}  // namespace

hipError_t launch_refine(const uint64_t* fwd, const uint64_t* bwd, const RefineGeom& g, SoA P,
                         int64_t n, KernelRef r, double* s_out, double* x_out, double* y_out,
                         int32_t* tests, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (n > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_refine, dim3((unsigned)n), dim3(64), 0, s, fwd, bwd, g, P, n, r, s_out,
                     x_out, y_out, tests);
  return hipGetLastError();
}

}  // namespace xtm
