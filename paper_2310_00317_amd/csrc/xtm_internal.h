// xtm_internal.h -- shared declarations between the C-ABI runtime and the
// gfx950 kernels of the tracking library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

namespace xtm {

// Device control block of a particle set (int32): [0] alive count, [1] turn
// of the alive particles, [2] alive count scanned by the last epilogue,
// [3] number of particles lost during the last chunk.

// Device element-table record: one 64-bit header word followed by `nw`
// FP64 parameter words.  Header bits: [0,8) kernel type, [8,16) multipole
// order, [16,32) parameter word count, [32,64) user element index.
enum KType : uint32_t {
  K_DRIFT = 1,
  K_DRIFT_EXP = 2,
  K_MULT = 3,       // coefficients only:  cr_N, ci_N, ..., cr_0, ci_0
  K_MULT_CURV = 4,  // coefficients, then hxl, knl0*hxl, Lr
  K_MULT_LR = 12,   // coefficients, then Lr (radiation length, no frame curvature)
  K_RF = 5,         // amp = charge0 V / p0c, k = 2 pi f / (beta0 c), phase [rad]
  K_SHIFT = 6,      // dx, dy
  K_SROT = 7,       // cos, sin
  K_AP_CIRC = 8,    // r^2
  K_AP_ELL = 9,     // 1/a^2, 1/b^2
  K_AP_RECT = 10,   // xmin, xmax, ymin, ymax
  K_MARKER = 11
};

__host__ __device__ inline uint64_t make_header(uint32_t ktype, uint32_t order, uint32_t nw,
                                                uint32_t index) {
  return (uint64_t)(ktype & 0xffu) | ((uint64_t)(order & 0xffu) << 8) |
         ((uint64_t)(nw & 0xffffu) << 16) | ((uint64_t)index << 32);
}

struct SoA {
  double *x, *px, *y, *py, *zeta, *delta, *ptau, *rpp, *rvv;
  int32_t *state, *at_element, *at_turn;
  int64_t* pid;
};

// Reference quantities and per-call radiation settings passed by value to
// every tracking kernel (the generated line kernels declare the same layout).
struct KernelRef {
  double beta0;
  double two_over_beta0;
  double gamma0;
  double c_mean;   // (2/3) r m                     [eV m], r = classical radius
  double c_quant;  // 55/(24 sqrt 3) r m hbar_c      [eV^2 m^2]
  double p0c;
  unsigned long long seed;
  int32_t rad_mode;  // 0 off, 1 mean, 2 mean + quantum (Gaussian), 3 photon by photon
  int32_t pad;
  float* rec;          // early-turn recorder [rec_turns][4][rec_n] (x, px, y, py) or null
  int32_t rec_turns;   // record the start of absolute turns 0 .. rec_turns-1
  int32_t rec_n;       // particles in the set (record stride)
  const double* photon_table;  // inverse photon spectrum on the device (mode 3), or null
  double c_nphot;      // 5/(2 sqrt 3) r m / hbar_c: mean photon count per gamma h Lr
  double c_ucrit;      // (3/2) hbar_c [eV m]: critical energy per gamma^3 h
};

// Inverse of the synchrotron photon-number spectrum for the photon-by-photon
// model: g(s) = x^(1/3) where the probability of a photon energy of at least
// x u_c is exp(-s), at s = i / 64, i = 0 .. kPhotonTableNodes - 1, each value
// rounded to single precision (host table, computed once per process).
constexpr int32_t kPhotonTableNodes = 2433;
const std::vector<double>& photon_table_host();
// The same table on the current device (uploaded once per device).
hipError_t photon_table_device(const double** out);

// 6D linear normal form of a one-turn Jacobian J (row-major 6x6, canonical
// x, px, y, py, zeta, pzeta): per mode k (the plane it dominates) the
// eigenvalue, the eigenvector normalised to v^H S v = 2i with v_2k real and
// positive, the tune arg(lambda)/2pi mod 1 and the damping -ln|lambda|.
// False for real eigenvalues (an unstable plane) or a failed iteration.
struct NormalForm6 {
  double co[6];
  double lam_re[3], lam_im[3], q[3], damping[3];
  double v_re[18], v_im[18];
};
bool normal_form6(const double J[36], NormalForm6* out);
// u = co + sum_k Re(v_k sqrt(eps_k) (g_2k + i g_2k+1)), delta from pzeta.
void matched_gaussian(const NormalForm6& nf, double beta0, const double eps[3],
                      const double* gauss, int64_t n, double* out);

// launch helpers implemented in xtm_kernels.hip; all are stream-ordered
hipError_t launch_init(const double* coords6, int64_t n, int64_t first_id, SoA P, KernelRef r,
                       hipStream_t s);
hipError_t launch_iota(int32_t* idx, int64_t n, int32_t* ctrl, int32_t n_alive, int32_t turn,
                       hipStream_t s);
hipError_t launch_advance(int32_t* ctrl, int32_t dk, hipStream_t s);
// words per LDS segment of the element table (the optics recorder); a record
// never straddles two segments
constexpr int kSegWords = 4096;
constexpr int32_t kLineBlock = 256;  // workgroup size of the per-line kernel
// the element interpreter (kernel variant 4)
hipError_t launch_track(const uint64_t* tab, int32_t n_el, SoA P, const int32_t* idx,
                        const int32_t* ctrl, int64_t grid_upper, int32_t block, int32_t n_turns, int32_t backward, KernelRef r,
                        int32_t variant, hipStream_t s);
// end-of-chunk bookkeeping: passes of the chunk (added to *passes), then an
// order-preserving compaction of the alive list into idx_out (if non-null)
// and of the particles lost during the chunk into lost_out (if non-null);
// ctrl[0] = new alive count, ctrl[3] = lost count
hipError_t launch_epilogue(const int32_t* idx_in, int32_t* idx_out, int32_t* lost_out,
                           int64_t grid_upper, SoA P, int32_t* ctrl, int32_t* blockcnt,
                           int64_t* passes, int32_t n_el, int32_t chunk_turns, int32_t backward,
                           hipStream_t s);
// coordinates of the particles in lost[0..ctrl[3]) re-tracked from the chunk
// start to their loss point (for kernels that record losses in registers)
hipError_t launch_track_batched(const uint64_t* const* tabs, const int32_t* first_slot, int32_t nv,
                                int32_t n_el, SoA P, const int32_t* idx, const int32_t* ctrl,
                                int64_t grid_upper, int32_t block, int32_t n_turns,
                                int32_t backward, KernelRef r, hipStream_t s);
hipError_t launch_replay_batched(const uint64_t* const* tabs, const int32_t* first_slot, int32_t nv,
                                 int32_t n_el, SoA P, const int32_t* lost, const int32_t* ctrl,
                                 int64_t grid_upper, int32_t backward, KernelRef r,
                                 hipStream_t s);
hipError_t launch_replay(const uint64_t* tab, int32_t n_el, SoA P, const int32_t* lost,
                         const int32_t* ctrl, int64_t grid_upper, int32_t backward, KernelRef r,
                         hipStream_t s);
hipError_t launch_fill_i64(int64_t* p, int64_t v, hipStream_t s);
// One kernel launch per element and turn (the measurement baseline); offsets
// and ktypes: host arrays of each element's record position in `tab` (word
// index) and kernel type.
hipError_t launch_per_element(const uint64_t* tab, const uint32_t* offsets, const uint32_t* ktypes,
                              int32_t n_el, SoA P, int64_t n, int32_t t0, int32_t n_turns,
                              KernelRef r, hipStream_t s);

constexpr int kScanBlock = 1024;

// One turn of n particles with the coordinates (x, px, y, py, zeta, delta)
// recorded at every element entry and after the last: out[(e n + i) 6 + c].
// (seg: the table's LDS segments, kSegWords words at most each)
hipError_t launch_record(const uint64_t* fwd, const int32_t* seg, int32_t n_seg, int32_t n_el,
                         const double* c6, int64_t n, double* out, KernelRef r, hipStream_t s);

// Loss-location refinement geometry (device pointers into one buffer):
// s of each element and of the line end (n_el + 1), line frame of each
// element's entry coordinates as (a11, a12, a21, a22, b1, b2) (n_el + 1),
// aperture polygons in the line frame (M vertices, x and y, per aperture),
// record positions of each element in the forward and backward tables, the
// previous aperture of each aperture and each element's aperture ordinal
// (-1: not an aperture).
struct RefineGeom {
  int32_t n_el, M, n_bisect;
  double ds;
  const double* s;
  const double* G;
  const double* poly;
  const int32_t* off_f;
  const int32_t* off_b;
  const int32_t* prev;
  const int32_t* ap_ord;
};
hipError_t launch_refine(const uint64_t* fwd, const uint64_t* bwd, const RefineGeom& g, SoA P,
                         int64_t n, KernelRef r, double* s_out, double* x_out, double* y_out,
                         int32_t* tests, hipStream_t s);

// Per-line tracking kernel generated from the lattice's cell structure and
// compiled at run time (xtm_jit.cpp).
struct LineKernel {
  bool ok = false;
  bool tried = false;
  int32_t style = 0;
  bool batched = false;  // variants of one cell structure, parameters per variant
  int32_t nv = 1;        // variants (batched)
  int64_t stride = 0;    // parameter words per variant
  hipFunction_t fn = nullptr;
  int32_t period = 0, n_cells = 0, n_kinds = 0;  // period = length of the repeating unit
  double* prm_d = nullptr;     // element parameters in element order, no headers
                               // (batched: one such block per variant)
  int32_t* cells_d = nullptr;  // per cell: kind, first parameter word, first element, words
  std::string source;
  std::string error;
};
// Generated-kernel forms ("styles"), all computing the same maps in the same
// order: the workgroup (256 lanes or one wave), the way element code reads
// its parameters from the LDS slot (line_fetch), where a lost particle's
// coordinates are stored (line_deferred), how many particles each lane
// carries (line_ppt) and whether the cells are long (line_long: units of up
// to 40 elements within 64 elements of code, instead of 24 within 48; fewer
// cell boundaries for a latency-bound set, more code and prefetch registers
// for a saturated one).  Kernel variant 5 + style.
struct LineStyle {
  int32_t lanes, fetch;
  bool deferred;
  int32_t ppt;
  bool long_cells;
};
constexpr LineStyle kLineStyle[] = {
    {256, 0, false, 1, false}, {64, 0, false, 1, false},  // 5, 6: parameters read at each use
    {256, 1, false, 1, false}, {64, 1, false, 1, false},  // 7, 8: an element's words in one group
    {256, 2, false, 1, false}, {64, 2, false, 1, false},  // 9, 10: the next element's group ahead
    {256, 2, true, 1, false},  {64, 2, true, 1, false},   // 11, 12: as 9, 10, one loss test per cell
    {64, 2, false, 2, false},                             // 13: as 10, two particles per lane
    {64, 2, false, 1, true},                              // 14: as 10, long cells
};
constexpr int32_t kLineStyles = (int32_t)(sizeof(kLineStyle) / sizeof(kLineStyle[0]));
inline int32_t line_block(int32_t style) { return kLineStyle[style].lanes; }
inline int32_t line_fetch(int32_t style) { return kLineStyle[style].fetch; }
inline bool line_deferred(int32_t style) { return kLineStyle[style].deferred; }
inline int32_t line_ppt(int32_t style) { return kLineStyle[style].ppt; }
inline bool line_long(int32_t style) { return kLineStyle[style].long_cells; }
// Radiation forms of a per-line kernel: which radiation steps its radiating
// multipoles carry, so that a kernel holds only the code its calls can take
// (the photon emitter is an out-of-line call whose register and stack cost a
// kernel pays across its whole element loop whether it runs or not).
//   0: none (radiation off, or a line without radiating multipoles);
//   1: the mean loss and Gaussian quantum excitation (modes 1 and 2, the
//      mode read at run time);
//   2: photon by photon (mode 3).
constexpr int32_t kRadForms = 3;
inline int32_t rad_form(bool line_radiates, int32_t mode) {
  return (!line_radiates || mode == 0) ? 0 : (mode == 3 ? 2 : 1);
}
// Whether an element table holds radiating multipoles (a curvature term or
// a radiation length).
bool table_radiates(const std::vector<uint64_t>& tab, int32_t n_el);
bool build_line_kernel(const std::vector<uint64_t>& tab, int32_t n_el, int32_t style,
                       int32_t rad_form, LineKernel* k);
// The same for a batch of lattice variants (batched = true: the kernel takes
// the slot partition and reads each variant's parameters); fails if the
// variants' element structures differ.
bool build_line_kernel_multi(const std::vector<const std::vector<uint64_t>*>& tabs, int32_t n_el,
                             int32_t style, bool batched, int32_t rad_form, LineKernel* k);
// The generated recording kernel of optics by tracking (the coordinates of
// one turn at every element's entry, as launch_record, or with all_rows =
// false only after the turn, row n_el); fails if the line has no cell
// decomposition.
bool build_record_kernel(const std::vector<uint64_t>& tab, int32_t n_el, LineKernel* k);
hipError_t launch_line_record(const LineKernel& k, int32_t n_el, const double* c6, int64_t n,
                              double* out, bool all_rows, KernelRef r, hipStream_t s);
void free_line_kernel(LineKernel* k);
hipError_t launch_line(const LineKernel& k, int32_t n_el, SoA P, const int32_t* idx,
                       const int32_t* ctrl, int64_t grid_upper, int32_t block, int32_t n_turns,
                       int32_t backward, KernelRef r, hipStream_t s);
hipError_t launch_line_batched(const LineKernel& k, int32_t n_el, SoA P, const int32_t* idx,
                               const int32_t* ctrl, int64_t grid_upper, int32_t n_turns,
                               int32_t backward, KernelRef r, const int32_t* first_slot,
                               hipStream_t s);

}  // namespace xtm

namespace xtm {
hipError_t launch_philox(unsigned long long seed, const uint32_t ctr0[4], int64_t n_blocks,
                         uint32_t* out, hipStream_t s);
// learned early stop (xtm_learn.hip)
hipError_t launch_mlp_forward(const float* theta, const float* norm, const float* X, int64_t B,
                              float* logit, hipStream_t s);
int64_t mlp_workspace_floats(int64_t B);
// Largest batch of the allocation-free gradient entry point: its per-block
// partial gradients live in a fixed device array of
// mlp_workspace_floats(kMlpNoAllocMaxBatch) floats (4.6 MiB) per device.
constexpr int64_t kMlpNoAllocMaxBatch = 4096;
// Device address of that array on the current device, looked up once per
// device with hipGetSymbolAddress and kept for the life of the process.
hipError_t mlp_noalloc_workspace(float** out);
hipError_t launch_mlp_grad(const float* theta, const float* norm, const float* X, const float* Y,
                           int64_t B, float pos_weight, float* grad, float* loss, float* work,
                           hipStream_t s);
hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr,
                       hipStream_t s);
hipError_t launch_gather_rows(const float* X, const float* Y, const int32_t* perm, int64_t B,
                              float* Xb, float* Yb, hipStream_t s);
hipError_t launch_mlp_init(float* theta, unsigned long long seed, hipStream_t s);
hipError_t launch_features(const float* rec, int64_t n, const double twiss4[4], double emit,
                           double r_ap, const float2* tw, const float* win, float* out,
                           hipStream_t s);
hipError_t launch_feature_stats(const float* f, const int32_t* mask, int64_t n, float* norm,
                                hipStream_t s);
hipError_t launch_retire(SoA P, const int32_t* idx, const int32_t* ctrl, int64_t grid_upper,
                         const float* logit, float threshold, unsigned long long audit_seed,
                         unsigned int audit_threshold, unsigned int* counts, int32_t* audit_flags,
                         hipStream_t s);
hipError_t launch_rule_score(const float* f, int64_t n, float* score, hipStream_t s);
}
