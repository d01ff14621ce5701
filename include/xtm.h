/*
 * xtm.h -- C ABI of the MI355X (gfx950) thin-lattice FP64 tracking library.
 *
 * The library tracks an ensemble of particles element by element through a
 * ring lattice for many turns (paper: Xsuite, arXiv 2310.00317, section
 * "Lattice modelling and single particle tracking": the beam line is a
 * sequence of element objects; the tracker runs the whole line in one
 * compiled kernel; aperture elements stop particles found outside and record
 * where they were lost, section "Particle-matter interaction and collimation
 * studies").  The user-facing operations are: build a lattice, bind and
 * initialise a particle set, track it n turns, read out the losses.
 *
 * Conventions for every entry point:
 *  - Return value: XTM_OK (0) or a negative xtm_status.  Nothing throws
 *    across the ABI.  xtm_last_error() gives a message for the calling
 *    thread's last failure.
 *  - Argument, element and reference validation is synchronous.  Device
 *    faults surface at the next synchronising call (xtm_sync,
 *    xtm_get_losses, or xtm_track when stats are requested) as XTM_E_HIP.
 *  - Streams are passed as `void*` holding a hipStream_t (NULL = the null
 *    stream).  All work is stream-ordered; only the calls documented as
 *    synchronising wait for the device.
 *  - Particle memory is CALLER-owned device memory; lattices and particle
 *    views are LIBRARY-owned handles.  The library never frees or
 *    reallocates caller memory.
 *  - Particle-level trouble is not an error: it is recorded per particle
 *    (state 1 alive, 0 lost on an aperture, -1 lost because the longitudinal
 *    momentum became imaginary or non-finite in a drift), with the element
 *    index (at_element) and turn (at_turn) of the loss.
 *  - A handle must not be used from two host threads at once.
 *
 * Coordinates (per particle, FP64): x, y [m]; px = Px/P0, py = Py/P0;
 * zeta = s - beta0 c t [m]; delta = (P-P0)/P0; derived and stored:
 * ptau = (E-E0)/(P0 c), rpp = 1/(1+delta), rvv = beta/beta0.
 */
#ifndef XTM_H
#define XTM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xtm_status;
enum {
  XTM_OK = 0,
  XTM_E_ARG = -1,         /* bad argument (null pointer, negative size, ...) */
  XTM_E_ELEMENT = -2,     /* unknown element type or invalid element data    */
  XTM_E_HIP = -3,         /* HIP runtime or device error                     */
  XTM_E_NOMEM = -4,       /* device allocation failed                        */
  XTM_E_REFERENCE = -5,   /* lattice and particles disagree on the reference */
  XTM_E_UNSUPPORTED = -6, /* valid request the library does not implement    */
  XTM_E_STATE = -7        /* call out of order (e.g. tracking an unset set)  */
};

/* Element type codes. */
enum {
  XTM_DRIFT = 1,          /* exact drift, length L                                   */
  XTM_DRIFT_EXPANDED = 2, /* drift of the paraxial (expanded) Hamiltonian, length L  */
  XTM_MULTIPOLE = 3,      /* thin multipole, orders 0..order, optional curvature     */
  XTM_RF = 4,             /* thin RF cavity                                          */
  XTM_XYSHIFT = 5,        /* reference-frame translation (misalignment)              */
  XTM_SROTATION = 6,      /* reference-frame rotation about s (tilt)                 */
  XTM_AP_CIRCLE = 7,      /* circular aperture                                       */
  XTM_AP_ELLIPSE = 8,     /* elliptic aperture                                       */
  XTM_AP_RECT = 9,        /* rectangular aperture                                    */
  XTM_MARKER = 10,        /* no-op                                                   */
  XTM_QUADRUPOLE = 11,    /* thick quadrupole, sliced at lattice creation            */
  XTM_SBEND = 12          /* thick sector bend, sliced at lattice creation           */
};
#define XTM_MAX_ORDER 10

/*
 * Element description (248 bytes, natural alignment).  Meaning by type:
 *  DRIFT, DRIFT_EXPANDED: length = L [m] (any sign; negative L undoes a drift).
 *  MULTIPOLE: order N in 0..10; knl[n], ksl[n] integrated normal/skew strengths
 *    of MAD index n [m^-n]; the kick is dpx - i dpy = -sum_n (knl_n + i ksl_n)
 *    (x + i y)^n / n!.  hxl [rad] bends the reference frame over the length
 *    `length` [m]: dpx += hxl (1+delta) - knl0 hxl x / length (last term only if
 *    length > 0), zeta -= hxl x (1 + beta0 ptau) rpp.
 *  RF: p[0] = V [V], p[1] = f [Hz], p[2] = lag [deg]:
 *    ptau += (charge0 V / p0c) sin(lag pi/180 - 2 pi f zeta / (beta0 c)).
 *  XYSHIFT: p[0] = dx, p[1] = dy [m]: x -= dx, y -= dy.
 *  SROTATION: p[0] = angle [rad]: (x,y) <- (c x + s y, c y - s x), same for (px,py).
 *  AP_CIRCLE: p[0] = r > 0.  AP_ELLIPSE: p[0] = a > 0, p[1] = b > 0.
 *  AP_RECT: p[0..3] = xmin < xmax, ymin < ymax.  A particle exactly on the
 *    boundary survives; a NaN coordinate is outside.
 *  QUADRUPOLE (thick; paper section on the tracking engine: thick elements
 *    by symplectic splitting): length = L > 0 [m], p[0] = k1, p[1] = k1s
 *    [m^-2], p[2] = N slices (an integer, 1..10000).  SBEND (thick sector
 *    bend): length = L > 0, p[0] = bending angle theta [rad], p[1] = k1
 *    [m^-2], p[2] = N.  xtm_lattice_create replaces each by N drift-kick-drift
 *    slices (kicks at the slice midpoints): with d = L/N, DRIFT(d/2), then N
 *    times [thin kick, DRIFT(d)] with the last drift d/2 instead:
 *      QUADRUPOLE kick: MULTIPOLE of order 1, knl[1] = k1 d, ksl[1] = k1s d;
 *      SBEND kick: MULTIPOLE of order 1, knl[0] = hxl = theta/N, length = d
 *        (the curvature's weak focusing and path-length terms), knl[1] = k1 d.
 *    Element indices everywhere (loss records, optics rows, refinement) then
 *    refer to the sliced line; xtm_lattice_user_index maps them back.
 *  Unused fields are ignored.
 */
typedef struct xtm_element_desc {
  int32_t type;
  int32_t order;
  double length;
  double knl[XTM_MAX_ORDER + 1];
  double ksl[XTM_MAX_ORDER + 1];
  double hxl;
  double p[6];
} xtm_element_desc;

/* Reference particle: rest mass [eV], charge [e], momentum p0c [eV].
   beta0 = p0c / sqrt(p0c^2 + m^2), gamma0 = sqrt(p0c^2 + m^2) / m. */
typedef struct xtm_reference {
  double mass0_eV;
  double charge0;
  double p0c_eV;
} xtm_reference;

typedef struct xtm_lattice_s* xtm_lattice;     /* library-owned */
typedef struct xtm_particles_s* xtm_particles; /* library-owned view of caller memory */

/* Caller-owned device arrays of length n (contiguous, 8-byte aligned). */
typedef struct xtm_arrays {
  double *x, *px, *y, *py, *zeta, *delta, *ptau, *rpp, *rvv;
  int32_t *state, *at_element, *at_turn;
  int64_t* particle_id;
  int64_t n;
} xtm_arrays;

const char* xtm_last_error(void);
const char* xtm_version(void);
/* Highest kernel number accepted in xtm_track_opts.variant (variants 5 to
   this value are the forms of the per-line kernel). */
int32_t xtm_max_variant(void);

/* Build a lattice from n element descriptions (host memory, copied; the
   caller may free `el` on return).  Validates every element (unknown type,
   order outside 0..10, non-positive aperture sizes, empty rectangle ->
   XTM_E_ELEMENT; mass or p0c not positive -> XTM_E_REFERENCE).  Packs a
   device table of per-element parameters for the forward and the inverse
   (backward) direction.  n = 0 is allowed (tracking is then a no-op). */
xtm_status xtm_lattice_create(const xtm_element_desc* el, int32_t n, const xtm_reference* ref,
                              xtm_lattice* out);
xtm_status xtm_lattice_destroy(xtm_lattice lat);
/* Number of elements (of the sliced line) and size in bytes of the device
   table (forward). */
xtm_status xtm_lattice_info(xtm_lattice lat, int32_t* n_elements, int64_t* table_bytes);

/* User element index of each element of the (sliced) line: h_out, host,
   n_elements values (xtm_lattice_info); a thin element maps to its own
   index, each slice of a thick element to the thick element's. */
xtm_status xtm_lattice_user_index(xtm_lattice lat, int32_t* h_out);

/* Bind caller-owned device arrays as a particle set for reference `ref`.
   Allocates the library's per-set work buffers (alive list, counters:
   ~9 bytes per particle).  The arrays must stay valid until release. */
xtm_status xtm_particles_bind(const xtm_arrays* a, const xtm_reference* ref, xtm_particles* out);
xtm_status xtm_particles_release(xtm_particles p);

/* Initialise the bound set from n x 6 row-major coordinates
   (x, px, y, py, zeta, delta), n = the bound length.  `coords` is device
   memory if coords_on_device != 0, host memory otherwise (copied before
   return).  Derives ptau, rpp, rvv from delta; state = 1; at_element =
   at_turn = 0; particle_id = first_id + i.  Resets the set's turn to 0 and
   its alive list to all particles.  Stream-ordered. */
xtm_status xtm_particles_init(xtm_particles p, const double* coords, int64_t first_id,
                              int32_t coords_on_device, void* stream);

/* Adopt externally written arrays (e.g. a snapshot restored by the caller):
   the set's turn becomes `turn` and its alive list is rebuilt from `state`
   on the device.  Alive particles must have at_turn == turn. */
xtm_status xtm_particles_reset(xtm_particles p, int32_t turn, void* stream);

/* Current turn of the set's alive particles (host-side counter). */
xtm_status xtm_particles_turn(xtm_particles p, int32_t* turn);

/* Tracking options (a zeroed struct, or NULL, selects defaults). */
typedef struct xtm_track_opts {
  int32_t turns_per_chunk; /* turns per kernel launch; 0 = automatic                  */
  int32_t block;           /* threads per workgroup (64..1024, multiple of 64); 0 = auto */
  int32_t no_compact;      /* 1 = keep lost particles in the alive list between chunks */
  int32_t use_graph;       /* 1 = replay the chunk sequence as a captured hipGraph    */
  int32_t time_kernels;    /* 1 = time each tracking launch with HIP events (stats)   */
  int32_t variant;         /* tracking kernel (all give bitwise the same results):
                              0 = default (14 when the line has a compact
                              periodic cell structure, else 4); 1..3 are not used
                              (XTM_E_ARG); 4 = interpreter, losses
                              kept in registers and replayed after the chunk;
                              5..xtm_max_variant() = per-line kernel generated from
                              the lattice's cell structure and compiled at first
                              use (a lost particle's coordinates are stored as it
                              is lost, no replay; the workgroup shares each cell's
                              parameters staged in LDS; `block` is ignored).
                              Variant 5 + s, s = 0..7: s & 1 selects one-wave
                              workgroups instead of 256 lanes; s >> 1 how element
                              code reads its parameters from LDS: 0 at each use,
                              1 all of an element's words in one group before its
                              arithmetic, 2 the next element's group issued
                              before the current element's arithmetic, 3 as 2
                              with one loss test per cell instead of a store at
                              every loss test (lanes lost in a cell re-apply the
                              cell's maps from its entry to find the coordinates
                              to store).  Variant 13: as 10 with two particles
                              per lane (slots i and i + 64 of a workgroup's
                              range), their maps interleaved.  Variant 14: as 10
                              with long cells (repeating units of up to 40
                              elements instead of 24: fewer cell boundaries per
                              turn, more code and prefetch registers).
                              XTM_E_UNSUPPORTED if it cannot be built */
  int32_t radiation;       /* synchrotron radiation in multipoles with length > 0:
                              0 off, 1 mean energy loss, 2 mean + quantum excitation
                              (Gaussian, see below), 3 photon by photon (see
                              xtm_photon_table); forward tracking with the
                              default, 4 or per-line kernels only */
  int32_t record_turns;    /* with record_buf: record the start of turns 0 .. record_turns-1 */
  uint64_t rng_seed;       /* key of the quantum-excitation deviates */
  float* record_buf;       /* early-turn recorder or NULL: device FP32
                              [record_turns][4][n] with n the set's size, indexed by
                              the particle's slot; at the start of each absolute turn
                              t < record_turns, (x, px, y, py) of every particle alive
                              at element 0 are written; lost particles leave their
                              entries untouched (caller-owned, caller-cleared).
                              Forward tracking with the default, 4 or per-line
                              kernels only */
  int32_t compact_every;   /* compact the alive list after every this many chunks (and
                              after the last); 0 = the plan's, else 1 */
  int32_t pad;
} xtm_track_opts;

typedef struct xtm_track_stats {
  int64_t passes;     /* (particle, element) applications made while alive, loss included */
  int64_t alive;      /* particles alive after the call */
  int32_t launches;   /* tracking-kernel launches made by the call */
  int32_t variant;    /* tracking kernel that ran (see xtm_track_opts) */
  double kernel_ms;   /* summed duration of those launches (time_kernels = 1), else 0 */
} xtm_track_stats;

/* Track the set n_turns turns forward through `lat`, continuing from the
   set's turn t: for each turn, each element in order is applied to every
   alive particle; a particle lost at element e of turn u gets state 0/-1,
   at_element = e, at_turn = u, and keeps its coordinates as they entered e;
   survivors end with at_turn = t + n_turns.  track(a) then track(b) gives
   bitwise the same result as track(a+b).  Returns after enqueueing, unless
   `stats` is non-NULL, in which case it synchronises the stream and fills
   the statistics.  XTM_E_REFERENCE if lat and p have different references. */
xtm_status xtm_track(xtm_lattice lat, xtm_particles p, int32_t n_turns,
                     const xtm_track_opts* opts, void* stream, xtm_track_stats* stats);

/* Track n_turns backward: turns in reverse, elements last to first, each
   applying its exact inverse (drift -L, kicks subtracted, shift +d, rotation
   -angle); apertures still check.  Survivors end with at_turn = t - n_turns;
   a particle lost while going back records the turn index being undone. */
xtm_status xtm_track_backward(xtm_lattice lat, xtm_particles p, int32_t n_turns,
                              void* stream, xtm_track_stats* stats);

/* Measurement baseline, not a tracking path to use: the same maps applied by
   one kernel launch per element and turn (n_turns x n_el launches), each
   launch reading every alive particle's state from HBM and writing it back,
   as a one-kernel-per-element tracker would.  Forward, from the set's turn;
   no radiation, recorder, chunking or graph.  Results (coordinates, states,
   loss turns and elements) equal xtm_track's bit for bit; the set's alive
   list is rebuilt afterwards.  With stats (synchronising): passes counted on
   the host from the states before and after, launches = n_turns x n_el,
   variant 0, kernel_ms = all launches together. */
xtm_status xtm_track_per_element(xtm_lattice lat, xtm_particles p, int32_t n_turns, void* stream,
                                 xtm_track_stats* stats);

/* Loss-location refinement (paper section on beam losses and its aperture
   figure: losses localised below the spacing of the aperture checks by
   backtracking each lost particle against an aperture model refined by
   polygonal interpolation).  For each particle i of p whose state is 0
   (lost on an aperture element e_L; its stored coordinates are those it
   entered e_L with): the particle is backtracked through the inverse maps to
   the exit of the previous aperture e_P (cyclically: the last aperture of
   the line when e_L is the first), then tracked forward again; in each drift
   its position in the frame of the line start (the coordinates mapped back
   through every XYShift and SRotation before the element) moves on a
   straight segment.  Each aperture is a polygon of n_vertices vertices: the
   points where rays from the aperture's own origin at angles
   2 pi k / n_vertices meet its boundary, in the line frame; between e_P and
   e_L vertex k moves linearly in s.  Each drift is cut into ceil(L / ds)
   equal sub-steps; the first sub-step whose end is outside the interpolated
   polygon (even-odd rule) is bisected n_bisect times.
   Output (device arrays of the set's length): d_s[i] = s of the loss [m]
   (s = 0 at the line start, increasing through the drifts, negative for a
   loss before the line start on the way from the previous turn's last
   aperture), d_x[i], d_y[i] = its position in the line frame [m]; NaN for
   particles not lost on an aperture; d_tests (device int32 array of the
   set's length, or NULL): number of polygon tests made for each particle
   (sub-step ends and bisection points; 0 for particles not refined).  A
   particle whose path never leaves the
   interpolated polygon, or whose backtracking meets an imaginary
   longitudinal momentum, gets s of e_L and its position there.  Radiation is
   not undone.  Arguments: n_vertices 4..4096, ds > 0 (at most 1e8 sub-steps
   per drift), n_bisect 0..60.  XTM_E_UNSUPPORTED when a rectangular aperture
   does not contain its own origin.  The polygon geometry is built on the
   host and kept on the lattice for the last n_vertices (first call with a
   new n_vertices synchronises); the kernel is stream-ordered, one thread per
   particle. */
xtm_status xtm_refine_losses(xtm_lattice lat, xtm_particles p, int32_t n_vertices, double ds,
                             int32_t n_bisect, double* d_s, double* d_x, double* d_y,
                             int32_t* d_tests, void* stream);

/* One turn of n particles (n <= 65536) from the line start, the coordinates
   recorded at the entry of every element and after the last (paper section
   "Twiss module": the lattice is probed by tracking).  d_in: device (n, 6)
   rows (x, px, y, py, zeta, delta), set up as by xtm_particles_init;
   d_out: device (n_el + 1) x n x 6, element-major: d_out[(e n + i) 6 + c]
   holds particle i entering element e (e = n_el: after the turn); 16-byte
   aligned (XTM_E_ARG otherwise).
   Apertures are not checked (optics of the bare lattice); a particle whose
   longitudinal momentum becomes imaginary in a drift keeps the coordinates
   it entered that drift with; no radiation.  One thread per particle, in
   a kernel generated from the lattice's cell structure and compiled at the
   lattice's first call (as the per-line tracking kernels; a line without a
   cell decomposition runs the element interpreter, with the same maps and
   records); stream-ordered. */
xtm_status xtm_track_record(xtm_lattice lat, const double* d_in, int64_t n, double* d_out,
                            void* stream);

/* Linear optics by tracking (paper section "Twiss module"), transverse and
   uncoupled, at a fixed momentum deviation delta0 (zeta starts at 0 and the
   longitudinal plane is not part of the orbit):
     1. closed orbit u* = T(u*) of the one-turn map on (x, px, y, py) by
        Newton's method, u <- u + (I - J)^-1 (T(u) - u), from co_guess (host,
        4 values, or NULL for 0) until the largest component of T(u) - u is
        at most tol, stops decreasing, or max_iter steps were made;
     2. J by central differences of particles displaced by +-h along each
        coordinate, the momentum column by +-hd in delta (11 particles
        tracked with xtm_track_record);
     3. the same differences at every element give the map M_e from the line
        start and its momentum column m_e;
     4. per plane, from the one-turn block [[a, b], [c, d]]:
        cos mu = (a + d)/2, sin mu = sign(b) sqrt(1 - cos^2 mu),
        beta0 = b/sin mu, alpha0 = (a - d)/(2 sin mu); at element e with block
        [[p, q], [r, t]] of M_e: beta = ((p beta0 - q alpha0)^2 + q^2)/beta0,
        alpha = -((p beta0 - q alpha0)(r beta0 - t alpha0) + q t)/beta0,
        phase = atan2(q, p beta0 - q alpha0), unwrapped to increase;
     5. dispersion eta_0 = (I - J)^-1 m, eta_e = M_e eta_0 + m_e.
   h_table: host, (n_el + 1) rows of 15 doubles: s, x, px, y, py (closed
   orbit), betx, alfx, mux, bety, alfy, muy, dx, dpx, dy, dpy at the entry of
   each element and at the line end.  summary: tunes (mu at the end / 2 pi),
   the closed orbit at the start, Newton steps made and the last residual.
   XTM_E_UNSUPPORTED for an unstable or integer/half-integer one-turn map.
   Step sizes: the tracked coordinates carry rounding of about 1e-16 of the
   orbit's size, so the maps carry about that divided by h; h ~ 1e-9 suits an
   orbit on the axis, h ~ 1e-6 an orbit of millimetres (truncation stays
   small for a nearly linear map).  Synchronising; allocates its own device
   scratch. */
typedef struct xtm_twiss_summary {
  double qx, qy;
  double co[4];
  int32_t iterations;
  int32_t pad;
  double residual;
} xtm_twiss_summary;
xtm_status xtm_twiss(xtm_lattice lat, double delta0, double h, double hd, int32_t max_iter,
                     double tol, const double* co_guess, double* h_table,
                     xtm_twiss_summary* summary, void* stream);

/* Transverse optics with linear coupling (paper section "Twiss module":
   the linear normal form from the eigenvalues and eigenvectors of the
   one-turn Jacobian, eigenvectors propagated by tracking).  From xtm_twiss's
   closed orbit (same arguments), the 4x4 one-turn map J and the maps M_e to
   every element (central differences of 9 recorded particles): the
   eigenvalues from lambda + 1/lambda = t, t^2 - tr(J) t + (m2 - 2) = 0 (m2:
   sum of the principal 2x2 minors); for each, the eigenvector with
   Im(v^H S v) > 0, scaled so that v^H S v = 2i (S the 4x4 symplectic form);
   mode I is the one whose summed |v_e,x|^2 along the line exceeds its summed
   |v_e,y|^2.  h_table: host, (n_el + 1) rows of 7 doubles: s, beta_xI,
   beta_yI, beta_xII, beta_yII (|component of v_e = M_e v|^2), phase of mode
   I (argument of its x component) and of mode II (of its y component), each
   advancing through a drift by the change of the argument in [0, 2 pi) and
   through a thin element by the change in (-pi, pi].  out_q (host, 2): the
   eigen-tunes, phases at the line end / 2 pi.  XTM_E_UNSUPPORTED for an
   unstable or integer/half-integer map.  Synchronising. */
xtm_status xtm_twiss_coupled(xtm_lattice lat, double delta0, double h, double hd, int32_t max_iter,
                             double tol, double* h_table, double* out_q, void* stream);

/* Optics of a line (or of a portion of a ring, given as its own element
   list) from given initial conditions, for an assigned momentum deviation
   delta0 (paper section "Twiss module").  init (host, 12 values): x, px, y,
   py, betx, alfx, bety, alfy, dx, dpx, dy, dpy at the line start (betas
   > 0).  The orbit is the tracked initial orbit; the maps to every element
   and their momentum columns come from central differences (+-h, +-hd) of
   11 recorded particles as in xtm_twiss; beta, alpha and phase propagate as
   there from the given beta and alpha (phase from 0), the dispersion as
   M_e eta_0 + m_e from the given eta_0.  h_table: as xtm_twiss.
   Synchronising. */
xtm_status xtm_twiss_open(xtm_lattice lat, double delta0, double h, double hd, const double* init,
                          double* h_table, void* stream);

/* 6D linear normal form by tracking (paper section "Twiss module": the
   closed orbit from a root finder on the one-turn map, the Jacobian by
   central differences, the linear normal form from its eigenvalues and
   eigenvectors; with radiation the eigenvalues' moduli are the damping per
   turn, section "Synchrotron radiation models and compensation").  In
   canonical coordinates u = (x, px, y, py, zeta, pzeta), pzeta = ptau/beta0,
   with every element of the line (RF included, apertures checked) and, with
   radiation = 1, the mean energy loss of radiating multipoles:
     1. closed orbit u* = T(u*) by Newton's method u <- u + (I - J)^-1 (T(u) - u)
        from 0, J by central differences at u (13 particles tracked one turn),
        until the largest component of T(u) - u is at most tol, stops
        decreasing, or max_iter steps were made;
     2. J at u* by central differences with steps h (h_steps: host, 6 values,
        or NULL for 1e-7, 1e-9, 1e-7, 1e-9, 1e-6, 1e-8) and h/2, Richardson-
        combined (4 J(h/2) - J(h)) / 3;
     3. its eigenvalues (Hessenberg reduction, shifted QR steps); of each
        complex-conjugate pair the eigenvector with Im(v^H S v) > 0, scaled to
        v^H S v = 2i (S the 6x6 symplectic form); mode k is assigned to the
        plane p = k (x, y, longitudinal) by the assignment maximising the
        summed shares Im(conj(v_2p) v_2p+1), and its phase is set so that
        v_2k is real and positive.
   For an uncoupled plane, |v_2k|^2 is the beta function at the line start,
   and a Gaussian beam with covariance sum_k eps_k (Re v_k Re v_k^T +
   Im v_k Im v_k^T) is matched (xtm_matched_gaussian).
   XTM_E_UNSUPPORTED for a real eigenvalue (an unstable plane), a singular
   I - J or a probe particle lost.  Synchronising; allocates its scratch. */
typedef struct xtm_normal_form6 {
  double co[6];          /* closed orbit at the line start (canonical)        */
  double J[36];          /* one-turn Jacobian at the closed orbit, row-major  */
  double lam_re[3], lam_im[3];  /* eigenvalue of mode k                       */
  double q[3];           /* tune of mode k: arg(lambda_k) / 2 pi, in [0, 1)   */
  double damping[3];     /* -ln |lambda_k| per turn (0 without radiation)     */
  double v_re[18], v_im[18];    /* eigenvector of mode k: components 6k..6k+5 */
  int32_t iterations;    /* Newton steps made                                 */
  int32_t pad;
  double residual;       /* largest component of T(u) - u at the last step    */
} xtm_normal_form6;
xtm_status xtm_twiss6d(xtm_lattice lat, int32_t radiation, const double* h_steps, int32_t max_iter,
                       double tol, xtm_normal_form6* out, void* stream);

/* Step 3 of xtm_twiss6d alone, for a given one-turn Jacobian J (host,
   row-major 6x6, canonical coordinates): fills everything of `out` but the
   closed orbit (zero), iterations and residual.  Host only. */
xtm_status xtm_normal_form_of_map(const double* J, xtm_normal_form6* out);

/* Gaussian ensemble matched to a 6D normal form (paper section "Twiss
   module": matched particle distributions from the linear normal form):
   particle i from six standard normal deviates g = h_gauss[6i .. 6i+5]
   (host, supplied by the caller): u = co + sum_k Re(v_k z_k) with
   z_k = sqrt(eps_k) (g_2k + i g_2k+1), eps = host[3] emittances of the three
   modes [m] (0 allowed); written to h_out[6i ..] as (x, px, y, py, zeta,
   delta), delta = w / (1 + sqrt(1 + w)) from ptau = beta0 pzeta,
   w = ptau (ptau + 2/beta0), ready for xtm_particles_init.  Host only. */
xtm_status xtm_matched_gaussian(const xtm_normal_form6* nf, const xtm_reference* ref,
                                const double eps[3], const double* h_gauss, int64_t n,
                                double* h_out);

/* Chromaticity by tracking (paper section "Twiss module": tunes and
   chromaticities measured on the tracking model): out_dq[0..1] (host) =
   (Q(delta0 + eps) - Q(delta0 - eps)) / (2 eps) for the horizontal and
   vertical tunes of xtm_twiss (same h, hd, max_iter, tol; each side finds its
   own closed orbit).  Synchronising. */
xtm_status xtm_chromaticity(xtm_lattice lat, double delta0, double eps, double h, double hd,
                            int32_t max_iter, double tol, double* out_dq, void* stream);

/* Copy the loss record into host buffers of the bound length (any may be
   NULL).  Synchronises the stream. */
xtm_status xtm_get_losses(xtm_particles p, int32_t* h_state, int32_t* h_at_turn,
                          int32_t* h_at_element, void* stream);

/* Raw Philox4x32-10 stream (Salmon et al., SC'11, "Parallel random numbers:
   as easy as 1, 2, 3"): block j (0 <= j < n_blocks) is the 4-word output for
   counter ctr0 + j (128-bit increment, ctr0 in host memory, word 0 least
   significant) and key (seed_lo, seed_hi), written to d_out[4j .. 4j+3]
   (device memory).  Radiation (paper section "Synchrotron radiation models
   and compensation") draws its Gaussians from this generator: counter
   (particle_id_lo, particle_id_hi, turn, element * 8), uniforms
   u = ((w_a << 20 | w_b >> 12) + 1/2) 2^-52 from words (0,1) and (2,3), and
   g = sqrt(-2 ln u1) cos(2 pi u2).  Mean radiation loss of a multipole of
   length Lr with field kick k: dE = (2/3) r m gamma^4 h^2 Lr, h = |k| rpp / Lr;
   quantum part sqrt(55/(24 sqrt 3) r m hbar_c gamma^7 |h|^3 Lr) g.
   Stream-ordered. */
xtm_status xtm_philox4x32_10(uint64_t seed, const uint32_t ctr0[4], int64_t n_blocks,
                             uint32_t* d_out, void* stream);

/* Photon-by-photon radiation (radiation = 3; paper section "Synchrotron
   radiation models and compensation": the quantum model emits individual
   photons).  After the kick of a multipole of radiation length Lr > 0, with
   h = |k| rpp / Lr and gamma = gamma0 (1 + beta0 ptau): photons arrive as a
   Poisson process of mean count nbar = (5/(2 sqrt 3)) (r m / hbar_c) gamma h Lr;
   photon j (j = 0, 1, ...; at most 255) uses Philox4x32-10 block (key seed,
   counter (pid_lo, pid_hi, turn, element * 256 + j)): its uniforms u1, u2
   (words 0,1 and 2,3, as for the Gaussian model) give the arrival
   t_j = t_{j-1} - ln u1 (t_{-1} = 0; emission stops at the first t_j > nbar)
   and the energy x_j u_c, u_c = (3/2) hbar_c gamma^3 h, x_j = g^3 where g
   interpolates this table linearly at s = -ln u2: h_out[i] = g(i / 64), the
   cube root of the photon energy (in units of u_c) exceeded with probability
   exp(-i/64) under the universal synchrotron photon-number spectrum
   3/(5 pi) int_x^inf K_{5/3}(t) dt, each value rounded to single precision.
   The loss sum_j x_j u_c is taken from ptau at once (delta, rpp, rvv follow;
   px, py keep their angles); its mean and variance are those of the mean and
   Gaussian models.  Host only; n must be XTM_PHOTON_TABLE_NODES; the table is
   computed once per process (a fraction of a second). */
#define XTM_PHOTON_TABLE_NODES 2433
xtm_status xtm_photon_table(double* h_out, int32_t n);

/* ---------------------------------------------------------------------------
   Batched tracking of lattice variants (e.g. the same machine under different
   field-error seeds) in one launch per chunk.  A batch references
   n_variants lattices (not copied: they must outlive the batch) with the same
   element count and reference.  One particle set holds all variants' particles:
   variant v owns slots first_slot[v] .. first_slot[v+1]-1 (host array of
   n_variants + 1 ascending values from 0 to the set's size).  Each particle
   follows exactly the maps of its own variant, so the results equal tracking
   each variant's particles through its lattice alone, bit for bit.  Forward
   only.  Kernels: when every variant has the same element structure (types
   and orders, element by element; only parameter values differ, as for
   error seeds) the one-wave per-line forms (6, 8, 10, 12, 13; the default is 10):
   one generated kernel holds every variant's parameters and a wave whose
   lanes span several variants makes one pass per variant; otherwise, or with
   variant 4, the register-loss interpreter.  The options and statistics are
   those of xtm_track.  XTM_E_ARG for a bad partition, XTM_E_REFERENCE for
   mixed references, XTM_E_UNSUPPORTED for other kernel variants, for a
   per-line form asked of variants with different structures, or backward
   tracking. */
typedef struct xtm_batch_s* xtm_batch;
xtm_status xtm_batch_create(const xtm_lattice* lattices, int32_t n_variants, xtm_batch* out);
xtm_status xtm_batch_destroy(xtm_batch b);
xtm_status xtm_track_batched(xtm_batch b, xtm_particles p, const int64_t* first_slot,
                             int32_t n_turns, const xtm_track_opts* opts, void* stream,
                             xtm_track_stats* stats);

/* Launch-plan autotuner.  Times candidate plans on a scratch copy of the
   set (the set itself is not advanced), each for probe_turns turns through
   the ordinary tracking path, and keeps the fastest as the plan of the
   lattice (or batch).  The search runs in three stages: (1) every kernel
   form (the per-line kernel's forms 5..xtm_max_variant() when the line has
   one, each with its own workgroup size; the interpreter 4 with blocks of 64,
   128 and 256 lanes) with automatic chunks compacted after each chunk;
   (2) for that form, the turns per chunk K in {1, 4, 16, 64, 256, 1024} up to
   probe_turns, besides the automatic length; (3) for that form and K, the
   compaction period 2, 4 or 8 chunks besides 1.  With warm_turns > 0 the
   copy is first tracked warm_turns turns (with the plan then in force, not
   timed) and every probe starts from there: a dynamic-aperture scan loses
   most of its lost particles in its first turns, and the probe should see
   the alive count and loss rate of the long stretch the plan is for.  Later
   xtm_track / xtm_track_batched calls use the plan's form and block when
   their options leave both `variant` and `block` at 0, its K when
   turns_per_chunk is 0 (reached by a ramp from one turn) and its period
   when compact_every is 0.  Give exactly one of `lat` and `batch`
   (`first_slot` as for xtm_track_batched with a batch, else ignored).
   Synchronises; allocates one scratch set of the same size (two with
   warm_turns). */
typedef struct xtm_plan {
  int32_t variant;          /* kernel variant chosen (4 or a per-line form) */
  int32_t block;            /* lanes per workgroup chosen */
  double passes_per_s;      /* its measured rate, chunk epilogues included */
  int32_t turns_per_chunk;  /* turns per chunk chosen, 0 = automatic */
  int32_t compact_every;    /* compaction period chosen, in chunks */
} xtm_plan;
xtm_status xtm_autotune(xtm_lattice lat, xtm_batch batch, xtm_particles p,
                        const int64_t* first_slot, int32_t probe_turns, int32_t warm_turns,
                        void* stream, xtm_plan* out);

/* ---------------------------------------------------------------------------
   Learned early stop.  The paper cites machine-learned dynamic-aperture
   estimates beside chaos indicators (applications, dynamic aperture) without
   fixing a model; the network, its features and the retire policy below are
   this library's reading.  All buffers are caller-owned device memory, all
   calls are ordered on `stream` and return without synchronising unless
   stated otherwise.  Arithmetic: FP32 features; BF16 GEMM operands (round to
   nearest even) with FP32 accumulation; FP32 bias, ReLU, sigmoid and loss.

   Network 16 -> 128 (ReLU) -> 128 (ReLU) -> 1 logit.  Parameter vector theta,
   XTM_MLP_PARAMS FP32: W1[16][128], b1[128], W2[128][128], b2[128], w3[128],
   b3[1], with W[i][j] mapping input i to output j.  Input normalisation
   `norm` (32 FP32): mean[16] then inverse standard deviation[16]; the network
   sees (x - mean) * inv_std. */
#define XTM_MLP_PARAMS 18817
#define XTM_N_FEATURES 16
#define XTM_RECORD_TURNS 1024

/* 16 FP32 features per particle from a 1024-turn record (xtm_track_opts
   record_buf, record_turns = 1024): with u = x / sqrt(beta),
   pu = (alpha x + beta px) / sqrt(beta), J = (u^2 + pu^2) / 2 and
   A = sqrt(2 J / emit):
     f0, f1 A_x, A_y at turn 0; f2 hypot(f0, f1); f3 atan2(f1, f0);
     f4, f5 tunes of turns 0..511; f6, f7 tunes of turns 512..1023 (Hann
     window, 512-point DFT of u - i pu, peak bin with the Hann three-point
     interpolation); f8, f9 log10 of the circular tune change + 1e-12;
     f10, f11 mean J of the last quarter over that of the first (each + 1e-6
     emit) - 1; f12, f13 std(J) / (mean(J) + 1e-6 emit) over all turns;
     f14 max hypot(x, y) / r_aperture; f15 max (A_x^2 + A_y^2) / (f2^2 + 1e-6).
   twiss4 = (beta_x, alpha_x, beta_y, alpha_y) at element 0; emit [m] defines
   one sigma.  d_feat: [n][16].  Rows of particles lost before turn 1024 hold
   values computed from a partly stale record; the caller masks them.
   XTM_E_ARG for non-positive beta, emit or aperture. */
xtm_status xtm_features(const float* d_record, int64_t n, const double twiss4[4], double emit,
                        double r_aperture, float* d_feat, void* stream);

/* Normalisation statistics of the rows i with d_mask[i] != 0 (all rows when
   d_mask is NULL): d_norm[0..15] = mean, d_norm[16..31] = 1 / std (population
   std; 1 when the std is 0 or no row is selected). */
xtm_status xtm_feature_stats(const float* d_feat, const int32_t* d_mask, int64_t n, float* d_norm,
                             void* stream);

/* He-normal initialisation: weight k of theta (packed index) is
   sqrt(2 / fan_in) times the Gaussian deviate of (seed, particle id k, turn 0,
   element 0, draw 0) of the Philox stream used for radiation; biases 0. */
xtm_status xtm_mlp_init(float* d_theta, uint64_t seed, void* stream);

/* Logits of B rows of d_x [B][16] (raw features, normalised inside). */
xtm_status xtm_mlp_forward(const float* d_theta, const float* d_norm, const float* d_x, int64_t B,
                           float* d_logit, void* stream);

/* Size in floats of the workspace xtm_mlp_grad needs for a batch of B. */
xtm_status xtm_mlp_workspace(int64_t B, int64_t* n_floats);

/* Gradient of the mean positively weighted binary cross-entropy
   mean(-[w y log s(z) + (1 - y) log(1 - s(z))]) over the batch (y in {0, 1},
   w = pos_weight) with respect to theta, into d_grad[XTM_MLP_PARAMS]; the
   loss into d_loss[0] when d_loss is non-NULL.  The back-propagated signals
   are rounded to BF16 where they enter a GEMM.  d_work: xtm_mlp_workspace
   floats.  B >= 1. */
xtm_status xtm_mlp_grad(const float* d_theta, const float* d_norm, const float* d_x,
                        const float* d_y, int64_t B, float pos_weight, float* d_grad,
                        float* d_loss, float* d_work, void* stream);

/* xtm_mlp_grad without a workspace argument and without any device
   allocation, for callers that cannot allocate: code recorded into a HIP
   graph, tight training or serving loops, harnesses that forbid hipMalloc.
   Same arithmetic and kernels as xtm_mlp_grad, so the results are bitwise
   those of xtm_mlp_grad with a caller workspace.  The per-block partial
   gradients go to a fixed device array of the library (4.6 MiB on each
   device it runs on, held until the process ends; its address is looked up
   once per device at the first call there).  B must be 1..4096, otherwise
   XTM_E_ARG.  Every call on one device shares that array: calls that
   overlap on one device (different streams, or host threads) race and must
   be serialised by the caller; stream-ordered calls on one stream are safe.
   Stream-ordered, no synchronisation. */
xtm_status xtm_mlp_grad_noalloc(const float* d_theta, const float* d_norm, const float* d_x,
                                const float* d_y, int64_t B, float pos_weight, float* d_grad,
                                float* d_loss, void* stream);

/* One Adam step (Kingma & Ba 2015; beta1 0.9, beta2 0.999, eps 1e-8) on the
   FP32 master parameters, step counted from 1; d_m, d_v start at zero. */
xtm_status xtm_mlp_adam(float* d_theta, float* d_m, float* d_v, const float* d_grad, int32_t step,
                        float lr, void* stream);

/* Training loop: `epochs` passes over the n rows of (d_x [n][16], d_y [n]),
   each in mini-batches of `batch` rows (the last one shorter) taken in the
   order of a fresh host-side permutation per epoch (Fisher-Yates driven by a
   64-bit Mersenne twister seeded with shuffle_seed); per batch one
   xtm_mlp_grad and one xtm_mlp_adam step.  *step is the Adam step counter
   (0 before the first step; advanced by the number of batches).
   h_epoch_loss[epochs] (or NULL) receives each epoch's mean batch loss.
   Allocates its work buffers; synchronises once per epoch. */
xtm_status xtm_mlp_train(float* d_theta, float* d_m, float* d_v, const float* d_norm,
                         const float* d_x, const float* d_y, int64_t n, float pos_weight,
                         int32_t epochs, int32_t batch, float lr, uint64_t shuffle_seed,
                         int32_t* step, float* h_epoch_loss, void* stream);

/* Retire threshold from held-out data: the smallest logit value tau among
   the rows such that, of the rows with logit >= tau, the fraction with label
   0 (particle lost within the horizon) is at most max_false_rate; +inf when
   no threshold qualifies.  Also reports that fraction and the number of rows
   at or above tau.  Synchronises. */
xtm_status xtm_select_threshold(const float* d_logit, const int32_t* d_label, int64_t n,
                                double max_false_rate, float* h_tau, double* h_false_rate,
                                int64_t* h_selected, void* stream);

/* Dynamic aperture of a polar scan from host arrays: particle j n_r + i is
   radius i of ray j; h_da[j] = the smallest h_radius over the ray's lost
   particles (state 0 or -1), +inf when the ray has none.  Retired particles
   (state 2) count as survivors. */
xtm_status xtm_dynamic_aperture(const int32_t* h_state, const double* h_radius, int32_t n_r,
                                int32_t n_theta, double* h_da);

/* Retire policy: every alive particle of the set (indexed by slot, as the
   set's arrays) with d_logit[slot] >= logit_threshold is retired (state 2,
   coordinates and at_turn left as they are, so it is no longer tracked and
   counts as a survivor) unless it belongs to the audit set: audited iff the
   first word of Philox4x32-10 with key audit_seed and counter (pid_lo, pid_hi,
   0xFFFFFFFF, 0) is below ceil(audit_fraction 2^32).  Audited particles stay
   alive and, when d_audit_flags (device int32, one per slot, caller-zeroed
   before the first decision) is non-NULL, get d_audit_flags[slot] = 1; the
   flags accumulate over repeated decisions and judge them all
   (xtm_audit_verdict).  Rebuilds the alive list; synchronises; the counts go
   to the host when non-NULL. */
xtm_status xtm_retire(xtm_particles P, const float* d_logit, float logit_threshold,
                      uint64_t audit_seed, double audit_fraction, int32_t* d_audit_flags,
                      int64_t* h_retired, int64_t* h_audited, void* stream);

/* Score of the same retire policy without the network: d_score[i] =
   -max(f8, f9) of row i of d_feat [n][16] (the two tune-diffusion features of
   xtm_features; NaN if either is NaN), to be thresholded like a logit. */
xtm_status xtm_rule_score(const float* d_feat, int64_t n, float* d_score, void* stream);

/* One-sided 95 % upper confidence bound of a loss fraction from n_lost of
   n_audited audited particles, Wilson's score interval with z = 1.6448536...:
   (p + z^2/(2n) + z sqrt(p (1-p)/n + z^2/(4n^2))) / (1 + z^2/n), p = k/n;
   1 when n_audited = 0.  Host only. */
xtm_status xtm_audit_upper_bound(int64_t n_lost, int64_t n_audited, double* out);

/* The audit's verdict after tracking to the horizon: the particles flagged in
   d_audit_flags (xtm_retire) are the audit; h_audited = their number,
   h_lost = how many of them are lost (state 0 or -1), h_upper = the bound of
   xtm_audit_upper_bound, h_fallback = 1 iff some particle is retired
   (state 2) and h_upper > fallback_rate (the retirements are then not
   trusted and xtm_resume_retired should follow).  Any output may be NULL.
   Synchronises. */
xtm_status xtm_audit_verdict(xtm_particles P, const int32_t* d_audit_flags, double fallback_rate,
                             int64_t* h_audited, int64_t* h_lost, double* h_upper,
                             int32_t* h_fallback, void* stream);

/* Full-tracking fallback: every retired particle (state 2) resumes from the
   coordinates and the turn (its at_turn) it was retired at and is tracked
   through `lat` up to the set's current turn (the horizon), as if it had
   never been retired; particles in other states are not touched.  The
   particles retired at one turn are tracked together, joined by those of
   the next retirement turn when they reach it, so the results equal those
   of uninterrupted tracking bit for bit.  Afterwards the set's alive list
   holds every particle alive at the horizon.  Options as for xtm_track
   (no recorder, no graph); stats (or NULL) sum the launches made.
   Synchronises. */
xtm_status xtm_resume_retired(xtm_lattice lat, xtm_particles P, const xtm_track_opts* opts,
                              void* stream, xtm_track_stats* stats);

/* Synchronise the stream and report any asynchronous device error. */
xtm_status xtm_sync(void* stream);

#ifdef __cplusplus
}
#endif
#endif /* XTM_H */
