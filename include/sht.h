/*
 * sht.h -- C ABI of the MI355X spin spherical-harmonic transform library.
 *
 * Implements the fast spin SHT of McEwen, "Fast, exact (but unstable) spin
 * spherical harmonic transforms" (arXiv:0807.4494): separation of variables
 * into a 2-D Fourier transform on the torus (Section 3.2, Eq. (sht_inv_fast))
 * and an O(L^3) contraction with Wigner functions at pi/2 (Eq. (fourier_coeff)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * L        band-limit: degrees 0 <= l < L.  N = 2L - 1 samples per torus axis.
 *          (The paper writes the largest degree as its band-limit, with
 *          N = 2 L_paper + 1; L here is L_paper + 1.)  1 <= L <= SHT_L_MAX
 *          (L = 1 is the single monopole sample).
 * spin     integer s with |s| < L.  Coefficients with l < |s| do not exist
 *          (Section 2.3): they are ignored on input and written as 0.
 * batch    number of maps per call, 1 <= batch <= SHT_BATCH_MAX.
 * sampling SHT_SAMPLING_MW: the equiangular nodes of Eq. (nodes_theta) and
 *          Eq. (nodes_phi), theta_t = pi (2t+1)/N for t = 0..L-1 (the ring
 *          theta = pi is kept) and phi_p = pi (2p+1)/N for p = 0..N-1.
 * precision
 *          SHT_FP64   all arithmetic in FP64 (FP64 MFMA contraction).
 *          SHT_FP32   Wigner recursion in FP64, contraction on FP32 MFMA with
 *                     FP32 accumulation, FFT stages in FP32.
 *          SHT_BF16X3 Wigner recursion in FP64, contraction as three BF16
 *                     MFMA products (hi*hi + hi*lo + lo*hi) with FP32
 *                     accumulation, FFT stages in FP32.
 *
 * Memory layouts (device memory, row-major, complex = interleaved re, im):
 *   flm  [batch][L*L]        coefficient f_lm at index l*l + l + m.
 *   map  [batch][L][N]       sample f(theta_t, phi_p) at [t][p].
 *   Element type: complex double for SHT_FP64, complex float otherwise.
 *   flm and map must be aligned to their complex element (16 bytes for
 *   SHT_FP64, 8 otherwise) and the workspace to 256 bytes
 *   (SHT_ERR_ALIGNMENT otherwise).
 *
 * Ownership: the caller owns flm, map and workspace and keeps them alive
 * until the stream reaches the call.  The library owns its plan cache (Wigner
 * seed tables, chirp tables, FFT kernels; device memory per (device, L,
 * precision) and per (device, L, spin)) until sht_release_all().
 *
 * Semantics: every transform call only enqueues work on `stream` (a
 * hipStream_t; NULL = the legacy default stream) and returns.  The first call
 * for a new (L, spin) on a device builds its plan: it allocates device memory,
 * runs the plan kernels on a stream of the library's own (one per device,
 * default priority) and waits for them, but not for the work already queued
 * on `stream`.  Results are deterministic for a given (L, spin, batch,
 * precision).  Calls may be made from several host threads: plans are built
 * one at a time, and calls whose plans are resident do not wait for a build.
 *
 * Errors: 0 on success, a negative SHT_ERR_* code otherwise.  All argument
 * checks run before any HIP call; a failed check enqueues nothing.  No C++
 * exception crosses this interface.  sht_status_string() gives the text.
 */
#ifndef SHT_H
#define SHT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SHT_VERSION 10000          /* 1.0.0 */
#define SHT_L_MAX 4096
#define SHT_BATCH_MAX 64
#define SHT_TRI_L_MAX 512          /* largest L of sht_forward_triangular / _lstsq */
#define SHT_MULTI_SEG_MAX 8        /* spin segments of one sht_*_multi call */

enum sht_status {
    SHT_OK = 0,
    SHT_ERR_INVALID_ARG = -1,   /* L, spin, batch out of range, NULL pointer */
    SHT_ERR_UNSUPPORTED = -2,   /* unknown sampling or precision */
    SHT_ERR_WORKSPACE = -3,     /* ws_bytes < sht_workspace_bytes(...) */
    SHT_ERR_ALIGNMENT = -4,     /* flm / map not element-aligned, workspace not 256-byte aligned */
    SHT_ERR_OOM = -5,           /* plan allocation failed */
    SHT_ERR_HIP = -6,           /* a HIP call or kernel launch failed */
    SHT_ERR_BUSY = -7,          /* the resource is in use (sht_plan_tables: a captured graph reads the table) */
    SHT_ERR_NOT_READY = -8      /* a call that allocates nothing found its plan missing */
};

enum sht_sampling { SHT_SAMPLING_MW = 0 };

enum sht_precision { SHT_FP64 = 0, SHT_FP32 = 1, SHT_BF16X3 = 2 };

/*
 * Inverse transform, Eq. (ssht_inv): f(theta_t, phi_p) = sum_{l,m} f_lm sY_lm,
 * with sY_lm = (-1)^s sqrt((2l+1)/4pi) d^l_{m,-s}(theta) e^{i m phi}
 * (Eq. (ssh_wigner)), computed as the contraction Eq. (fourier_coeff) followed
 * by the torus sum Eq. (sht_inv_fast) on the sampling nodes (Section 3.4.3).
 *   flm        in:  [batch][L*L] complex
 *   map        out: [batch][L][2L-1] complex
 *   workspace  scratch of at least sht_workspace_bytes(...) bytes (device)
 *   stream     hipStream_t to enqueue on
 */
int sht_inverse(int L, int spin, int batch, int sampling, int precision,
                const void *flm, void *map, void *workspace, size_t ws_bytes,
                void *stream);

/*
 * Forward transform, Eq. (ssht_fwd): f_lm = integral of f sY*_lm over the
 * sphere.  Computed exactly for band-limited maps: phi DFT, per-order parity
 * extension in theta (Section 3.2), theta DFT (Eq. (fourier_series)), the
 * exact sin(theta) quadrature on the torus, and the contraction with the
 * Wigner functions of the conjugated Eq. (shf_exp).
 *   map        in:  [batch][L][2L-1] complex
 *   flm        out: [batch][L*L] complex (entries with l < |spin| are 0)
 */
int sht_forward(int L, int spin, int batch, int sampling, int precision,
                const void *map, void *flm, void *workspace, size_t ws_bytes,
                void *stream);

/*
 * Maps of several spins at one band-limit in one call (a serving loop's
 * same-L group): nseg segments, segment k holding batches[k] maps of spin
 * spins[k], stored one after another in flm and map (segment 0's maps first;
 * layouts per map as for sht_inverse / sht_forward).  The result of each map
 * is that of sht_inverse / sht_forward at its spin.  The layout, theta and
 * phi stages run one launch each over all maps (the layout and theta kernels
 * look up each map's segment); the O(L^3) contraction runs one launch per
 * kernel it needs, its column blocks carrying their segment's spin factors
 * (on the FP32 path the spin-0 segments take the kernel that skips the
 * products Delta^l_{m',0}(pi/2) = 0 of odd l + m', the others one launch).
 *
 * Spin pairs.  A segment of spin -s that directly follows one of spin s != 0
 * (not itself so paired) shares that segment's contraction: at theta = pi/2,
 * Delta^l_{m',s} = (-1)^{l+m'} Delta^l_{m',-s} (Eq. (wignerd_sym6)), so its
 * columns join the column range of s, contracted with the factors of s, and
 * the layout and theta stages apply the signs (-1)^l and (-1)^{m'}.  Each
 * Wigner entry the contraction generates then serves both spins' maps (on
 * the FP32 path in one 128-column tile: 16 maps of s and 16 of -s).  The
 * paired maps agree with their own single-spin calls to rounding (the two
 * spins' factor tables are tabulated separately); every other map's result
 * is bitwise that of its single-spin call.  Order the segments
 * {s, -s, ...} to get the sharing.
 *   nseg       1 <= nseg <= SHT_MULTI_SEG_MAX
 *   spins, batches  host arrays of nseg entries: |spins[k]| < L,
 *              batches[k] >= 1, sum of batches <= SHT_BATCH_MAX
 *   workspace  sht_workspace_bytes(L, 0, sum of batches, sampling, precision)
 * Errors, ownership and semantics as for sht_inverse / sht_forward.
 */
int sht_inverse_multi(int L, int nseg, const int *spins, const int *batches, int sampling, int precision,
                      const void *flm, void *map, void *workspace, size_t ws_bytes, void *stream);
int sht_forward_multi(int L, int nseg, const int *spins, const int *batches, int sampling, int precision,
                      const void *map, void *flm, void *workspace, size_t ws_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the inverse
 * transform of sht_inverse, with the workspace taken from a static device
 * array of SHT_NOALLOC_SCRATCH_BYTES bytes that the library holds on each
 * device it runs on until the process ends.  The caller still passes flm and
 * map (layouts, alignment and precisions as for sht_inverse).
 *   - The plan of (L, spin) must be resident on the current device: call
 *     sht_plan_warmup (which allocates) beforehand, else SHT_ERR_NOT_READY.
 *   - Shapes whose sht_workspace_bytes(...) exceeds SHT_NOALLOC_SCRATCH_BYTES
 *     return SHT_ERR_WORKSPACE (e.g. L = 512 fits up to 8 maps in FP32 and 4 in
 *     FP64).
 *   - The call allocates nothing: no hipMalloc / hipFree, no trace events.
 *   - Every call on one device uses that device's single array, which keeps
 *     the previous call's contents (nothing in it needs clearing): calls that
 *     overlap on one device (several streams, or several host threads) race
 *     and give wrong results; serialise them.
 * Errors as for sht_inverse, plus SHT_ERR_NOT_READY; argument, alignment and
 * size checks run before any HIP call.
 */
#define SHT_NOALLOC_SCRATCH_BYTES (64u << 20)
int sht_inverse_noalloc(int L, int spin, int batch, int sampling, int precision,
                        const void *flm, void *map, void *stream);

/*
 * Real spin-0 signals (Section 3.3): for a real map f, f_{l,-m} =
 * (-1)^m conj(f_lm), and only the orders m >= 0 are transformed (half the
 * contraction columns and half the theta-stage rows of the complex path).
 *   sht_inverse_real: flm in [batch][L*L] complex (entries with m < 0 are not
 *                     read), map out [batch][L][2L-1] REAL (double for
 *                     SHT_FP64, float otherwise).
 *   sht_forward_real: map in (real, as above), flm out [batch][L*L] complex
 *                     with every m written (m < 0 from the symmetry).
 * The map needs element alignment (8 or 4 bytes), flm complex alignment; the
 * workspace size is sht_workspace_bytes(L, 0, batch, sampling, precision).
 * Precisions and errors as for sht_inverse / sht_forward.
 */
int sht_inverse_real(int L, int batch, int sampling, int precision,
                     const void *flm, void *map, void *workspace, size_t ws_bytes,
                     void *stream);
int sht_forward_real(int L, int batch, int sampling, int precision,
                     const void *map, void *flm, void *workspace, size_t ws_bytes,
                     void *stream);

/*
 * Spin pairs (Section 3.3): when the spin -s field is the conjugate of the
 * spin s field (e.g. Q + iU and Q - iU), one transform serves both:
 *   {}_{-s}f_{lm} = (-1)^{s+m} conj({}_s f_{l,-m}),
 * and the spin -s map is the conjugate of the spin s map.  This call writes
 * the spin -s coefficients flm_ms [batch][L*L] from the spin s ones flm_s
 * (distinct buffers, complex of the precision's type; zero for l < |s|),
 * enqueued on `stream`.
 */
int sht_spin_pair(int L, int spin, int batch, int precision, const void *flm_s, void *flm_ms,
                  void *stream);

/*
 * The paper's own forward transform (Section 3.4.2): phi DFT, the per-order
 * extension and theta DFT of Section 3.2 (Eq. (fourier_series)), then for
 * each order m0 the triangular system of Eq. (matrix_fwd),
 *   F_{m0 m'} = sum_{l >= m'} (-1)^s i^{-(m0+s)} sqrt((2l+1)/4pi)
 *               d^l_{m' m0}(pi/2) d^l_{m',-s}(pi/2) f_{l m0},
 * solved on its square block of rows and columns max(|m0|, |s|) .. L-1 by
 * back substitution.  Exact for band-limited maps in exact arithmetic, but
 * the systems are ill conditioned (Section 4.2: condition number ~6e14 at
 * band-limit 50); use sht_forward for accurate results.  Provided as the
 * paper's method for comparison.
 *   precision  SHT_FP64 only (SHT_ERR_UNSUPPORTED otherwise)
 *   L          1 <= L <= SHT_TRI_L_MAX (SHT_ERR_UNSUPPORTED above)
 *   map, flm, workspace, stream: as for sht_forward (same workspace size).
 */
int sht_forward_triangular(int L, int spin, int batch, int sampling, int precision,
                           const void *map, void *flm, void *workspace, size_t ws_bytes,
                           void *stream);

/*
 * The stable comparison to sht_forward_triangular: the same per-order
 * systems of Eq. (matrix_fwd), but all their rows m' = 0..L-1 (the square
 * block plus the rows m' < max(|m0|, |s|) that the paper's solve drops),
 * solved in the least-squares sense -- not the paper's method.  Those extra
 * rows make the systems well conditioned, so the result stays at FP64
 * rounding where the triangular solve loses all accuracy (Section 4.2).
 * Solved on the GPU by conjugate gradients on the normal equations until
 * the normal-equation residual has fallen by 1e-14 (at most 2L + 32
 * iterations).
 *   Arguments, precision, L limit, workspace and errors: as for
 *   sht_forward_triangular.
 */
int sht_forward_lstsq(int L, int spin, int batch, int sampling, int precision,
                      const void *map, void *flm, void *workspace, size_t ws_bytes,
                      void *stream);

/* Workspace bytes needed by sht_inverse / sht_forward with these arguments
 * (the same size serves both directions).  0 if the arguments are invalid. */
size_t sht_workspace_bytes(int L, int spin, int batch, int sampling, int precision);

/* Build (or find) the plan for (L, spin, precision) on the current device
 * (the plan kernels run on the library's own stream and are waited for;
 * `stream` is not used).  Optional: transforms build plans on first use.
 * Returns SHT_OK or an error code. */
int sht_plan_warmup(int L, int spin, int sampling, int precision, void *stream);

/*
 * Cached contraction tables (a measured alternative to generating the Wigner
 * factors on the fly).  enable = 1 builds, for (L, spin) on the current
 * device, the table of M_m(m', l) = sqrt((2l+1)/4pi) d^l_{m'm}(pi/2)
 * d^l_{m',-s}(pi/2) for all 0 <= m, m', l < L -- L^3 entries in FP64 for
 * SHT_FP64, in FP32 for SHT_FP32 and SHT_BF16X3 (4 GiB at L = 1024 in FP32)
 * -- the precomputation Section 4.1 describes; from then on the transforms at
 * that (L, spin) and precision class stream M from the table instead of
 * running the recursions.  enable = 0 frees the table.  Synchronises the
 * stream.  SHT_ERR_OOM if the table does not fit.  A graph captured
 * (sht_graph_create) while the table existed reads it on every replay, so
 * enable = 0 returns SHT_ERR_BUSY, and frees nothing, until every such graph
 * has been destroyed.
 */
int sht_plan_tables(int L, int spin, int precision, int enable, void *stream);

/*
 * Captured transforms, for callers that run one shape many times (a serving
 * loop): the inverse transform of flm_in into map followed by the forward
 * transform of map into flm_out (both as sht_inverse / sht_forward, with the
 * same L, spin, batch, sampling and precision), recorded once as a HIP graph
 * and replayed by sht_graph_launch on any stream of the same device.
 *   flm_in     in:  [batch][L*L] complex, read when the graph runs
 *   map        out: [batch][L][2L-1] complex (the inverse's result)
 *   flm_out    out: [batch][L*L] complex (the forward's result)
 *   workspace  at least sht_workspace_bytes(...) bytes, used by every launch
 * The graph binds these device buffers: they stay owned by the caller, must
 * outlive the graph, and a launch overwrites map, flm_out and the workspace.
 * Launches of one graph, or of graphs sharing buffers, that overlap on
 * different streams race.  Creation builds the plan if needed (as a first
 * transform call does) and records without executing anything; *out receives the handle (NULL on
 * error).  Errors as for sht_inverse; SHT_ERR_INVALID_ARG for a NULL out or
 * an unknown handle, or a launch on another device than the creation's.
 * sht_release_all destroys every live graph.
 */
typedef struct sht_graph_s *sht_graph;
int sht_graph_create(int L, int spin, int batch, int sampling, int precision,
                     const void *flm_in, void *map, void *flm_out, void *workspace, size_t ws_bytes,
                     void *stream, sht_graph *out);
int sht_graph_launch(sht_graph graph, void *stream);
int sht_graph_destroy(sht_graph graph);

/*
 * Contraction tile shapes.  Each contraction workgroup takes 16, 32 or 64 of
 * the transform's columns (4 x batch for sht_inverse / sht_forward, 2 x batch
 * for the real-signal calls), or 128 on the FP32 path; more column blocks
 * mean the Wigner products are generated once per block, wider blocks waste
 * matrix-core work on empty columns (the 128-column tile only in 64-column
 * halves: each half skips its work when it has no columns).  By default a
 * call takes the tile t that minimises the sum over its column blocks of
 * (the block's columns rounded up to t, or to 64 for t = 128) + 24 (the
 * Wigner generation of a block costs about as much as 24 columns); several
 * spins in one call sum over their column ranges, where a spin -s that
 * follows s shares the range of s (sht_inverse_multi).  So 16 up to 16
 * columns, 32 up to 32, 64 up to 64, and 128 for the FP32 ranges of 65 to
 * 128 columns, e.g. 16 maps of s with 16 of -s.
 *
 * sht_tile_set pins the tile (16, 32 or 64, 128 for SHT_FP32; 0 restores the
 * default) for (current device, L, columns, precision).  SHT_ERR_INVALID_ARG
 * for other tiles, L outside 1..SHT_L_MAX or columns outside
 * 1..4*SHT_BATCH_MAX.
 *
 * sht_tune is the autotuner: it times the contraction kernels of the inverse
 * and the forward of (L, spin, batch, precision) with each tile, using the
 * workspace as scratch (its contents are overwritten; at least
 * sht_workspace_bytes(...) bytes), pins the fastest for those columns, writes
 * it to *tile_out (if not NULL) and synchronises the stream.  Errors as for
 * sht_inverse.
 */
int sht_tile_set(int L, int columns, int precision, int tile);
int sht_tune(int L, int spin, int batch, int precision, void *workspace, size_t ws_bytes, void *stream,
             int *tile_out);

/*
 * Error metrics of a reconstruction against a reference: the five measures
 * of the paper's round-trip stability test (Section 4.2), computed on the GPU
 * in FP64.  Over the n complex entries of ref (f) and val (g):
 *   out[0] = max |f - g|          out[1] = mean |f - g|
 *   out[2] = median |f - g|       (for even n the mean of the two middle
 *                                  values; the exact elements, by radix
 *                                  selection)
 *   out[3] = rms = sqrt(mean |f - g|^2)
 *   out[4] = relative rms = sqrt(sum |f - g|^2 / sum |f|^2), or
 *            sqrt(sum |f - g|^2) if f is all zero
 * All five are 0 for n = 0.  Finite inputs.
 *   precision  element type: SHT_FP64 complex double, SHT_FP32 / SHT_BF16X3
 *              complex float (SHT_ERR_UNSUPPORTED otherwise)
 *   ref, val   device arrays of n elements (may be NULL if n = 0), aligned
 *              to the element's real part; only read
 *   out        device array of 5 doubles, 8-byte aligned, written
 *   workspace  device scratch of at least sht_error_workspace_bytes() bytes,
 *              256-byte aligned, owned by the caller, overwritten
 *   stream     HIP stream (NULL = default); the call is asynchronous, out is
 *              ready when the stream reaches this point
 * Errors: SHT_ERR_INVALID_ARG (NULL out / workspace, NULL arrays with n > 0,
 * more than 2^40 bytes per array), SHT_ERR_ALIGNMENT, SHT_ERR_WORKSPACE,
 * SHT_ERR_HIP.  Checks run before any HIP call.
 */
size_t sht_error_workspace_bytes(void);
int sht_error_metrics(int precision, size_t n, const void *ref, const void *val, double *out, void *workspace,
                      size_t ws_bytes, void *stream);

/* Free every cached plan on every device, after destroying every live graph.
 * The caller must make sure no enqueued transform still uses them (e.g.
 * synchronise first). */
int sht_release_all(void);

/* Static text for a status code (never NULL). */
const char *sht_status_string(int status);

/* SHT_VERSION of the built library. */
int sht_version(void);

/* Text of the last HIP error seen by the library in this thread ("" if none). */
const char *sht_last_hip_error(void);

/*
 * Stage tracing (a profiling aid, off by default).  While enabled, every
 * transform records a pair of HIP events on its own stream around each of its
 * stages.  sht_trace_read() waits for the recorded events, adds each stage's
 * elapsed milliseconds into ms[stage] and its launch count into count[stage]
 * for stage < nstages (SHT_STAGE_COUNT covers them all), and forgets them.
 * Stages: SHT_STAGE_* below.  Not thread-safe against concurrent transforms.
 */
enum sht_stage {
    SHT_STAGE_LAYOUT_IN = 0,   /* inverse: coefficients -> order-major panels */
    SHT_STAGE_CONTRACT_INV,    /* inverse: Wigner chains + MFMA contraction */
    SHT_STAGE_THETA_INV,       /* inverse: theta torus sum */
    SHT_STAGE_PHI_INV,         /* inverse: phi torus sum */
    SHT_STAGE_PHI_FWD,         /* forward: phi DFT */
    SHT_STAGE_THETA_FWD,       /* forward: extension, theta DFT, quadrature */
    SHT_STAGE_CONTRACT_FWD,    /* forward: Wigner chains + MFMA contraction */
    SHT_STAGE_LAYOUT_OUT,      /* forward: panels -> coefficients */
    SHT_STAGE_COUNT
};
int sht_trace_enable(int on);
int sht_trace_read(double *ms, int *count, int nstages);

#ifdef __cplusplus
}
#endif

#endif /* SHT_H */
