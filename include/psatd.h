/*
 * psatd.h -- C ABI of the MI355X PSATD field step.
 *
 * The operation (Sec. III.B, item 2 of Blaclard, Vincenti, Lehe, Vay,
 * arXiv:1608.05739; Table 1, PSATD row): on a periodic grid, forward-FFT the
 * fields E, B and the sources J, rho; advance every k mode analytically over
 * one time step with the sources held constant during the step (dispersion
 * free, no Courant condition); inverse-FFT E and B.  The per-mode update, in
 * normalized units with the forward transform f^(k) = sum_x f(x) e^{-i k.x}:
 *
 *   E^' = C E^ + i c^2 S (k x B^) - (S/eps0) J^ + i k (X3 rho^_old - X2 rho^_new)
 *   B^' = C B^ - i S (k x E^) + i X1 (k x J^)
 *
 *   theta = c|k|dt,  C = cos theta,  S = sin theta / (c|k|),
 *   X1 = (1 - C)/(eps0 c^2 |k|^2),  X2 = (1 - sin theta/theta)/(eps0 |k|^2),
 *   X3 = (C - sin theta/theta)/(eps0 |k|^2)         (all finite at k = 0).
 *
 * (the "rho form"; the "J form" replaces the rho term by
 *  eps0 c^2 X1 k (k.E^) - dt X2 k (k.J^), which assumes continuity.)
 * The wavenumber of the Nyquist index of every (even) axis is taken as 0.
 *
 * Layout.  Every field component is a dense real array, x fastest:
 * [nz][nx] in 2D (the (x, z) plane, ny = 1) and [nz][ny][nx] in 3D.  A plan
 * may hold many independent patches; patch p occupies elements
 * [offset_p, offset_p + nx*ny*nz) of every component buffer.  Element type is
 * float (PSATD_FP32) or double (PSATD_FP64).  Buffers must be 8-byte aligned
 * (FP32) or 16-byte aligned (FP64) at every patch offset.
 *
 * Ownership.  The caller owns all field buffers and the HIP stream.  A plan
 * owns its device tables and, unless psatd_set_workspace was called, its
 * workspace; psatd_destroy frees only plan-owned memory.
 *
 * Errors.  Every function returns a psatd_status.  Argument, size and state
 * errors are detected on the host before anything is enqueued, so the fields
 * are untouched; psatd_last_error() then describes the problem (thread-local
 * text, valid until the next call on the same thread).  HIP launch errors give
 * PSATD_ERR_HIP; faults inside kernels surface at the caller's next stream
 * synchronization.  Nothing aborts or throws across this interface.
 */
#ifndef PSATD_H
#define PSATD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psatd_plan_s* psatd_plan_t;

typedef enum {
  PSATD_OK = 0,
  PSATD_ERR_INVALID_ARG = -1,      /* null pointer, bad enum, non-positive spacing or dt ... */
  PSATD_ERR_UNSUPPORTED_SIZE = -2, /* axis length not an even 2^a 3^b in [2, 4096], ...      */
  PSATD_ERR_OOM = -3,              /* device allocation failed                                */
  PSATD_ERR_HIP = -4,              /* a HIP runtime call or kernel launch failed              */
  PSATD_ERR_WORKSPACE = -5,        /* workspace missing, too small or misaligned              */
  PSATD_ERR_STATE = -6             /* call not valid in the plan's current state              */
} psatd_status;

enum { PSATD_FP32 = 0, PSATD_FP64 = 1 };                               /* field element type */
enum { PSATD_VACUUM = 0, PSATD_SOURCES_RHO = 1, PSATD_SOURCES_J = 2 }; /* update form        */
/* Kernel composition.  PLAIN: separate z transforms and a per-mode update
 * pass.  FUSED: one pass runs the forward z transforms, the update and the
 * inverse z transforms of whole z lines in a workgroup; where the z lines of
 * the plan are too long for one workgroup (nz above 4096 FP32 2D, 2048 FP64
 * 2D or FP32 3D, 1024 FP64 3D) it runs the plain z passes instead.  Same
 * results up to rounding either way. */
enum { PSATD_PATH_FUSED = 0, PSATD_PATH_PLAIN = 1 };

/* psatd_config.flags */
/* Time each pass alone at plan time (on scratch fields) over its candidate
 * launch grids, tiles (lines per workgroup), modes per thread (fused pass) and,
 * for the generic line passes, both radix schedules (PSATD_FLAG_RADIX4_LINES
 * below or not); keep the fastest.  Grid and tile choices do not change
 * results; the radix schedule changes them in the last bits. */
#define PSATD_FLAG_AUTOTUNE 0x1u
/* Capture one step into a hipGraph at plan time (or in psatd_set_workspace when
 * the plan has no workspace yet); psatd_push then writes the field pointers
 * into a plan-owned device table (one small kernel) and replays the graph
 * nsteps times.  Pushes on a stream that the caller is capturing enqueue the
 * kernels themselves instead, so that the caller's graph records them. */
#define PSATD_FLAG_GRAPH 0x2u
#define PSATD_FLAG_NO_WORKSPACE 0x4u /* allocate no workspace: call psatd_set_workspace first */
#define PSATD_FLAG_GENERIC_KERNELS 0x8u /* never pick shape-specialized kernels (cross-checks) */
/* order p > 0: take k_p from the centered (collocated) order-p stencil,
 * sum_l a_l (2/d) sin(l k d), instead of the staggered one of Sec. III.B.
 * Its symbol vanishes smoothly at the Nyquist wavenumber, so every operator of
 * the step stays local in real space (what guard-cell decompositions need). */
#define PSATD_FLAG_CENTERED_STENCIL 0x10u
/* The PSTD contrast solver (Table 1, PSTD row) instead of PSATD: the same
 * transforms and k tables, but a leapfrog in time, E at integer and B at
 * half-integer times.  One push takes E^n, B^{n-1/2}, J^{n+1/2} to
 *   B^{n+1/2} = B^{n-1/2} - dt curl E^n,
 *   E^{n+1}   = E^n + dt (c^2 curl B^{n+1/2} - J^{n+1/2} / eps0)
 * with curl -> i k x.  source_mode must be PSATD_VACUUM or PSATD_SOURCES_J
 * (PSTD uses no rho); the generic kernels run it.  Planning fails with
 * PSATD_ERR_INVALID_ARG when c dt |k|max / 2 > 1 for a patch (its Courant
 * condition; |k|max over the patch's k table). */
#define PSATD_FLAG_PSTD 0x20u
/* The generic line passes (any size other than the 4096 x 4096 2D grid)
 * factor each line into radix-4 stages (then one radix-2 and the radix-3
 * stages) at 4 points per thread, instead of the default radices of at most 8
 * at 8 points per thread.  Half the registers, twice the waves per SIMD:
 * faster on short lines (2D patches with sides of a few hundred cells),
 * slower on long ones.  The factorization rounds differently, so results
 * differ from the default ones in the last bits.  With PSATD_FLAG_AUTOTUNE
 * both schedules are timed per pass and this flag only sets the untuned
 * starting point.  A pass with a line longer than 2048 points keeps the
 * default schedule (512 threads at 4 points hold no more). */
#define PSATD_FLAG_RADIX4_LINES 0x40u

typedef struct {
  int32_t ndim;  /* 2: (x, z) plane, n[1] must be 1;  3: (x, y, z)                   */
  int32_t reserved0;
  int64_t n[3];  /* nx, ny, nz: each an even 2^a 3^b with 2 <= n <= 4096 (ny = 1 in 2D) */
  double d[3];   /* dx, dy, dz > 0 (dy ignored in 2D)                                 */
  double dt;     /* > 0; no Courant limit                                             */
  int64_t offset;/* element offset of this patch in every component buffer           */
} psatd_patch_desc;

typedef struct {
  int32_t precision;   /* PSATD_FP32 or PSATD_FP64                                    */
  int32_t source_mode; /* PSATD_VACUUM, PSATD_SOURCES_RHO or PSATD_SOURCES_J          */
  int32_t path;        /* PSATD_PATH_FUSED or PSATD_PATH_PLAIN                        */
  int32_t order;       /* 0: exact k; even p >= 2: order-p stencil wavevector k_p
                          (staggered stencil, or centered with the flag below)      */
  double c;            /* speed of light (> 0; 1 in normalized units)                 */
  double eps0;         /* vacuum permittivity (> 0; 1 in normalized units)           */
  uint32_t flags;      /* PSATD_FLAG_*                                                */
  int32_t reserved0;
} psatd_config;

typedef struct {
  void* E[3];            /* in/out: Ex, Ey, Ez (device pointers, caller-owned)          */
  void* B[3];            /* in/out: Bx, By, Bz                                           */
  const void* J[3];      /* in: J^{n+1/2}; NULL for PSATD_VACUUM                         */
  const void* rho_old;   /* in: rho^n (PSATD_SOURCES_RHO only, else NULL)                */
  const void* rho_new;   /* in: rho^{n+1} (PSATD_SOURCES_RHO only, else NULL)            */
} psatd_fields;

/* Create a plan for npatches periodic patches on HIP device `device`.
 * Validates every descriptor, builds the 1-D k tables, FFT twiddles and r2c
 * post-twiddles in FP64 on the device, allocates the workspace (unless
 * PSATD_FLAG_NO_WORKSPACE is set), optionally autotunes, and synchronizes
 * once.  *out is set only on success. */
psatd_status psatd_plan(const psatd_config* cfg, const psatd_patch_desc* patches,
                        int32_t npatches, int32_t device, psatd_plan_t* out);

/* The plan's kernel choices as a NUL-terminated string: per pass, the
 * kernel family, tile (lines per workgroup), modes or points per thread and
 * launch grid that psatd_plan chose (by PSATD_FLAG_AUTOTUNE's timing, or its
 * defaults).  *needed (if not NULL) receives the string's size including the
 * NUL; buf may be NULL to query it, else PSATD_ERR_INVALID_ARG if len is
 * smaller.  The string is meant for psatd_plan_tuned on the same
 * configuration and patches: autotuning once and reusing its result skips
 * the timing launches at plan time, and keeps the kernel choice fixed where
 * timing would be distorted (under a profiler that serializes dispatches). */
psatd_status psatd_plan_tuning(psatd_plan_t plan, char* buf, size_t len, size_t* needed);

/* psatd_plan with the kernel choices of `tuning` (a string from
 * psatd_plan_tuning) instead of its defaults or autotuning: no timing launch
 * (PSATD_FLAG_AUTOTUNE is ignored).  Each choice is checked against the
 * candidates the autotuner would offer this plan (the same kernels, tiles and
 * grids); PSATD_ERR_INVALID_ARG if the string does not parse, has a choice
 * count other than the plan's pass count, or names a choice the plan does
 * not offer.  Results are those of the plan the string came from, bit for
 * bit.  Other errors as psatd_plan. */
psatd_status psatd_plan_tuned(const psatd_config* cfg, const psatd_patch_desc* patches,
                              int32_t npatches, int32_t device, const char* tuning,
                              psatd_plan_t* out);

/* Host-only planning: the same validation, workspace layout, pass and
 * work-list construction and work-list verification as psatd_plan, with no
 * HIP call and no device memory (the autotune and graph flags are ignored:
 * both need a device).  On success *ws_bytes (if not NULL) is the workspace
 * psatd_plan would allocate and info (if not NULL) holds the pass description
 * psatd_plan_info would give before autotuning, NUL-terminated and truncated
 * to len.  Errors are the ones psatd_plan returns for the same arguments.
 * Safe to call without a GPU; used to check the planner on the CPU. */
psatd_status psatd_plan_describe(const psatd_config* cfg, const psatd_patch_desc* patches,
                                 int32_t npatches, size_t* ws_bytes, char* info, size_t len);

/* Bytes of device workspace the plan needs: the k-space spectra of all inputs
 * (twice that in 3D, where the y passes move them between two blocks). */
psatd_status psatd_workspace_size(psatd_plan_t plan, size_t* bytes);

/* Hand the plan a caller-owned device workspace of at least
 * psatd_workspace_size() bytes, 256-byte aligned.  Frees any plan-owned
 * workspace.  The caller keeps it alive until psatd_destroy.  With
 * PSATD_FLAG_GRAPH this (re)captures the step graph, which allocates. */
psatd_status psatd_set_workspace(psatd_plan_t plan, void* device_ptr, size_t bytes);

/* Advance the fields by nsteps steps, asynchronously on `hip_stream` (a
 * hipStream_t; NULL = the default stream).  J is J^{n+1/2}, rho_old = rho^n,
 * rho_new = rho^{n+1}; with sources nsteps must be 1.  No allocation, host
 * synchronization or host copy happens here once the workspace exists (with
 * PSATD_FLAG_GRAPH as well: the graph was built beforehand), so the call can
 * be captured into a caller's hipGraph.  Not thread-safe for concurrent
 * pushes on one plan: with PSATD_FLAG_GRAPH, pushes of different fields on
 * different streams would race on the plan's field table. */
psatd_status psatd_push(psatd_plan_t plan, const psatd_fields* fields, int32_t nsteps,
                        void* hip_stream);

/* Bytes of the device-resident workspace of psatd_push_scratch. */
#define PSATD_SCRATCH_BYTES (256u << 20)

/* psatd_push for callers that cannot allocate device memory at all (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results as psatd_push, but the workspace
 * is a fixed array of PSATD_SCRATCH_BYTES bytes that the library keeps in
 * device memory, one copy per GPU, until the process ends.  The plan may be
 * created with PSATD_FLAG_NO_WORKSPACE; its own workspace, graph and
 * PSATD_FLAG_GRAPH are not used (the kernels are enqueued on hip_stream).
 * Plans whose psatd_workspace_size exceeds PSATD_SCRATCH_BYTES are rejected
 * with PSATD_ERR_WORKSPACE, nothing enqueued.  No allocation, host
 * synchronization or host copy.  Every call on one GPU shares that GPU's
 * array: calls that may overlap on one GPU (other streams, other threads,
 * other plans) race and must be ordered by the caller.  Nothing in the array
 * needs clearing: each step writes every workspace element it reads before
 * reading it. */
psatd_status psatd_push_scratch(psatd_plan_t plan, const psatd_fields* fields, int32_t nsteps,
                                void* hip_stream);

/* Like psatd_push, but records a HIP event pair around every pass on
 * `hip_stream`, synchronizes at the end and writes the mean duration of each
 * pass in milliseconds to ms_per_pass[0 .. npass-1] (npass from
 * psatd_pass_count).  A PSATD_FLAG_GRAPH plan launches each pass as a graph
 * of its own, captured at plan time like the step's graph (a pass launched
 * once per line length runs those launches as parallel branches), so each
 * pass is timed as the step's graph runs it; other plans enqueue the
 * kernels one after the other.  With sources, nsteps > 1 reuses the same J
 * and rho in every step.  For measurement only. */
psatd_status psatd_push_profiled(psatd_plan_t plan, const psatd_fields* fields,
                                 int32_t nsteps, void* hip_stream, double* ms_per_pass,
                                 int32_t max_pass);

/* Number of kernel launches (passes) per step, and the name of pass i
 * (static string, e.g. "x_r2c_fwd", "z_fused", "x_c2r_inv"). */
psatd_status psatd_pass_count(psatd_plan_t plan, int32_t* npass);
const char* psatd_pass_name(psatd_plan_t plan, int32_t i);

/* Bytes each pass reads and writes in HBM per step by the pass model (fields,
 * spectra; tables excluded).  Used to report achieved bandwidth. */
psatd_status psatd_pass_bytes(psatd_plan_t plan, int32_t i, double* bytes);

/* Human-readable description of the chosen kernels, tiles and launch shapes
 * (NUL-terminated, truncated to len). */
psatd_status psatd_plan_info(psatd_plan_t plan, char* buf, size_t len);

/* Free plan-owned device memory and the plan.  NULL is accepted. */
psatd_status psatd_destroy(psatd_plan_t plan);

const char* psatd_status_string(psatd_status status);
const char* psatd_last_error(void);

/* ---------------------------------------------------------------------------
 * Guard-cell domain decomposition (Sec. II.A: the pseudo-spectral solvers of
 * PXR split the domain into subdomains whose guard regions copy the adjacent
 * subdomains, and solve each with local FFTs; the price is a truncation error
 * that falls with the guard width for finite stencil orders p).
 *
 * A periodic global grid is split into parts[0] x parts[1] x parts[2] boxes of
 * n[a] / parts[a] cells.  Each box, extended by guard[a] cells on both sides of
 * every split axis (parts[a] > 1), is one periodic patch of an internal batched
 * plan; its side box + 2 guard must be an even 2^a 3^b <= 4096, and the x
 * guard even.  Each step of psatd_domain_push is one step of that plan, whose
 * forward x pass reads every patch, interior and guards, straight from the
 * global fields at the periodic global positions (the guard exchange: the
 * neighbours' current values; sources likewise), and whose inverse x pass
 * writes each patch's interior straight back to its box of the global E and
 * B.  No local copy of the fields is made.
 * The guard cells introduce the truncation error; use order p > 0 with
 * PSATD_FLAG_CENTERED_STENCIL for operators that stay local.
 * ------------------------------------------------------------------------- */
typedef struct psatd_domain_s* psatd_domain_t;

typedef struct {
  int32_t ndim;     /* 2: (x, z) plane, n[1] = parts[1] = 1;  3: (x, y, z)         */
  int32_t reserved0;
  int64_t n[3];     /* global nx, ny, nz (periodic)                                */
  int32_t parts[3]; /* boxes per axis, each dividing n[a]                          */
  int32_t guard[3]; /* guard cells per side on split axes (ignored where parts = 1) */
  double d[3];      /* dx, dy, dz > 0                                              */
  double dt;        /* > 0                                                         */
} psatd_domain_desc;

/* Build the decomposition and its internal plan (same config; the config's
 * flags apply to it; its x passes are the generic kernels, which read and
 * write through the patches' places in the global grid).  Allocates the
 * plan's workspace.  Errors as psatd_plan; PSATD_ERR_UNSUPPORTED_SIZE if a
 * local side is not a supported length; PSATD_ERR_INVALID_ARG for an odd x
 * guard on a split x axis. */
psatd_status psatd_domain_create(const psatd_config* config, const psatd_domain_desc* domain,
                                 int32_t device, psatd_domain_t* out);

/* Number of local patches and their shape (nx, ny, nz incl. guards). */
psatd_status psatd_domain_local_shape(psatd_domain_t domain, int64_t* npatch, int64_t local_n[3]);

/* Advance the global fields by nsteps decomposed steps on hip_stream (E, B of
 * the global grid in place; J, rho as in psatd_push; nsteps > 1 in vacuum
 * only).  Asynchronous, no allocation. */
psatd_status psatd_domain_push(psatd_domain_t domain, const psatd_fields* global_fields,
                               int32_t nsteps, void* hip_stream);

psatd_status psatd_domain_destroy(psatd_domain_t domain);

/* ---------------------------------------------------------------------------
 * FDTD contrast solvers (Sec. III.A; Table 1, Yee, CKC and FDTD p-order rows):
 * the finite-difference schemes the paper measures PSATD against.  No kernel
 * is shared with the PSATD path.
 *
 * Leapfrog: E at integer times, B at half-integer times.  One step takes
 * E^n, B^{n-1/2}, J^{n+1/2} to
 *   B^{n+1/2} = B^{n-1/2} - dt curl+ E^n
 *   E^{n+1}   = E^n + dt (c^2 curl- B^{n+1/2} - J^{n+1/2} / eps0)
 * on the periodic Yee grid.  Each component array is dense [nz][ny][nx]
 * (x fastest; [nz][nx] in 2D) at the patch's offset, element (i, j, k)
 * holding the component at its staggered position:
 *   Ex (i+1/2, j, k)  Ey (i, j+1/2, k)  Ez (i, j, k+1/2)   (J likewise)
 *   Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
 * curl+ uses forward and curl- backward differences with the staggered
 * order-p weights C_l of Sec. III.B (p = 2: nearest neighbours, the Yee
 * scheme).  PSATD_FDTD_CKC (2D, dx = dz, order 2) averages, in curl+ only,
 * each x-difference over z and each z-difference over x with weights
 * (3/4, 1/8, 1/8) (beta = 1/4).
 * ------------------------------------------------------------------------- */
typedef struct psatd_fdtd_s* psatd_fdtd_t;

enum { PSATD_FDTD_YEE = 0, PSATD_FDTD_CKC = 1 };

/* Plan one periodic patch.  config: precision (field element type),
 * source_mode PSATD_VACUUM or PSATD_SOURCES_J, order 0 or 2 (second order) or
 * an even p <= 32 (Yee scheme only), c, eps0; path and flags must be 0.
 * patch: ndim 2 (n[1] = 1) or 3 (CKC: 2 only), max(2, p) <= n[a] <= 2^24, at
 * most 2^31 cells, d > 0, offset >= 0.  dt must satisfy the scheme's Courant
 * condition: c dt sqrt(sum_a (sum_l |C_l| / d_a)^2) <= 1 (Yee, order p), or
 * c dt <= dx (CKC); otherwise PSATD_ERR_INVALID_ARG.  Allocates no device
 * memory; *out is set only on success. */
psatd_status psatd_fdtd_plan(const psatd_config* config, int32_t scheme,
                             const psatd_patch_desc* patch, int32_t device, psatd_fdtd_t* out);

/* Advance E and B in place by nsteps steps on hip_stream (J read when
 * source_mode is PSATD_SOURCES_J; nsteps > 1 only in vacuum).  Two kernel
 * launches per step (the B half, then the E half), asynchronous, no
 * allocation and no synchronization.  Argument errors are returned before
 * anything is enqueued. */
psatd_status psatd_fdtd_push(psatd_fdtd_t fdtd, const psatd_fields* fields, int32_t nsteps,
                             void* hip_stream);

/* Free the plan (it owns no device memory).  NULL is accepted. */
psatd_status psatd_fdtd_destroy(psatd_fdtd_t fdtd);

#ifdef __cplusplus
}
#endif

#endif /* PSATD_H */
