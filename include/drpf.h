/*
 * drpf -- dual-resolution phase-field step for AMD MI355X (gfx950).
 *
 * One coupled time step of the dual-resolution phase-field solver of Bazesefidpar, Brandt
 * and Tammisola: Cahn-Hilliard (Dong's stabilised splitting into two constant-coefficient
 * Helmholtz equations, eqs. NS25-NS34 of the paper) on a phase-field grid twice as fine as
 * the flow grid, Navier-Stokes with variable density and viscosity by the
 * constant-coefficient projection (eqs. NS35-NS39), and an Oldroyd-B polymer stress
 * (eq. NS4 with alpha = 0, advanced by the second-order TVD Runge-Kutta of eqs. NS40-NS44
 * in stress form). The grids exchange data through the divergence-preserving prolongation
 * (eq. dual1) and averaging restriction (eqs. dual2, dual3) of Sec. 3.1.
 *
 * Conventions
 *   - Array layout [z][y][x], x contiguous. x and y periodic, z wall-normal with walls at
 *     z = 0 and z = lz.
 *   - Coarse grid nx * ny * nz cells (spacings lx/nx, ly/ny, lz/nz). The phase-field grid
 *     has 2nx * ry*ny * 2nz cells with ry = 2, or ry = 1 when ny == 1 (the 2D form).
 *   - Staggering: p and tau at cell centres; u[k][j][i] at x = (i+1) hx, v[k][j][i] at
 *     y = (j+1) hy, w[k][j][i] at z = (k+1) hz (w[nz-1][.][.] is the top wall and stays 0;
 *     the bottom-wall w is implicit and 0). phi at fine cell centres.
 *   - Nondimensional groups follow the paper's problem statement (Sec. 4): Re, Ca, Cn, Pe,
 *     Wi, beta, static contact angles (eq. NS16, measured through the drop, phase
 *     phi = +1), rho_ratio = drop/ambient density, mu_ratio = drop/ambient viscosity.
 *   - Scalars are double on the host. Device arrays hold double when precision == 64 and
 *     float when precision == 32.
 *
 * Memory ownership: the caller allocates every device buffer (state arrays, the workspace)
 * and keeps it valid until the work queued on the stream has completed. The library never
 * allocates or frees device memory. A drpf_grid is a host object owned by the library,
 * released by drpf_destroy.
 *
 * Streams: every call that takes a stream queues its work asynchronously on it (a
 * hipStream_t passed as void*; NULL is the default stream), except drpf_observables, which
 * synchronises that stream before returning. Calls on one grid must not overlap. On a
 * viscoelastic grid drpf_step runs each step's polymer update on a stream the library creates
 * (default priority, created by drpf_init_grid, released by drpf_destroy), forked from the
 * caller's stream by an event after the velocity correction and joined back by an event before
 * the next step's momentum right-hand side and before drpf_step returns: the caller's stream
 * orders all of the call's work as if it had run on it alone.
 *
 * Errors: every call returns one of the DRPF_* codes below; drpf_last_error() gives a
 * thread-local message for the last failure on the calling thread.
 */
#ifndef DRPF_H
#define DRPF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DRPF_OK 0
#define DRPF_EINVAL 1        /* invalid argument or parameter set                      */
#define DRPF_EWORKSPACE 2    /* workspace missing, too small or misaligned             */
#define DRPF_EHIP 3          /* a HIP runtime call or kernel launch failed             */
#define DRPF_ENONFINITE 4    /* a non-finite value was found (drpf_observables, or
                                drpf_step with check_finite_every > 0)                  */
#define DRPF_EUNSUPPORTED 5  /* valid but not supported by this library                */

/* Locations for drpf_restrict (eq. dual2 generalised to 3D as a tensor product of the
 * 1D rules: along a centre-located axis coarse index i averages fine 2i and 2i+1; along a
 * face-located axis it averages the two fine cells either side of the face at (i+1)h).
 * Outputs for FACE_Z, EDGE_XZ and EDGE_YZ have nz+1 z layers, the bottom wall first; a
 * fine neighbour beyond a wall is replaced by the wall-adjacent fine cell. */
enum drpf_location {
  DRPF_CENTER = 0,
  DRPF_FACE_X = 1,
  DRPF_FACE_Y = 2,
  DRPF_FACE_Z = 3,
  DRPF_EDGE_XY = 4,
  DRPF_EDGE_XZ = 5,
  DRPF_EDGE_YZ = 6
};

/* Grids and boundary kinds for drpf_helmholtz_solve. */
enum drpf_which_grid { DRPF_GRID_FINE = 0, DRPF_GRID_COARSE = 1 };
enum drpf_bc {
  DRPF_BC_NEUMANN = 0,          /* cell-centred in z, zero normal gradient at the walls */
  DRPF_BC_DIRICHLET = 1,        /* cell-centred in z, zero value (ghost = -adjacent)    */
  DRPF_BC_FACE_DIRICHLET = 2    /* z-face located, unknowns k = 0..nz-2, walls 0        */
};

typedef struct drpf_params {
  int nx, ny, nz;              /* coarse cells; powers of two; 4 <= nx <= 1024, 4 <= nz <= 512;
                                  ny == 1 (2D form) or 4 <= ny <= 1024                       */
  double lx, ly, lz;           /* box lengths (> 0)                                         */
  double re, ca, cn, pe;       /* Reynolds, capillary, Cahn, Peclet numbers (> 0)           */
  double wi, beta;             /* Weissenberg number and solvent-viscosity ratio of drop    */
  double theta_bottom_deg;     /* static contact angle at z = 0, degrees in [0, 180]        */
  double theta_top_deg;        /* static contact angle at z = lz                            */
  double rho_ratio, mu_ratio;  /* drop / ambient density and total viscosity (> 0)          */
  double dt;                   /* time step (> 0)                                           */
  double s_factor;             /* stabilisation S as a multiple of the bound of eq. NS30, >= 1 */
  double a_ext[3];             /* body acceleration (x, y, z)                               */
  int viscoelastic;            /* 1: drop phase carries a polymer stress (Oldroyd-B, or
                                  Giesekus when giesekus_alpha > 0)                         */
  int precision;               /* 64 or 32: element type of every device array              */
  int constitutive;            /* form of the polymer update: 0 stress form (eq. NS4 with the
                                  RK2-TVD of eqs. NS42-NS44 on tau), 1 log-conformation
                                  (eqs. NS22, NS40-NS46 on Theta = log c); 1 needs
                                  viscoelastic                                               */
  double giesekus_alpha;       /* Giesekus mobility alpha in [0, 0.5] (eqs. NS4, NS18); 0 is
                                  Oldroyd-B; > 0 needs viscoelastic and beta < 1            */
  int refine;                  /* phase-field grid: 2 (or 0) the dual resolution of Sec. 3.1,
                                  twice the flow grid in x, z (and y in 3D); 1 a single
                                  resolution (the phase field on the flow grid, faces and
                                  edges by two- and four-cell means). The transfer and
                                  adjoint entry points need 2.                               */
  int advection;               /* advection of the phase field (eq. NS25) and of the polymer
                                  (eq. NS41): 0 second-order central flux form; 1 fifth-order
                                  WENO-Z face values (Sec. 3.2.1, 3.2.3). The adjoint covers
                                  both                                                       */
  double d_w;                  /* wall relaxation D_w >= 0 of eq. NS15, discretised as eq.
                                  NS34 at both walls: the wall derivative of phi^{n+1} gains
                                  D_w (gamma0 phi^{n+1} - phi_hat) / dt at the wall-adjacent
                                  cell (a Robin condition; NS25 is solved with it and with
                                  NS33 exactly). 0 (default): static contact angles. The
                                  adjoint covers both (with d_w > 0 it solves with the
                                  transposed relaxed operator)                               */
  double u_wall_bottom[2];     /* tangential wall velocity (x, y) at z = 0 and ...            */
  double u_wall_top[2];        /* ... at z = lz: the no-slip condition u = u_w of eq. NS13
                                  (ghost = 2 u_w - adjacent in every stencil and in the
                                  implicit velocity solves). Finite; 0 (default): walls at
                                  rest. With d_w > 0, eq. NS34 also carries the wall
                                  advection D_w u_w . grad phi* (central differences on the
                                  wall-adjacent layer). The adjoint covers moving walls with
                                  d_w == 0 (DRPF_EUNSUPPORTED for moving relaxed walls)      */
  int check_finite_every;      /* > 0: drpf_step checks the phase field and the velocities for
                                  NaN/Inf after every check_finite_every-th step (counted by the
                                  state's step counter), synchronising the stream there, and
                                  stops with DRPF_ENONFINITE at the first failed check. 0
                                  (default): no checks, fully asynchronous                   */
} drpf_params;

/* Device pointers of one solution state. Level n is index 0, level n-1 index 1.
 * phi[2] is a third fine buffer the step writes the new phase field into.
 * drpf_step rotates the pointers in this host struct after every step (no copies):
 * afterwards phi[0] is level n+1, phi[1] level n, phi[2] the free buffer, and for the
 * coarse fields [0] points to level n+1 (stored in the former n-1 buffer) and [1] to level
 * n. tau[level][c], c = xx, yy, zz, xy, xz, yz, is read and written only when
 * viscoelastic != 0. step counts completed steps; step == 0 takes the one-level start
 * (gamma0 = 1, extrapolations replaced by level n). theta[c] (same component order, coarse
 * centres) is the log-conformation Theta = log c at level n, read and overwritten in place with
 * level n+1 only when constitutive == 1 (it must then be non-null; zero means c = I); the step
 * then writes tau of level n+1 from it (eq. NS46), and the momentum equation uses tau as in
 * the stress form. */
typedef struct drpf_state {
  void* phi[3];
  void* u[2];
  void* v[2];
  void* w[2];
  void* p[2];
  void* tau[2][6];
  long long step;
  void* theta[6];
} drpf_state;

typedef struct drpf_grid drpf_grid;

/* Fields of a state, for drpf_state_layout. */
enum drpf_field {
  DRPF_FIELD_PHI = 0,   /* phase field at fine cell centres                                */
  DRPF_FIELD_U = 1,     /* x velocity at x faces                                           */
  DRPF_FIELD_V = 2,     /* y velocity at y faces                                           */
  DRPF_FIELD_W = 3,     /* z velocity at z faces (layer nz-1 is the top wall)              */
  DRPF_FIELD_P = 4,     /* pressure at coarse centres                                      */
  DRPF_FIELD_TAU = 5,   /* polymer stress at coarse centres, 6 components                  */
  DRPF_FIELD_THETA = 6, /* log-conformation at coarse centres, 6 components                */
  DRPF_NFIELDS = 7
};

/* Shape, strides and placement of one field's device arrays. Element (i, j, k) of an array
 * sits at offset i*stride[0] + j*stride[1] + k*stride[2] (elements) and at the point
 * (origin[0] + i*spacing[0], origin[1] + j*spacing[1], origin[2] + k*spacing[2]). */
typedef struct drpf_field_layout {
  int n[3];             /* extents in x, y, z                                              */
  size_t stride[3];     /* element strides in x, y, z: 1, n[0], n[0]*n[1]                  */
  size_t elems;         /* elements of one array: n[0]*n[1]*n[2]                           */
  int arrays;           /* device arrays of this field in a drpf_state: 3 for PHI (levels
                           n, n-1 and the spare buffer), 2 for U..P, 12 for TAU (2 levels x
                           6 components) when viscoelastic, 6 for THETA when constitutive
                           == 1, else 0                                                    */
  double origin[3];     /* coordinates of element (0, 0, 0)                                */
  double spacing[3];    /* grid spacings                                                   */
} drpf_field_layout;

typedef struct drpf_layout {
  int elem_bytes;                           /* 8 (precision 64) or 4 (precision 32)          */
  drpf_field_layout field[DRPF_NFIELDS];
  size_t state_bytes;                       /* sum over fields of arrays * elems * elem_bytes */
} drpf_layout;

/* Observables returned by drpf_observables, in this order. */
enum drpf_observable {
  DRPF_OBS_MASS = 0,            /* h_f^3 * sum(phi), FP64 tree sum                        */
  DRPF_OBS_WETTED_RADIUS = 1,   /* 2D: half the wetted length; 3D: sqrt(wetted area / pi),
                                   from (1+phi)/2 on the wall-adjacent fine layer           */
  DRPF_OBS_CENTROID_HEIGHT = 2, /* sum(z (1+phi)/2) / sum((1+phi)/2)                        */
  DRPF_OBS_KINETIC_ENERGY = 3,  /* 0.5 h^3 sum(u^2 + v^2 + w^2) over the face arrays        */
  DRPF_OBS_MAX_DIV = 4,         /* max |div u| over coarse cells                            */
  DRPF_OBS_COUNT = 5
};

/* Fills every field with the defaults: C1-like 2D box, Newtonian, s_factor 1, FP64. */
int drpf_params_default(drpf_params* p);

/* Checks a parameter set (the rules in the struct comments). DRPF_EINVAL on failure. */
int drpf_validate(const drpf_params* p);

/* Element counts of the fine (phase-field) and coarse arrays. */
int drpf_field_elems(const drpf_params* p, size_t* fine, size_t* coarse);

/* Bytes of device workspace that drpf_init_grid needs (spectral buffers, tables, the
 * restricted coarse set, stage buffers). */
int drpf_workspace_bytes(const drpf_params* p, size_t* bytes);

/* Validates p, carves the caller's workspace (device memory, 256-byte aligned, at least
 * drpf_workspace_bytes) and uploads the transform and eigenvalue tables on `stream`.
 * *out receives a host handle. DRPF_EINVAL / DRPF_EWORKSPACE / DRPF_EHIP on failure. */
int drpf_init_grid(const drpf_params* p, void* d_workspace, size_t bytes, void* stream,
                   drpf_grid** out);

/* Releases the host handle (the workspace stays the caller's). */
int drpf_destroy(drpf_grid* g);

/* Fills *out with the element counts, strides, placement on the staggered grids (Sec. 3.1:
 * pressure and stress at cell centres, each velocity component at the faces normal to it,
 * the phase field at the centres of the refined grid) and array counts of every field of a
 * drpf_state for this grid. Host only. DRPF_EINVAL for null arguments. */
int drpf_state_layout(const drpf_grid* g, drpf_layout* out);

/* Advances `s` by `nsteps` coupled steps (Sec. 3.2: CH, restriction, NS projection,
 * polymer), rotating the state pointers after each step as described above. With
 * check_finite_every > 0 the state is checked after every step whose new step counter is a
 * multiple of it; a failed check returns DRPF_ENONFINITE with s holding the state after that
 * step (its counter says which) and the remaining steps not taken. */
int drpf_step(drpf_grid* g, drpf_state* s, int nsteps, void* stream);

/* Coarse face velocities (u, v, w) -> fine face velocities (uf, vf, wf) by eq. dual1
 * (Rudman's divergence-preserving interpolation). Fine arrays have the fine grid's
 * element count; wf's layer 2nz-1 is the top wall (0). */
int drpf_prolong(drpf_grid* g, const void* u, const void* v, const void* w, void* uf,
                 void* vf, void* wf, void* stream);

/* Fine cell-centred field -> coarse location (eq. dual2). `location` is a drpf_location;
 * `coarse` must hold nx*ny*nz elements, or nx*ny*(nz+1) for FACE_Z, EDGE_XZ, EDGE_YZ. */
int drpf_restrict(drpf_grid* g, const void* fine, void* coarse, int location, void* stream);

/* Solves coeff * L x - shift * x = rhs on the fine or coarse grid with the 7-point
 * second-order Laplacian L (periodic x, y; boundary kind `bc` in z) by FFT in x and y and
 * a batched tridiagonal solve per Fourier mode across the walls (the "FFT solver" of
 * Sec. 3.2.1-3.2.2). coeff > 0, shift >= 0; shift == 0 is allowed only with
 * DRPF_BC_NEUMANN and returns the pseudo-inverse's solution: the z-mean of the right-hand
 * side's (0,0) Fourier mode is dropped and the result has zero mean.
 * wall_data: null for homogeneous walls, else a device array of 2 * nx * ny elements of the
 * grid's x-y layer, the bottom wall's layer then the top wall's, giving
 *   DRPF_BC_NEUMANN: the outward normal derivative g (ghost = adjacent + hz g; the wetting
 *     data of eq. NS34 has this form),
 *   DRPF_BC_DIRICHLET: the wall value (ghost = 2 value - adjacent; u = u_w of eq. NS13),
 *   DRPF_BC_FACE_DIRICHLET: the value of the face field on the wall itself.
 * The known wall terms move to the right-hand side (the workspace's spectral buffers and
 * right-hand-side buffer are overwritten). For DRPF_BC_FACE_DIRICHLET layer nz-1 of rhs is
 * ignored and that layer of x is set to the top wall's value (0 without wall data). rhs and
 * x may alias; wall_data must not overlap x. */
int drpf_helmholtz_solve(drpf_grid* g, int which_grid, int bc, double coeff, double shift,
                         const void* rhs, const void* wall_data, void* x, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): drpf_helmholtz_solve with the same arguments,
 * kernels and results, whose scratch (the spectral buffer, and with wall_data the right-hand
 * side with the wall terms) is a static 32 MiB device array of the library instead of the
 * grid's workspace, so that the grid's workspace is left untouched. It calls no hipMalloc,
 * hipFree or allocating routine. DRPF_EWORKSPACE if the solve needs more than 32 MiB of
 * scratch: ((nx/2 + 1) * ny * nz complex elements of the chosen grid, plus nx * ny * nz
 * elements with wall data, the first rounded up to 256 bytes). Every call on one GPU uses that
 * GPU's one array: calls that overlap on a GPU (on different streams, or from several threads)
 * race and must be serialised by the caller. */
int drpf_helmholtz_solve_static(drpf_grid* g, int which_grid, int bc, double coeff, double shift,
                                const void* rhs, const void* wall_data, void* x, void* stream);

/* Computes the first min(n, DRPF_OBS_COUNT) observables of level n of `s` in FP64 into
 * the host array out. Synchronises `stream`. DRPF_ENONFINITE if the phase field holds a
 * NaN or Inf (the values are still written). */
int drpf_observables(drpf_grid* g, const drpf_state* s, double* out, int n, void* stream);

/* Device pointer and element count of an internal coarse array left by the last step,
 * for inspection in tests: 0 phi_c, 1 G_c, 2..4 G at x/y/z faces, 5..7 1/rho at x/y/z
 * faces, 8 mu_c, 9 mu at xy edges, 10..11 mu at xz/yz edges (nz+1 layers),
 * 12..14 momentum right-hand sides r_u, r_v, r_w. */
int drpf_debug_field(drpf_grid* g, int id, void** ptr, size_t* count);

/* Per-kernel timing with HIP events on the caller's stream. After drpf_profile_begin, every
 * kernel launch of drpf_step is followed by an event (up to max_launches of them);
 * drpf_profile_end waits for the last one and writes, per kernel id in [0, n), the summed
 * milliseconds between the event before and after each of its launches and the launch
 * count. Kernel ids: 0 ch_rhs, 1-2 fine x/y forward transforms, 3 fine wall-normal pass,
 * 4-5 fine y/x inverse transforms, 6 restriction and chemical potential, 7 momentum
 * right-hand side, 8-9 coarse x/y forward transforms, 10 coarse wall-normal pass (NS
 * projection), 11-12 coarse y/x inverse transforms, 13-14 polymer stages, 15 WENO-Z
 * advection of the phase field (advection 1 only; it precedes ch_rhs), 16-17 the coarse x and
 * y transforms in one kernel, forward and inverse (in place of 8-9 and 11-12 where a coarse
 * layer fits in one block's LDS: 128 x 128 in either precision), 18 both polymer stages in one
 * pass (in place of 13-14 for 3D grids with central advection and the stress form). */
#define DRPF_NKERNELS 19
int drpf_profile_begin(drpf_grid* g, int max_launches, void* stream);
int drpf_profile_end(drpf_grid* g, double* total_ms, int* launches, int n);
/* Short name of kernel id (see above); "" for an unknown id. */
const char* drpf_kernel_name(int id);

/* ---- discrete adjoint (FP64 grids only) --------------------------------------------
 * The transpose of the Jacobian of one drpf_step, for gradients of a functional of the
 * final state by reverse accumulation. Not in the paper: it differentiates the discrete
 * step of Sec. 3.2 (every stencil, transfer (eqs. dual1-dual3) and spectral solve
 * transposed; the fused Dong solve of eqs. NS25-NS27, the velocity Helmholtz solves and the
 * pseudo-inverse Poisson solve of eqs. NS36-NS37 are symmetric and reused as they are; with
 * relaxed walls, eq. NS34, the fused solve is not, and its transpose is solved instead). It
 * covers central and WENO-Z advection, static, relaxed and moving walls (not relaxed walls
 * that move), and the stress form of the polymer update (Oldroyd-B or Giesekus), not the
 * log-conformation form.
 *
 * Adjoint state: the same levels as drpf_state without the spare fine buffer. phi[l] fine,
 * the others coarse; tau only when viscoelastic != 0 (may be null otherwise). */
typedef struct drpf_adj {
  void* phi[2];
  void* u[2];
  void* v[2];
  void* w[2];
  void* p[2];
  void* tau[2][6];
} drpf_adj;

/* Bytes of the second device workspace the adjoint needs (forward intermediates of the
 * recomputed step and the adjoint stage buffers). DRPF_EUNSUPPORTED unless precision 64, the
 * polymer update is the stress form (constitutive 0: Oldroyd-B, or Giesekus with
 * giesekus_alpha > 0) and relaxed walls (d_w > 0) are at rest. */
int drpf_adjoint_workspace_bytes(const drpf_params* p, size_t* bytes);

/* Hands the grid that workspace (device memory, 256-byte aligned, at least the size above;
 * it stays the caller's and must outlive the grid's adjoint calls). */
int drpf_adjoint_attach(drpf_grid* g, void* d_workspace, size_t bytes);

/* One reverse step. x_n is the state before the step (its step counter selects the
 * first-step scheme); it is read only. x_next, if not null, is the state after the step
 * (drpf_step's result from x_n: level n+1 in [0], level n in [1], step counter x_n's + 1),
 * read only; then only the restricted coarse set and the first polymer stage are
 * recomputed, otherwise the whole forward step is. On entry *lam holds the adjoint of the
 * state after the step (lam->X[0]: level n+1, lam->X[1]: level n); on exit, with the
 * pointers of *lam swapped in place (no copies), the adjoint of x_n (lam->X[0]: level n,
 * lam->X[1]: level n-1). For the functional J = <lam_in, step(x_n)> this is dJ/dx_n;
 * d_grad3 (device, three doubles) is incremented by (dJ/dtheta_bottom per radian, dJ/dPe,
 * dJ/dWi). The top-wall layer of both w levels of the adjoint is set to 0 (w is identically
 * 0 there). The restricted set and stage buffers of the grid's workspace are overwritten.
 * Queued on `stream`; no synchronisation. DRPF_EUNSUPPORTED for FP32 grids; DRPF_EINVAL
 * without an attached workspace, with null pointers, or with an x_next whose step counter
 * is not x_n's + 1. */
int drpf_adjoint_step(drpf_grid* g, const drpf_state* x_n, const drpf_state* x_next, drpf_adj* lam,
                      double* d_grad3, void* stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* drpf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DRPF_H */
