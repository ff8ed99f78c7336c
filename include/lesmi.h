/*
 * lesmi: MI355X (gfx950) LES residual and time stepping for the filtered compressible
 * Navier-Stokes equations on a structured curvilinear grid, after Junqueira-Junior,
 * Yamouni, Azevedo & Wolf, "Large Eddy Simulations of Supersonic Jet Flows for
 * Aeroacoustic Applications" (arXiv 2212.12365).
 *
 * Plain C ABI: host or device pointers and sizes only.
 *
 * Data layout. A grid has ni x nj x nk distinct nodes (periodic directions are not
 * duplicated). Node (i,j,k) has offset n = i + ni*(j + nj*k). A conserved field q is five
 * contiguous component planes q[c][n], c = 0..4 for (rho, rho u, rho v, rho w, e), FP64,
 * in the paper's dimensionless units (density by rho_ref, velocity by a_ref, pressure and
 * energy by rho_ref a_ref^2, length by L_ref, time by L_ref/a_ref). Directions 0,1,2 are
 * xi (i), eta (j), zeta (k); for the jet these are axial, radial and azimuthal.
 *
 * Ownership. The caller owns every array passed in; the context owns the grid metrics,
 * the Runge-Kutta stage buffers, the boundary data and the time-step scalar. Device memory
 * is allocated or freed only by les_init_grid, les_destroy, les_stats_reset (first call),
 * les_mlp_fit_norm and the batch calls les_batch_create, les_batch_set_tuning,
 * les_batch_autotune and les_batch_destroy.
 *
 * Streams. `stream` is a hipStream_t (NULL = the null stream). Every call except
 * les_init_grid and les_destroy is asynchronous on that stream, and may be issued from
 * one host thread at a time per context. les_step synchronises once, at its end, to read
 * its status flag; les_diagnostics synchronises to return host values.
 *
 * Errors. Every call returns an les_status and never aborts; les_last_error() gives a
 * message for the context's last failure.
 */
#ifndef LESMI_H
#define LESMI_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct les_ctx les_ctx;

typedef enum {
  LES_OK = 0,
  LES_EINVAL = -1,      /* bad argument or unsupported parameter set */
  LES_ENOMEM = -2,      /* device allocation failed */
  LES_EGRID = -3,       /* J^-1 <= 0 at an updated node (left-handed or folded grid) */
  LES_EHIP = -4,        /* a HIP runtime call failed */
  LES_ENONFINITE = -5,  /* non-finite value or non-positive density/pressure produced */
  LES_ESTATE = -6       /* call not valid in the context's current state */
} les_status;

typedef enum {
  LES_BC_PERIODIC = 0,
  LES_BC_AXIS = 1,        /* jet centreline (j-) */
  LES_BC_JET_INFLOW = 2,  /* jet entrance (i-) */
  LES_BC_FARFIELD = 3,    /* Riemann-invariant far field (j+) */
  LES_BC_EXIT = 4         /* exit plane (i+) */
} les_bc;

typedef enum { LES_FP64 = 0, LES_MIXED = 1 } les_precision;
typedef enum { LES_SMAGORINSKY = 0, LES_MLP = 1 } les_closure;

/* Learned subgrid closure (closure = LES_MLP). The paper's eddy-viscosity form
 * mu_t = rho c Delta^2 |S| (Subgrid Scale Modeling) with the coefficient c predicted per
 * node by a 6-64-64-1 network from six scale-free invariants of the resolved velocity
 * gradient A (S = sym A, O = skew A, S^d its deviatoric part, |S| = (2 S:S)^(1/2)):
 *   f = (tr S/|S|, tr(S^d S^d)/|S|^2, tr(O O)/|S|^2, tr(S^d S^d S^d)/|S|^3,
 *        tr(S^d O O)/|S|^3, tr(S^d S^d O O)/|S|^4),
 *   x = (f - mean) inv_std, h1 = gelu(W1 x + b1), h2 = gelu(W2 h1 + b2),
 *   c = softplus(w3 . h2 + b3)   (gelu in its tanh form).
 * Where |S| = 0, an input is not finite or lies outside [lo, hi], c = C_s^2 (plain
 * Smagorinsky). Parameters are FP32, LES_MLP_NPARAMS values in the order
 * W1[64][6], b1[64], W2[64][64], b2[64], w3[64], b3; the products run in BF16 with FP32
 * accumulation. */
#define LES_MLP_INPUTS 6
#define LES_MLP_HIDDEN 64
#define LES_MLP_NPARAMS 4673
typedef struct {
  float mean[LES_MLP_INPUTS], inv_std[LES_MLP_INPUTS];  /* input normalisation */
  float lo[LES_MLP_INPUTS], hi[LES_MLP_INPUTS];         /* trained input range */
} les_mlp_norm;

/* Largest grid, ni * nj * nk nodes: the kernels address planes of per-node arrays with 32-bit
 * offsets (at most 11 planes of N values), so N must satisfy 11 N <= 2^31 - 1. That is
 * 195,225,786 nodes, about 58 GB of FP64 state and metrics; les_init_grid rejects larger
 * grids with LES_EINVAL before touching the device. */
#define LES_MAX_NODES 195225786LL

/* Problem parameters (paper: Dimensionless Formulation, LES formulation, Subgrid Scale
 * Modeling, Spatial Discretization, Boundary Conditions). Supported boundary sets:
 * all six faces periodic (a box), or the jet set {i-: JET_INFLOW, i+: EXIT, j-: AXIS,
 * j+: FARFIELD, k: PERIODIC}. Each direction needs at least 4 nodes, and the grid at most
 * LES_MAX_NODES nodes. */
typedef struct {
  int ni, nj, nk;
  int bc[6];                  /* faces i-, i+, j-, j+, k-, k+ (les_bc) */
  double period_shift[3][3];  /* [direction][x,y,z]: coordinate jump across a periodic wrap */
  double gamma;               /* ratio of specific heats */
  double prandtl;             /* molecular Prandtl number (0.72) */
  double prandtl_sgs;         /* SGS Prandtl number (0.6) */
  double re_acoustic;         /* rho_ref a_ref L_ref / mu_ref; 0 = no molecular viscosity */
  double suth_s1;             /* Sutherland constant / reference temperature (110.4 K / T_ref) */
  double cs;                  /* Smagorinsky constant */
  double k2, k4;              /* Turkel-Vatsa dissipation constants (0.25, 0.016) */
  double mach_jet;            /* jet exit velocity / a_ref */
  double jet_radius;          /* entrance nodes with sqrt(y^2+z^2) <= jet_radius are jet */
  double rho_inf, u_inf[3], p_inf;  /* free stream for the far field and exit */
  int precision;              /* les_precision */
  int closure;                /* les_closure */
} les_params;

/* Grid metrics (paper, Transformation of Coordinates): computes on the device
 * S_d = J^-1 grad(xi_d) in conservative form and J^-1 = det(dx/dxi) from the node
 * coordinates, and the boundary normals. `xyz` is a HOST array [3][nk][nj][ni] (x, y, z).
 * Synchronous. Returns LES_EGRID if J^-1 <= 0 at an updated node (the context is still
 * created so the caller may inspect it), LES_EINVAL for unsupported parameters or a grid of
 * more than LES_MAX_NODES nodes (checked before any device call; *out stays NULL). */
int les_init_grid(const les_params* params, const double* xyz, les_ctx** out);

/* Residual RHS_ijk of the semi-discrete system dQ/dt = -J RHS (paper, Spatial
 * Discretization: central interface flux with Turkel-Vatsa artificial dissipation minus
 * the viscous and subgrid fluxes, summed over the three directions). q and rhs are DEVICE
 * arrays [5][N]. rhs is written at every node: 0 on boundary-condition nodes. */
int les_residual(les_ctx* ctx, const double* q, double* rhs, void* stream);

/* Advances q (DEVICE [5][N], in place) by nsteps steps of the five-stage Runge-Kutta
 * scheme, alpha = (1/4, 1/6, 3/8, 1/2, 1) (paper, Time Marching Method), applying the
 * boundary conditions after every stage. If cfl > 0 each step uses
 * dt = cfl * min over updated nodes of J^-1 / sum_d (|S_d.u| + a|S_d|), computed on the
 * device from the state at the start of the step; otherwise dt = dt_fixed. dt_last (HOST,
 * may be NULL) receives the dt of the last step. q is expected to satisfy the boundary
 * conditions on entry (see les_apply_bc). Returns LES_ENONFINITE if a non-finite value or
 * non-positive density or pressure appeared; q then holds the failing state. */
int les_step(les_ctx* ctx, double* q, int nsteps, double cfl, double dt_fixed,
             double* dt_last, void* stream);

/* Dual time stepping (the paper's Concluding Remarks ask for a dual-time procedure to lift its
 * explicit time step; the low-Mach preconditioning of the pseudo-time term is not part of
 * this one). Advances q (DEVICE [5][N], in place) by nsteps physical steps of size dt of the
 * backward-difference discretisation (a0 Q^{n+1} + a1 Q^n + a2 Q^{n-1})/dt + J RHS(Q^{n+1}) = 0,
 * (a0, a1, a2) = (3/2, -2, 1/2), or (1, -1, 0) (backward Euler) for a first step without
 * history. Each step takes `subiters` pseudo-time iterations of the five-stage scheme
 * (alpha = 1/4, 1/6, 3/8, 1/2, 1) with the local pseudo-time step
 * dtau_i = cfl_tau J^-1 / sum_d (|S_d.u| + a|S_d|) of the iteration's starting state, the
 * physical-time term point-implicit:
 *   Q^(l) = [Q^(0) - alpha_l dtau (J RHS(Q^(l-1)) + (a1 Q^n + a2 Q^{n-1})/dt)]
 *           / (1 + alpha_l dtau a0 / dt),
 * and the boundary conditions after every stage. q_prev (DEVICE [5][N], may be NULL) holds
 * Q^{n-1} on entry (NULL: the first step is backward Euler) and receives Q^n of the last step
 * on return, so that calls chain. res_out (HOST [nsteps * subiters], may be NULL) receives
 * the r.m.s. over updated nodes of the unsteady mass residual at the start of every
 * iteration. The first call allocates four state-sized buffers; synchronises once, at the
 * end. q_prev must not alias q. LES_EINVAL for nsteps < 0, subiters < 1, dt or cfl_tau not
 * positive, or nsteps * subiters above 2^24; otherwise errors as les_step. */
int les_dual_step(les_ctx* ctx, double* q, double* q_prev, int nsteps, double dt,
                  int subiters, double cfl_tau, double* res_out, void* stream);

/* Smagorinsky eddy viscosity mu_sgs = rho (C_s Delta)^2 (2 S_ij S_ij)^(1/2) at every node
 * (paper, Subgrid Scale Viscosity), Delta = (J^-1)^(1/3), 0 where J^-1 <= 0. q DEVICE
 * [5][N], mu_t DEVICE [N], in units of rho_ref a_ref L_ref. */
int les_sgs_viscosity(les_ctx* ctx, const double* q, double* mu_t, void* stream);

/* Sets the boundary-condition nodes of q (DEVICE [5][N], in place) from its updated nodes
 * (paper, Boundary Conditions): far field, then centreline (azimuthal mean of the first
 * ring), then entrance, then exit. A no-op for a periodic box. */
int les_apply_bc(les_ctx* ctx, double* q, void* stream);

/* Diagnostics over updated nodes, summed in a fixed order: out[0] = volume-weighted mean
 * kinetic energy sum J^-1 rho|u|^2/2 / sum J^-1; out[1..5] = sum J^-1 Q_c. q DEVICE [5][N];
 * out HOST [6]. Synchronises the stream. */
int les_diagnostics(les_ctx* ctx, const double* q, double* out, void* stream);

/* Residual norms of the mass equation over updated nodes: out[0] = (mean of RHS_rho^2)^(1/2),
 * out[1] = max |RHS_rho| (out HOST [2]). Uses the context's stage buffer; synchronises. */
int les_residual_norms(les_ctx* ctx, const double* q, double* out, void* stream);

/* Running statistics of the primitive variables (rho, u, v, w, p) at every node, summed in
 * FP64 on the device. les_stats_reset starts (and on first use allocates) the
 * accumulators; les_stats_accumulate adds the state q (DEVICE [5][N]) as one sample;
 * les_stats_read writes the mean and the r.m.s. fluctuation (DEVICE [5][N] each, either may
 * be NULL) and the number of samples (HOST, may be NULL). The jet centreline profile is the
 * mean at j = 0. */
int les_stats_reset(les_ctx* ctx);
int les_stats_accumulate(les_ctx* ctx, const double* q, void* stream);
int les_stats_read(les_ctx* ctx, double* mean, double* rms, long long* samples, void* stream);

/* Azimuthal reduction of the running statistics, the products the paper's Numerical Results
 * need from a converged run of the round jet: out DEVICE [2][5][nj][ni]; out[0][c][j][i] is
 * the mean over the azimuthal index k (summed in increasing k, divided by nk) of the time
 * mean of component c of (rho, u, v, w, p) at (i, j, k), out[1][c][j][i] the same of the
 * r.m.s. fluctuation. The centreline decay is out[0][1][0][i] over the axial stations i; a
 * radial profile at station i is out[.][c][j][i] over j. Needs at least one sample
 * (LES_ESTATE otherwise). */
int les_stats_azimuthal(les_ctx* ctx, double* out, void* stream);

/* Copies the context's metrics to DEVICE arrays S [9][N] (S_d^c at index 3d + c) and
 * jinv [N]; either may be NULL. */
int les_get_metrics(les_ctx* ctx, double* S, double* jinv, void* stream);

/* Number of nodes updated by the time integration (those not on a non-periodic face). */
long long les_updated_nodes(const les_ctx* ctx);

/* Launch tuning of the stage kernel: `tile` indexes the table of thread-tile shapes
 * (0 .. les_tuning_count()-1, named by les_tuning_name), `kmin` is the smallest number of
 * z-planes one block marches through. Results do not depend on the choice (the same
 * arithmetic runs in the same order for every node); only the speed does. */
int les_set_tuning(les_ctx* ctx, int tile, int kmin);

/* enable != 0 (the default): les_step captures one Runge-Kutta step in a HIP graph on the
 * context's own stream, keeps it, and replays it on the caller's stream (recaptured when the
 * state pointer, the time-step mode or value, the tuning or the network changes; not used
 * while les_profile is on). 0: the kernels are launched one by one. The results are the
 * same either way. */
int les_set_graph(les_ctx* ctx, int enable);
int les_tuning_count(void);
const char* les_tuning_name(int tile);

/* Instrumentation: with enable != 0, les_step records HIP events on its stream around the
 * two kernels of every Runge-Kutta stage: the node-record kernel (eddy viscosity, spectral
 * radii, sensors; with the learned closure also its inputs and evaluation) and the face
 * kernel (fluxes, flux differences and the stage update); boundary conditions and the
 * time-step reduction are excluded.
 * les_profile_read waits for the last recorded event and returns, since the last read (or
 * since les_profile), the summed node-kernel and face-kernel times in milliseconds and the
 * number of timed stages, then resets the record. Either time pointer may be NULL. */
int les_profile(les_ctx* ctx, int enable);
int les_profile_read(les_ctx* ctx, double* nodes_ms, double* faces_ms, long long* stages);

/* Autotuner of a single context: times every stage-kernel tile shape with z-chunk depths
 * 4, 8 and 16 on Runge-Kutta stage updates of q (DEVICE [5][N], read, not modified) with
 * dt = 0 into the context's stage buffer, and keeps the fastest (les_set_tuning). tile and
 * kmin (HOST, may be NULL) receive the choice. Synchronises the stream. */
int les_autotune(les_ctx* ctx, const double* q, int* tile, int* kmin, void* stream);

void les_destroy(les_ctx* ctx);

/* ---------------------------------------------------------------------------------------
 * Learned closure entry points (layout and fallback rule above).
 * ------------------------------------------------------------------------------------- */

/* Installs the network of an LES_MLP context: theta DEVICE [LES_MLP_NPARAMS] (copied),
 * norm HOST. Until it is called, stepping or evaluating an LES_MLP context returns
 * LES_ESTATE. Synchronous. */
int les_mlp_set_network(les_ctx* ctx, const float* theta, const les_mlp_norm* norm);

/* Number of node evaluations that fell back to C_s^2 since the last call (resets it).
 * Synchronous. */
int les_mlp_fallback_count(les_ctx* ctx, unsigned long long* count);

/* Network inputs of a state: feat DEVICE [6][N] (FP32), smag DEVICE [N] = |S| (FP32). */
int les_mlp_features(les_ctx* ctx, const double* q, float* feat, float* smag, void* stream);

/* Coefficient c (DEVICE [n]) of n samples with inputs feat DEVICE [6][n] and |S| smag
 * DEVICE [n], by the network theta DEVICE with normalisation norm HOST; fallback DEVICE
 * (may be NULL) is incremented by the number of samples that took c = cs2. */
int les_mlp_coefficient(const float* theta, const les_mlp_norm* norm, float cs2,
                        const float* feat, const float* smag, long long n, float* c,
                        unsigned* fallback, void* stream);

/* Training: the loss sum_s w (c_s - y_s)^2 * inv_wsum over the samples idx[0..n-1]
 * (DEVICE int32 node numbers into feat [6][nfeat], target [nfeat], weight [nfeat]) and its
 * gradient grad DEVICE [LES_MLP_NPARAMS]; loss DEVICE [1] may be NULL. work DEVICE holds
 * les_mlp_work_size(n) floats (per-wave partial gradients, summed in a fixed order). */
long long les_mlp_work_size(long long n);
int les_mlp_loss_grad(const float* theta, const les_mlp_norm* norm, const float* feat,
                      long long nfeat, const float* target, const float* weight, const int* idx,
                      long long n, float inv_wsum, float* grad, float* loss, float* work,
                      void* stream);

/* Allocation-free form of les_mlp_loss_grad, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight training loops, harnesses that forbid hipMalloc):
 * the same loss and gradient, bit for bit, with the per-wave partial gradients kept in a
 * static device array of the library instead of a `work` argument. That array holds
 * (LES_MLP_NOALLOC_MAX_SAMPLES / 128) * 4 * (LES_MLP_NPARAMS + 1) floats (4.8 MB) on every
 * GPU the library runs on, until the process ends. n <= LES_MLP_NOALLOC_MAX_SAMPLES, else
 * LES_EINVAL (nothing is launched). The call allocates and frees nothing and does not
 * synchronise. Every call on one GPU shares that GPU's array: calls ordered on one stream
 * are safe, calls that overlap in time on one GPU (other streams, other host threads) race
 * and give wrong gradients. */
#define LES_MLP_NOALLOC_MAX_SAMPLES 8192
int les_mlp_loss_grad_noalloc(const float* theta, const les_mlp_norm* norm, const float* feat,
                              long long nfeat, const float* target, const float* weight,
                              const int* idx, long long n, float inv_wsum, float* grad,
                              float* loss, void* stream);

/* One Adam step (Kingma & Ba) on theta with moments m, v (all DEVICE
 * [LES_MLP_NPARAMS]); step counts from 1. */
int les_mlp_adam(float* theta, const float* grad, float* m, float* v, int step, float lr,
                 float beta1, float beta2, float eps, void* stream);

/* Normalisation from the inputs of samples with weight > 0: mean and 1/standard deviation
 * of each input, and the range [min - widen*span, max + widen*span]. feat DEVICE [6][n],
 * weight DEVICE [n], out HOST. Allocates a small device buffer; synchronous. */
int les_mlp_fit_norm(const float* feat, const float* weight, long long n, float widen,
                     les_mlp_norm* out, void* stream);

/* Training data: box-filters the fine state q_fine (DEVICE [5][Nf], fine context with
 * exactly twice the coarse nodes per direction) over 2 x 2 x 2 node blocks onto the coarse
 * grid: q_coarse DEVICE [5][Nc] (block means of the conserved variables) and the subgrid
 * stress sigma DEVICE [6][Nc] = mean(rho u_m u_n) - rho~ u~_m u~_n (components 00, 11, 22,
 * 01, 02, 12). On the coarse grid it writes the network inputs feat [6][Nc] and |S~|
 * smag [Nc] of u~, the least-squares coefficient
 * target = max(0, -sigma^d : S~^d / (2 rho~ Delta^2 |S~| S~^d : S~^d)), and weight = 1 at
 * updated nodes with |S~| >= smin, else 0 (all FP32 DEVICE [Nc]). */
int les_filter_target(les_ctx* fine, les_ctx* coarse, const double* q_fine, float smin,
                      double* q_coarse, double* sigma, float* feat, float* smag, float* target,
                      float* weight, void* stream);

/* ---------------------------------------------------------------------------------------
 * Batched ensembles: n independent contexts (for instance seeded jet realisations on grids
 * of different sizes) advanced together. Each kernel of a Runge-Kutta step runs as one
 * persistent launch over a work list spanning every member, and a whole step is captured
 * once in a HIP graph and replayed. Every member keeps its own time step (its own CFL
 * reduction). The arithmetic per node and face is that of les_step, so each member's result
 * equals its single-context run.
 *
 * The batch borrows its members' device buffers (metrics, stage buffers, node records,
 * time-step scalars): while a batch exists its members must not be stepped on their own,
 * and they must outlive it. All members share one precision and device.
 * ------------------------------------------------------------------------------------- */
typedef struct les_batch les_batch;

/* members: HOST array of n context handles (Smagorinsky closure). On failure *out may
 * still be set so that les_batch_last_error can be read; les_batch_destroy it. */
int les_batch_create(les_ctx* const* members, int n, les_batch** out);

/* Advances every member by nsteps steps (as les_step: cfl > 0 gives each member
 * dt = cfl * its own reduction, else dt_fixed for all). q: HOST array of n DEVICE state
 * pointers [5][N_m], each satisfying its boundary conditions on entry. dt_last: HOST [n] or
 * NULL. Synchronises once, at the end. Returns LES_ENONFINITE naming the failing members. */
int les_batch_step(les_batch* b, double* const* q, int nsteps, double cfl, double dt_fixed,
                   double* dt_last, void* stream);

/* Stage-kernel launch shape of the batch (the tile table of les_tuning_name; kmin >= 1). */
int les_batch_set_tuning(les_batch* b, int tile, int kmin);
int les_batch_get_tuning(const les_batch* b, int* tile, int* kmin);

/* Autotuner of the batch: times every tile shape with z-chunk depths 4, 8 and 16 on the
 * first two Runge-Kutta stages of all members with dt = 0 (the states q are read, not
 * modified; the members' stage buffers are overwritten) and keeps the fastest.
 * Synchronises the stream. */
int les_batch_autotune(les_batch* b, double* const* q, int* tile, int* kmin, void* stream);

/* enable != 0 (the default): steps replay a captured graph; 0: launches are issued one by
 * one (the same kernels). */
int les_batch_set_graph(les_batch* b, int enable);

void les_batch_destroy(les_batch* b);
const char* les_batch_last_error(const les_batch* b);
const char* les_last_error(const les_ctx* ctx);

/* ---------------------------------------------------------------------------------------
 * Far-field noise by the Ffowcs Williams-Hawkings analogy (the paper's Introduction and
 * Concluding Remarks name it as the route from the jet LES to far-field acoustics; it states
 * no formulation). Formulation 1A of Farassat for a stationary permeable control surface in a
 * medium at rest, viscous stresses left out of the loading: with Q_n = rho u.n and
 * L_i = (p - p0) n_i + rho u_i (u.n) at a surface node y of unit outward normal n and area dS,
 *   4 pi p'(x, t) = sum_nodes dS [ dQ_n/dtau / r + dL_r/dtau / (c0 r) + L_r / r^2 ]
 * evaluated at the retarded time tau = t - r/c0, r = |x - y|, L_r = L . (x - y)/r. Time
 * derivatives are central differences of the samples (second-order one-sided at the first and
 * last), values at tau linear interpolations between the two samples around it.
 * ------------------------------------------------------------------------------------- */
typedef struct les_fwh les_fwh;

/* Control surface on a jet context: the lateral cylinder j = js over i1 <= i <= i2 (every k),
 * plus the end caps i = i1 (caps bit 0) and i = i2 (caps bit 1) over 0 <= j <= js. Node areas
 * and normals come from the metric vectors (S_eta on the cylinder, -S_xi and +S_xi on the
 * caps), with half weights on the edges of each patch. xyz: HOST [3][N] coordinates (those
 * given to les_init_grid). capacity >= 3: samples the history holds (5 doubles per node and
 * sample, plus 7 for the sources). dtau > 0: the sampling interval, which the caller keeps
 * uniform (for instance a sample every m steps of fixed dt). Allocates; synchronous.
 * LES_EINVAL for a periodic box or indices outside the grid (*out is then NULL). If a later
 * step fails (LES_ENOMEM, LES_EHIP), *out holds the object so that les_fwh_last_error can
 * say why; destroy it. ctx must outlive the surface. */
int les_fwh_create(les_ctx* ctx, const double* xyz, int i1, int i2, int js, int caps,
                   int capacity, double dtau, les_fwh** out);
/* Number of surface nodes, and of samples taken. */
int les_fwh_nodes(const les_fwh* f);
int les_fwh_samples(const les_fwh* f);
/* Surface geometry: geo DEVICE [7][ns] = positions (3), unit normals (3), areas. */
int les_fwh_geometry(les_fwh* f, double* geo, void* stream);
/* Appends one sample of q (DEVICE [5][N]): rho, u, v, w, p of every surface node.
 * LES_ESTATE when the history is full. */
int les_fwh_sample(les_fwh* f, const double* q, void* stream);
/* Forgets the samples. */
int les_fwh_reset(les_fwh* f);
/* Acoustic pressure at no observers (HOST [no][3]) and nt times (HOST [nt]): p_out DEVICE
 * [no][nt]; scale_out DEVICE [no][nt] or NULL receives the sum of the absolute values of the
 * terms; skipped HOST or NULL the number of (observer, time, node) triples whose retarded
 * time fell outside [tau0, tau0 + (samples - 1) dtau] and were left out. Sample m is taken
 * to be at tau0 + m dtau. Needs 3 samples or more (LES_ESTATE); LES_EINVAL for no or nt
 * below 1, c0 not positive, or no * nt above about 2^28. Synchronises the stream; may
 * allocate a small observer buffer. */
int les_fwh_pressure(les_fwh* f, const double* observers, int no, const double* times, int nt,
                     double c0, double p0, double tau0, double* p_out, double* scale_out,
                     long long* skipped, void* stream);
void les_fwh_destroy(les_fwh* f);
const char* les_fwh_last_error(const les_fwh* f);

#ifdef __cplusplus
}
#endif
#endif
