/*
 * mifoam: free-surface lattice Boltzmann foaming sweep on AMD Instinct MI355X (gfx950).
 *
 * C ABI of the shared library libmifoam.so. Every function returns an int status
 * (MF_OK = 0, negative on error); no C++ exception crosses this boundary. After an
 * error, mf_last_error() returns a message. Pointers are plain host pointers unless a
 * parameter says "device". Sizes are in bytes unless stated otherwise.
 *
 * The method is that of Ataei et al., "LBfoam: an open-source software package for the
 * simulation of foaming using the lattice Boltzmann method" (arXiv 1908.04262):
 *   - lattice Boltzmann flow on D2Q9 / D3Q19 with BGK collision (Sec. 2, Eqs. LBE,
 *     collisionstep, streamingstep, collision, equilibrium), Newtonian or power-law
 *     relaxation (Eqs. tau, carreauTau);
 *   - volume-of-fluid interface capturing by mass tracking (Sec. 2.1, Eqs. alpha,
 *     massexchange and the weights Theta) with cell conversion and excess-mass
 *     redistribution;
 *   - free-surface reconstruction at the bubble pressure with surface tension and
 *     disjoining pressure (Sec. 2.2, Eqs. reconstruct, rhob, idealgas; Sec. 3.3, Eq.
 *     rhobplusdisjoining, Appendix A Algorithm 1);
 *   - dissolved gas on D2Q5 / D3Q7 with a Henry's-law interface condition and per-bubble
 *     gas flux (Sec. 3.1-3.2, Eqs. diffusion, diffusionconst, gascurrent, henryslaw,
 *     reconstructdiffusion);
 *   - bubble tracking by flood fill with merge / split bookkeeping (Sec. 3.5).
 *
 * Lattice units throughout. Cell index n = x + nx*(y + ny*z); grids include the wall
 * layer of every closed axis. Device work is enqueued on the stream given to
 * mf_create; functions that return host data synchronise that stream.
 */
#ifndef MIFOAM_H
#define MIFOAM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MF_ABI_VERSION 4

enum mf_status {
  MF_OK = 0,
  MF_EINVAL = -1,       /* bad argument or parameter */
  MF_ENOMEM = -2,       /* workspace too small or allocation failed */
  MF_EHIP = -3,         /* a HIP runtime call failed */
  MF_ECAPACITY = -4,    /* bubble table or labelling tables overflowed */
  MF_ENUMERIC = -5,     /* the device flagged an invalid state (see mf_last_error) */
  MF_ESTATE = -6,       /* call not valid in the context's current state */
  MF_EUNSUPPORTED = -7, /* option not built into this library */
  MF_EINTERNAL = -8
};

/* storage / arithmetic forms of the populations */
enum mf_precision {
  MF_FP64 = 0,     /* f, g and all cell fields in binary64 */
  MF_FP32 = 1,     /* f, g and cell fields in binary32; bubble table in binary64 */
  MF_F16S = 2,     /* f stored as binary16 offsets f_i - w_i, arithmetic in binary32 */
  MF_BF16S = 3,    /* f stored as bfloat16 offsets f_i - w_i, arithmetic in binary32 */
  MF_F16S_G16 = 4  /* f as in MF_F16S; g stored as binary16 scaled offsets
                      (g_i - w_i c0) / c0 (c0 = initial concentration, or k_H p_atm
                      when c0 = 0), arithmetic in binary32 */
};

enum mf_rheology { MF_NEWTONIAN = 0, MF_POWER_LAW = 1, MF_CARREAU_YASUDA = 2 };
enum mf_curvature { MF_CURV_PLAIN = 0, MF_CURV_MLP = 1 };

/* Gas flux into the bubbles (Sec. 3.2, Eq. gascurrent).
 * MF_FLUX_LEDGER: each interface cell books, per direction whose source is gas, the
 *   dissolved gas it sent to the gas side minus what the Henry's-law rebuild returned;
 *   cell conversions move the dissolved gas of emptied cells into their bubble and take
 *   that of new interface cells out of it. Dissolved gas plus bubble, atmosphere and
 *   collapsed gas is then conserved exactly.
 * MF_FLUX_PAPER: the printed formula, with F read as the liquid and interface cells and
 *   rho as 1: every interface cell x of bubble j books the populations its fluid
 *   neighbours send towards it minus those it sends to them, less c(x)(alpha_new(x) -
 *   alpha_old(x)); conversions move no gas. Gas is not conserved in this mode. */
enum mf_flux_mode { MF_FLUX_LEDGER = 0, MF_FLUX_PAPER = 1 };

/* cell types reported by MF_FIELD_TYPE */
enum mf_cell_type { MF_GAS = 0, MF_INTERFACE = 1, MF_LIQUID = 2, MF_WALL = 3 };

/* fields for mf_read_field / mf_write_field */
enum mf_field {
  MF_FIELD_TYPE = 0,  /* uint8 [N] cell type (mf_cell_type) */
  MF_FIELD_LABEL = 1, /* int32 [N] bubble id of gas / interface cells (0 = atmosphere), -1 elsewhere */
  MF_FIELD_RHO = 2,   /* double [N] density of interface cells */
  MF_FIELD_UX = 3,    /* double [N] velocity of interface cells */
  MF_FIELD_UY = 4,
  MF_FIELD_UZ = 5,
  MF_FIELD_ALPHA = 6, /* double [N] fill fraction (1 on liquid, 0 on gas and walls) */
  MF_FIELD_MASS = 7,  /* double [N] liquid mass M of interface cells */
  MF_FIELD_CONC = 8,  /* double [N] dissolved gas c = sum_i g_i (liquid and interface cells) */
  MF_FIELD_KAPPA = 9, /* double [N] curvature of interface cells */
  MF_FIELD_PI = 10,   /* double [N] disjoining pressure of interface cells */
  MF_FIELD_F = 11,    /* double [Q][N] post-collision populations f */
  MF_FIELD_G = 12     /* double [Qg][N] post-collision ADE populations g */
};

typedef struct mf_ctx mf_ctx; /* opaque; one context is used by one host thread at a time */

typedef struct mf_params {
  size_t struct_size;    /* = sizeof(mf_params) */
  int32_t dim;           /* 2 (D2Q9 + D2Q5) or 3 (D3Q19 + D3Q7) */
  int32_t nx, ny, nz;    /* grid incl. wall layers; nz = 1 in 2D */
  int32_t periodic[3];   /* 1: periodic axis, 0: closed by a wall layer on both sides */
  int32_t gas_from;      /* cells whose last coordinate >= gas_from start as headspace
                            gas of the atmosphere (id 0); < 0: no headspace */
  int32_t precision;     /* mf_precision */
  int32_t rheology;      /* mf_rheology */
  int32_t curvature;     /* mf_curvature */
  int32_t cleanup;       /* 1: stranded interface cells are filled / emptied */
  int32_t max_ids;       /* bubble-table capacity (ids 0..max_ids-1, never reused) */
  double tau;            /* BGK relaxation time (Newtonian) */
  double D;              /* gas diffusivity; tau_g = 1/2 + D / c_s,g^2 */
  double sigma;          /* surface tension (gamma in the paper) */
  double kH;             /* Henry constant: c = kH p at interfaces */
  double RT;             /* ideal-gas constant times temperature */
  double k_pi;           /* disjoining-pressure constant (0: off) */
  double d_max;          /* disjoining-pressure range in cells */
  double p_atm;          /* pressure of the atmosphere (id 0) */
  double q;              /* gas source per cell and step */
  double eps;            /* conversion threshold: fill if M > (1+eps) rho, empty if M < -eps rho */
  double S0;             /* initial supersaturation c0 / (kH p_atm) */
  double pl_n, pl_nu_ref, pl_gdot_ref; /* power law nu = nu_ref (gdot/gdot_ref)^(n-1) */
  double tau_min, tau_max;             /* clamp of the power-law relaxation time */
  double accel[3];       /* body-force acceleration a (gravity), lattice units; all zero:
                            no force term. Liquid and interface cells take the external
                            force term of Eq. collision in the form of Guo, Zheng and Shi
                            (2002): F = rho a, velocity (sum f e + F/2) / rho, and
                            (1 - omega/2) w_i [(e_i - u)/c_s^2 + (e_i.u) e_i/c_s^4].F added
                            after the relaxation; the power-law strain rate takes the
                            force correction (u F + F u)/2. |a_k| <= 1e-2; a_z = 0 in 2D. */
  double cy_tau0, cy_tau_inf, cy_lambda, cy_a, cy_n;
                         /* Carreau-Yasuda (rheology MF_CARREAU_YASUDA, Eq. carreauTau):
                            (tau - tau_inf)/(tau0 - tau_inf) = (1 + (lambda gdot)^a)^((n-1)/a),
                            gdot = sqrt(2 S:S) from the non-equilibrium momentum flux at the
                            cell's own tau (implicit, solved per cell). Shear thinning:
                            1/2 < tau_inf <= tau0, 0 < n <= 1, a > 0, lambda >= 0, and
                            (tau0 - tau_inf)(1 - n) < tau_inf, which makes tau unique. */
  int32_t flux_mode;     /* a value of mf_flux_mode: Sec. 3.2, Eq. gascurrent */
} mf_params;

/* One entry of the bubble table (Sec. 3.5: per-bubble volume, gas content and pressure). */
typedef struct mf_bubble {
  int32_t id;
  int32_t alive;
  double volume;      /* sum over the bubble's cells of (1 - alpha) */
  double gas_mass;    /* m_g */
  double pressure;    /* m_g RT / max(volume, 1/2) (Eq. idealgas) */
  int32_t n_cells;    /* gas and interface cells carrying the id */
  int32_t reserved;
  double centroid[3]; /* centre of the gas volume: sum (1 - alpha) x / sum (1 - alpha) over
                         the bubble's cells (plain coordinates, no unwrapping across periodic
                         axes; z = 0 in 2D) */
} mf_bubble;

typedef struct mf_totals {
  int64_t step;
  double lost_liquid;   /* excess liquid mass that found no interface neighbour */
  double atm_gas;       /* gas handed to the atmosphere */
  double collapsed_gas; /* gas of bubbles whose last cell vanished */
  int32_t next_id;
  int32_t n_bubbles;    /* live bubbles, atmosphere excluded */
  int32_t n_interface;  /* interface cells entering the last step */
  int32_t status;       /* device status bits, 0 when healthy */
  double liquid_mass;   /* sum of rho over liquid cells and of M over interface cells
                           (Sec. 2.1: the mass that conversions and the excess split conserve) */
  double dissolved_gas; /* sum of c = sum_i g_i over liquid and interface cells */
  double bubble_gas;    /* sum of m_g over the live bubbles (atmosphere excluded) */
} mf_totals;

/* Library ABI version (MF_ABI_VERSION of the build). Infrastructure of the boundary; it
 * implements no passage of the paper. */
int mf_abi_version(void);

/* Message of the last failed call on ctx; with ctx == NULL, of the last failed call
 * without a context (mf_create, mf_workspace_bytes, networks, batches) on this thread.
 * The pointer stays valid until the next call on the same context. Infrastructure; no
 * passage of the paper. */
const char *mf_last_error(const mf_ctx *ctx);

/* Device bytes a context with these parameters needs: the populations f and g of the
 * lattice Boltzmann equation (Sec. 2, Eq. LBE; Sec. 3.1, Eq. diffusion) in two buffers
 * each, the cell fields of the free-surface model (Sec. 2.1: type, mass M, fill
 * fraction alpha), interface lists, labelling tables and the bubble table (Sec. 3.5).
 * MF_EINVAL on invalid parameters (the rules of mf_create). */
int mf_workspace_bytes(const mf_params *p, size_t *bytes);

/* Create a context (Sec. 2 set-up: a liquid at rest below the headspace, walls on closed
 * axes): validates p (MF_EINVAL), carves its arrays out of dev_workspace (device memory of
 * at least mf_workspace_bytes, owned by the caller and kept alive until mf_destroy; a
 * smaller one gives MF_ENOMEM) or, when dev_workspace is NULL, allocates them itself
 * (MF_ENOMEM on failure). stream is a hipStream_t (NULL: the null stream). Initialises the
 * equilibrium at rest f = w_i (Eq. equilibrium) and g = w_i c0 with c0 = S0 kH p_atm
 * (Sec. 3.1), and the atmosphere (id 0, pressure p_atm). */
int mf_create(const mf_params *p, void *dev_workspace, size_t ws_bytes, void *stream, mf_ctx **out);

/* Destroy a context: waits for its stream, frees only memory the library allocated
 * (never the caller's workspace). NULL is accepted. Infrastructure; no passage. */
int mf_destroy(mf_ctx *ctx);

/* Nucleation (Sec. 3.4): n spheres (disks in 2D) with centres [n][3] (z ignored in
 * 2D), radii [n] and initial pressures p0 [n] (host arrays). Each is voxelised with 8
 * sample points per axis and cell; nucleus k gets id k+1; overlapping nuclei merge to
 * the smaller id. Gas mass = p0 V / RT (Eq. idealgas). Valid once, before mf_step
 * (MF_ESTATE otherwise). MF_EINVAL if a nucleus is not inside the liquid. */
int mf_nucleate(mf_ctx *ctx, int32_t n, const double *centers, const double *radii, const double *p0);

/* Nucleation sites from a nucleation probability field by Poisson-disk sampling (Sec. 3.4;
 * host code, no GPU work). The liquid region of the grid p describes (dim, nx, ny, nz,
 * periodic, gas_from) is filled by the active-list method: sites are sphere centres with
 * radii uniform in [r_min, r_max]; two sites keep |x_i - x_j| >= r_i + r_j + gap (the spheres
 * never overlap and gap cells of liquid separate them; distances wrap on periodic axes); each
 * sphere stays one cell clear of the wall layers and of the headspace; each site tries
 * `attempts` candidates in the shell [d, 2d], d = r_i + r_new + gap, around it. The field prob
 * (host, one value in [0, 1] per cell in cell order, x fastest; NULL: all ones) then thins the
 * filled set: in placement order a site is kept with the probability of its nearest cell,
 * until max_n are kept. centers (host, max_n x 3, z = 0 in 2D) and radii (host, max_n) receive
 * the kept sites in order and *n_out their number; the result depends only on the arguments
 * (SplitMix64 stream from seed, binary64 arithmetic without contraction). MF_EINVAL on a bad
 * grid, r_min <= 0, r_max < r_min, gap < 0, attempts < 1, max_n < 0 or a field value outside
 * [0, 1]. Feed the sites to mf_nucleate. */
int mf_poisson_nuclei(const mf_params *p, const float *prob, int32_t max_n, double r_min, double r_max,
                      double gap, int32_t attempts, uint64_t seed, double *centers, double *radii,
                      int32_t *n_out);

/* Advance nsteps time steps (enqueued on the context stream; returns without waiting;
 * nsteps < 0 gives MF_EINVAL, a learned-curvature context without a network MF_ESTATE).
 * Each step is the paper's time step: stream and collide f (Sec. 2, Eqs. LBE,
 * streamingstep, collisionstep, equilibrium, tau / carreauTau) and g (Sec. 3.1, Eqs.
 * diffusion, diffusionconst), the interface mass exchange (Sec. 2.1, Eq. massexchange),
 * the free-surface and Henry's-law rebuilds (Eqs. reconstruct, rhob,
 * rhobplusdisjoining; Eqs. henryslaw, reconstructdiffusion), cell conversion with
 * excess redistribution (Sec. 2.1), bubble labelling with the gas bookkeeping (Sec.
 * 3.2 Eq. gascurrent, Sec. 3.5) and pressures (Eq. idealgas), curvature (Sec. 2.2) and
 * disjoining pressure (Sec. 3.3, Appendix A Algorithm 1). The labelling and geometry of
 * a step run on streams of the context's own, beside the next step's bulk sweep; all
 * work is joined into the context stream before mf_step returns. Device-side failures
 * surface at the next mf_sync. */
int mf_step(mf_ctx *ctx, int32_t nsteps);

/* Wait for the context stream and report the device status word that the kernels set
 * themselves: MF_ENUMERIC for a non-positive or non-finite density in a collision (Sec.
 * 2, Eq. collision), a liquid cell next to gas or an interface cell with an invalid
 * bubble id (the invariants of Sec. 2.1); MF_ECAPACITY for a full bubble or labelling
 * table (Sec. 3.5). The state is left in place for inspection. */
int mf_sync(mf_ctx *ctx);

/* Copy a field (mf_field: the cell type and fill fraction of Sec. 2.1, populations of
 * Sec. 2 and 3.1, curvature of Sec. 2.2, disjoining pressure of Sec. 3.3, bubble ids of
 * Sec. 3.5) into dst (caller-owned host memory, or device memory when dst_on_device is
 * 1), converted to the element type mf_field states, cell index x fastest. dst_bytes
 * must hold the field (MF_EINVAL otherwise). Synchronises the context stream. */
int mf_read_field(mf_ctx *ctx, int32_t field, void *dst, size_t dst_bytes, int32_t dst_on_device);

/* Overwrite a field from host memory (hand-built states of the free-surface model of
 * Sec. 2.1); same layout as mf_read_field. Allowed before the first mf_step (MF_ESTATE
 * after). Call mf_refresh afterwards. A type field must keep walls on the outer layer of
 * every closed axis (MF_EINVAL otherwise). */
int mf_write_field(mf_ctx *ctx, int32_t field, const void *src, size_t src_bytes);

/* Set one bubble-table entry (Sec. 3.5: gas mass, volume, pressure of Eq. idealgas) for
 * hand-built states; MF_EINVAL for an id outside the table. The gas side of the
 * interface cells (Eq. reconstruct at the bubble pressure) follows before the next step. */
int mf_set_bubble(mf_ctx *ctx, int32_t id, double gas_mass, double volume, double pressure, int32_t alive);

/* Recompute the derived state of a hand-written state: interface lists, curvature (Sec.
 * 2.2), disjoining pressure (Sec. 3.3) and the gas side of the interface cells (Eqs.
 * rhob, rhobplusdisjoining). relabel = 1 also runs the bubble labelling of Sec. 3.5 with
 * no gas flux. Synchronises; reports the device status like mf_sync. */
int mf_refresh(mf_ctx *ctx, int32_t relabel);

/* The bubble table of Sec. 3.5 (volume, gas content and Eq. idealgas pressure of every
 * bubble; cell counts and gas-volume centroids from one pass over the grid): live
 * bubbles (atmosphere excluded) in ascending id into dst (caller-owned host array of
 * capacity entries; NULL only with capacity 0); *n_out = number of live bubbles (may
 * exceed capacity; then only capacity entries are written). Synchronises. */
int mf_read_bubbles(mf_ctx *ctx, mf_bubble *dst, int32_t capacity, int32_t *n_out);

/* Conserved totals and ledgers: liquid mass (Sec. 2.1, conserved by the mass exchange,
 * conversions and excess split), dissolved gas (Sec. 3.1) and bubble gas (Sec. 3.2), the
 * atmosphere, collapsed and lost-liquid ledgers of Sec. 3.5, and counters. The liquid
 * mass and dissolved gas are summed on the device in fixed point (independent of
 * order). Synchronises. */
int mf_totals_get(mf_ctx *ctx, mf_totals *out);

/* Checkpoint (no passage of the paper: a production form). mf_save writes the whole
 * state of ctx (device arena, step count, buffer parities, attached network weights)
 * to the file path; mf_load reads such a file into a context created with the same
 * parameters (MF_EINVAL otherwise, or for a file of another library version) and
 * continues from it bit for bit. Both wait for the context stream; MF_EHIP on an I/O or
 * copy failure (after a failed mf_load the state is undefined). */
int mf_save(mf_ctx *ctx, const char *path);
int mf_load(mf_ctx *ctx, const char *path);

/* Fault injection for tests of the failure path (no passage of the paper): overwrite one
 * element of a field in its storage form: MF_FIELD_F or MF_FIELD_G (comp = direction),
 * MF_FIELD_RHO, MF_FIELD_ALPHA or MF_FIELD_MASS (comp = 0) at cell. No check of the
 * value: a non-finite population is reported as MF_ENUMERIC by mf_sync after the next
 * step. MF_EINVAL for other fields, cells or components. Synchronises. */
int mf_debug_poke(mf_ctx *ctx, int32_t field, int64_t cell, int32_t comp, double value);

/* ------------------------------------------------------------ learned curvature ---
 * A small network (125-64-64-1, GELU, bfloat16 weights and activations, binary32
 * accumulation on the matrix cores) maps the 5x5x5 fill-fraction stencil of an interface
 * cell, brought to a canonical orientation by the cube symmetry that orders its
 * central-difference normal as m_x >= m_y >= m_z >= 0, to its mean curvature (the
 * curvature of Eq. rhob). It is trained on stencils of voxelised spheres and ellipsoids
 * with exact curvature labels. The plain paraboloid fit remains the fallback. */
typedef struct mf_mlp mf_mlp; /* opaque trained network (device parameters) */

typedef struct mf_mlp_train_spec {
  size_t struct_size;  /* = sizeof(mf_mlp_train_spec) */
  int64_t n_train;     /* training stencils (e.g. 1.9M) */
  int64_t n_val;       /* validation stencils (e.g. 0.1M), generated after the training ones */
  int32_t epochs;      /* passes over the training set */
  int32_t batch;       /* multiple of 64 (e.g. 4096) */
  double lr;           /* Adam step, cosine-decayed to 0 over the run */
  double noise;        /* standard deviation of the fill noise on cut cells (0.01) */
  uint64_t data_seed;  /* stencil generator seed */
} mf_mlp_train_spec;

/* Number of binary32 parameters in the layout of mf_mlp_get_params: W1 [128][64] (rows
 * 125..127 zero), b1 [64], W2 [64][64], b2 [64], W3 [64], b3. */
int mf_mlp_param_count(void);

/* Create a network with weights uniform in +-1/sqrt(fan_in) (SplitMix64 stream of
 * init_seed) and zero biases; device memory is owned by the network. */
int mf_mlp_create(uint64_t init_seed, mf_mlp **out);
int mf_mlp_destroy(mf_mlp *m);

/* Train on the GPU (stream: hipStream_t, NULL = null stream): generate the stencils, then
 * Adam on the mean squared error of 8 kappa for spec->epochs epochs; *val_rmse receives
 * the validation root-mean-square curvature error. Synchronises. */
int mf_mlp_train(mf_mlp *m, const mf_mlp_train_spec *spec, void *stream, double *val_rmse);

/* Copy the binary32 master parameters out / in (host buffers of mf_mlp_param_count floats). */
int mf_mlp_get_params(const mf_mlp *m, float *dst);
int mf_mlp_set_params(mf_mlp *m, const float *src);

/* Write the network's binary32 parameters to the file path / create a network from such
 * a file (*out owned by the caller, released with mf_mlp_destroy). MF_EINVAL for a file
 * that is not a network file of this library, MF_EHIP on an I/O or copy failure. */
int mf_mlp_save(const mf_mlp *m, const char *path);
int mf_mlp_load(mf_mlp **out, const char *path);

/* Generate n stencils (sample indices first..first+n-1 of the counter-based generator)
 * into host buffers: raw stencils [n][125] (dz outer, dx inner) and exact curvature [n]. */
int mf_mlp_generate(uint64_t data_seed, int64_t first, int64_t n, double noise, float *stencils,
                    float *kappa, void *stream);

/* Curvature of n raw stencils [n][125] (host) through canonicalisation and the network. */
int mf_mlp_eval(const mf_mlp *m, const float *stencils, int64_t n, float *kappa, void *stream);

/* For callers that cannot allocate device memory (code under stream capture, serving
 * loops, harnesses that forbid hipMalloc): the curvature of n raw stencils as
 * mf_mlp_eval computes it, with stencils [n][125] and kappa [n] in device memory,
 * enqueued on stream (hipStream_t, NULL = null stream) without waiting. The call
 * allocates nothing: its intermediate arrays live in a static device array of 12.6 MB
 * that every GPU the library runs on holds until the process ends, sized for at most
 * 8192 stencils per call (MF_EINVAL beyond). All calls on one GPU share that array, so
 * calls that overlap on one GPU (different streams, threads) race. */
int mf_mlp_eval_noalloc(const mf_mlp *m, const float *stencils, int64_t n, float *kappa, void *stream);

/* Loss and parameter gradient on one batch of raw stencils [B][125] with targets 8 kappa
 * (host buffers; grad has mf_mlp_param_count floats). For gradient checks. */
int mf_mlp_grad(const mf_mlp *m, const float *stencils, const float *target8, int32_t B, float *grad,
                double *loss, void *stream);

/* Use the network for the curvature of ctx (the curvature of Eq. rhob; requires
 * curvature = MF_CURV_MLP in the parameters, MF_ESTATE otherwise); the weights are copied,
 * the network may be destroyed afterwards. */
int mf_attach_mlp(mf_ctx *ctx, const mf_mlp *m);

/* Time spent in a kernel group over the steps since mf_profile_enable(ctx, 1), in
 * milliseconds (total) with the number of steps timed, measured with HIP events on the
 * context stream: group 0 = the bulk lattice sweep kernel (the whole sweep on domains
 * that use the per-cell kernel), 1 = whole step (from its list build to the end of its
 * labelling and geometry, which overlap the next step), 2 = the interface-cell sweep
 * kernel (zero on domains that use the per-cell kernel). At most 4096 steps are timed
 * per enable; a further mf_step returns MF_ESTATE until the next enable. */
int mf_profile_enable(mf_ctx *ctx, int32_t on);
int mf_profile_get(mf_ctx *ctx, int32_t group, double *ms_total, int64_t *launches);

/* ---------------------------------------------------------------- tuning, batching
 * Production forms beyond the paper: a tuner for the launch shape of the bulk lattice
 * sweep, and the advance of many independent domains with one launch per kernel for all
 * of them.
 */

/* Number of launch variants of the bulk lattice sweep (cells per thread x threads per
 * work-group: 0 = 4 x 256, 1 = 2 x 256, 2 = 4 x 128, 3 = 2 x 128, 4 = 8 x 256, 5 = 8 x 128,
 * 6 = 8 x 64, 7 = 4 x 64). */
#define MF_SWEEP_VARIANTS 8

/* Time every applicable variant of the bulk sweep on the context's current state (reps
 * launches each; the kernel writes only the spare population buffer, so the state is not
 * changed), select one of those with 256-thread work-groups (0, 1, 4: inside a step the
 * bulk kernel shares the GPU with the labelling and curvature kernels, which one-wave
 * work-groups starve) for later steps: the default shape (4 for 16-bit storage, 0 for
 * binary32), unless another is more than 5% faster alone, then the fastest; inside a step
 * the default runs faster than shapes that tie with it alone. Return it in *best_variant (-1 when
 * none applies: binary64, periodic axes, or rows that are not a multiple of the vector
 * width). ms_per_variant (MF_SWEEP_VARIANTS floats, nullable) receives the mean time per
 * launch of every variant, -1 for variants that do not apply. Synchronises the context
 * stream. Every variant computes the same results. */
int mf_tune(mf_ctx *ctx, int32_t reps, int32_t *best_variant, float *ms_per_variant);

/* Select a bulk-sweep variant by hand (-1: the default). */
int mf_set_sweep_variant(mf_ctx *ctx, int32_t variant);

/* A batch of n distinct contexts (created, nucleated and, for the learned curvature,
 * with a network attached) advanced together (the time step of mf_step; a production form
 * beyond the paper). The batch owns a stream of its own; the contexts stay owned by the
 * caller and must outlive the batch. Errors are reported through mf_last_error(NULL). */
typedef struct mf_batch mf_batch;
int mf_batch_create(int32_t n, mf_ctx *const *ctxs, mf_batch **out);

/* The batch's autotuner: for every group of domains that share their kernels and every
 * domain shape in it, time the batched bulk-sweep launch over the domains of that shape in
 * every launch shape that fits them (reps launches each; the bulk kernel writes only the
 * spare population buffer, so the state is not changed) and keep the fastest for those
 * domains; variants (n ints, nullable) receives each domain's launch shape (-1: per-cell
 * sweep). Synchronises. */
int mf_batch_tune(mf_batch *b, int32_t reps, int32_t *variants);

/* Advance every domain by nsteps. The domains are grouped by the kernels they use
 * (dimension, storage, bulk or per-cell sweep, body force, learned curvature; at most 64
 * per group), and every kernel of a step runs as one launch for all domains of a group:
 * each domain takes its range of the launch's work-groups, and each work-group finds its
 * domain by a binary search over the ranges passed with the launch. Each group has two
 * streams of its own: as in mf_step, the second half of a step's conversions, the labelling
 * and the geometry run beside the next step's bulk sweep. The per-domain tables are built
 * on first use and again after any state change made outside the time step (nucleation,
 * field writes, refresh, network attachment, tuning) or when the domains' buffer parities
 * no longer agree (a domain stepped alone by an odd count). Results are those of mf_step
 * on each context, bit for bit. Work already queued on the contexts' streams runs first,
 * and later work queued there waits for the batch. Profiling must be off (MF_ESTATE). */
int mf_batch_step(mf_batch *b, int32_t nsteps);

/* Wait for the batch stream and free the batch (not the contexts). */
int mf_batch_destroy(mf_batch *b);

#ifdef __cplusplus
}
#endif
#endif
