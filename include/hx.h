/*
 * hx.h - C ABI of libhx.so: matrix-free residual and linearised operator of finite-strain
 * hyperelasticity on hexahedral Q_p elements, evaluated by sum factorisation on AMD MI355X
 * (gfx950).
 *
 * The operation is the one of the paper (Schussnig, Fehn, Munch, Kronbichler, "Matrix-free
 * higher-order finite element methods for hyperelasticity"):
 *   - residual   r(v, u) = (Grad v, P)_Omega0 with P = F S          (Section 2, material residual)
 *   - linearised D_u r(v, du)|_u = (Grad v, Grad du S + F D_u S)    (Section 2, directional
 *                derivative of the residual; Problem 2.2)
 *   - laws       compressible / nearly incompressible neo-Hookean and the dispersed two-fibre
 *                model (Section 3), in the stable forms of Section 4
 *   - storage    quadrature-point data recomputed on the fly or stored once per Newton step
 *                and reused by every operator application (Section 5, Algorithm 1)
 *
 * No C++ exception crosses this boundary. Every call returns hx_status; hx_last_error() gives a
 * message for the last failing call on a context. No torch or HIP type appears in a signature:
 * device buffers are plain pointers, streams are passed as void* (a hipStream_t, NULL = the
 * default stream).
 *
 * Conventions shared by all calls
 * -------------------------------
 * Meshes (the domain Omega0 of Problem 2.1 in Section 2, cut into hexahedra), in two forms:
 *   - hx_setup: a general conforming mesh of hexahedra given by connectivity (vertex ids of each
 *     cell's 8 corners) with boundary ids on the cell faces;
 *   - hx_setup_lattice: a structured nx x ny x nz lattice (cells e = ex + nx*(ey + ny*ez)),
 *     each lattice direction optionally periodic; the fast case, addressed by index arithmetic.
 * The geometry of a cell is the trilinear map of its 8 vertices, or a polynomial map of degree g
 * given by its values at the (g+1)^3 equispaced points (i/g, j/g, k/g) of the reference cell
 * [0,1]^3, local point index i + (g+1)(j + (g+1)k) (curved cells, as high-order mesh files
 * describe them; g = p is the isoparametric case). Corner a + 2b + 4c of a cell is its reference
 * corner (a, b, c), and every cell must be positively oriented (det J0 > 0 at its Gauss points).
 *
 * Nodes: the Gauss-Lobatto points of degree p in every cell, shared between cells along common
 * vertices, edges and faces. Lattice: N_d = n_d*p (+1 if direction d is not periodic) points per
 * direction, node = I + N_x*(J + N_y*K). General mesh: first-touch order - cells in order, each
 * cell's local nodes (i, j, k) with i fastest, a node numbered where it is first met; which local
 * nodes coincide is decided by the vertex ids of the vertex, edge or face they lie on, whatever
 * the cells' local orientations (meshes in which two distinct edges join the same two vertices,
 * or two distinct faces the same four, are outside this contract). Quadrature: (p+1)^3 Gauss
 * points per cell.
 *
 * Vectors: device arrays in structure-of-arrays layout [3][n_nodes] (DoF index c*n_nodes+node),
 * contiguous, owned by the caller. FP64 (double) unless a call says otherwise.
 *
 * Dirichlet: nodes on the constrained faces (lattice: hx_lattice.dirichlet_faces; general mesh:
 * the faces whose boundary id is in hx_options.dirichlet_bid_mask) carry homogeneous data
 * (the test space H^1_0 of Problems 2.1/2.2). hx_residual writes 0 on constrained rows;
 * hx_apply_tangent treats du as 0 on constrained DoFs for the free rows and writes dst = du on
 * constrained rows (operator P_f K P_f + P_c, symmetric).
 *
 * Asynchrony: operator calls enqueue kernels on the given stream and return without waiting,
 * except hx_update_linearization, which waits on its stream to read the device status flag.
 * Calls on one context must not overlap in time on different streams: hx_residual and
 * hx_apply_tangent share the context's element-vector buffer (below).
 *
 * Assembly (Section 6, the sum of the element vectors): an apply or residual is two kernels. The
 * element kernel writes each cell's element vector into a per-context buffer in which every cell
 * owns its own (p+1)^3 brick; a node kernel then adds, in a fixed order, the bricks of the cells
 * that share each node and writes every row of the output, the constrained rows included. No
 * atomics are used, so repeated calls give bit-identical results. (General meshes read each
 * cell's nodes from an int32 map and each node's brick entries from a list built at setup.)
 */
#ifndef HX_H
#define HX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hx_ctx_s* hx_ctx;

typedef enum {
  HX_OK = 0,
  HX_E_ARG = 1,           /* invalid argument (null pointer, size, unknown enum value) */
  HX_E_HIP = 2,           /* a HIP runtime call failed */
  HX_E_NOMEM = 3,         /* device allocation failed */
  HX_E_STATE = 4,         /* call out of order (e.g. apply before any linearisation update) */
  HX_E_INVERTED = 5,      /* det J0 <= 0 in a cell (setup) or J <= 0 at a q-point (update) */
  HX_E_NONFINITE = 6,     /* NaN or Inf in the linearisation data */
  HX_E_NOT_CONVERGED = 7, /* iterative solve did not reach its tolerance */
  HX_E_UNSUPPORTED = 8    /* combination of degree / law / precision / mode not built */
} hx_status;

typedef enum { HX_LAW_CNH = 0, HX_LAW_INH = 1, HX_LAW_FIBER = 2 } hx_law;

/* What hx_update_linearization keeps per quadrature point (Section 5, storage strategies).
 *   NONE     nothing: every apply re-interpolates u_k and recomputes kinematics and the law
 *            (the "on-the-fly" variant); the library keeps a copy of u_k.
 *   FINV_J   F^-1 (9 words) and J - 1 (1 word); the apply recomputes the law scalars and the
 *            trilinear geometry.
 *   TANGENT  the symmetric 9x9 tangent in reference coordinates, 45 words:
 *            D_(i a)(k b) = w_q detJ0 sum_{J,L} J0^-1_aJ A_iJkL J0^-1_bL, A = dP/dF,
 *            geometry and weight folded in; the apply is a 9x9 product per q-point. */
typedef enum {
  HX_STORE_NONE = 0,
  HX_STORE_FINV_J = 1,
  HX_STORE_TANGENT = 2,
  HX_STORE_SPATIAL = 3, /* integration over the spatial configuration (Section 2, spatial residual
                           and its linearisation; Section 5, spatial forms): the inverse Jacobian of
                           the deformed map X + u_k scaled by sqrt(w det J0), the Kirchhoff stress
                           tau and the law's data for J c : (.)^S (cNH 2(mu - 2 lambda ln J); iNH c1,
                           c2 and (2 mu / 3) J^-2/3 b; fibre per family F H_i F^T and
                           2 c3 (2 k2 E_i^2 + 1)): 16 / 23 / 37 words for cNH / iNH / fibre;
                           FP64 or FP32 data */
  HX_STORE_SPATIAL_RECOMPUTE = 4, /* the spatial-configuration operator with nothing stored: every
                                     apply re-interpolates u_k and forms the SPATIAL mode's data
                                     on the fly (the paper's "recompute all" variant over Omega_t);
                                     the library keeps a copy of u_k */
  HX_STORE_SCALARS = 5, /* the paper's stored-scalar stage over the reference configuration (Section
                           5 and Tab. overview_precompute): the law's scalars are stored (cNH ln J;
                           iNH J - 1, J^-2/3, c1, c2; fibre adds c3 and E_i per family: 1 / 4 / 8
                           words) and every apply re-interpolates u_k for F (the library keeps a
                           copy of u_k); FP64 or FP32 data */
  HX_STORE_TENSORS = 6, /* the paper's stored-tensor stage over the reference configuration: F, S,
                           F^-1, C^-1 (9 + 6 + 9 + 6 words, S and C^-1 symmetric) and the scalars of
                           D_u S (cNH ln J; iNH J^-2/3, c1, c2; fibre adds 2 c3 (2 k2 E_i^2 + 1) per
                           family: 31 / 33 / 35 words); the apply forms P' = G S + F D_u S[G]
                           term by term; FP64 or FP32 data */
  HX_STORE_SPATIAL_SCALARS = 7, /* the paper's stored-scalar stage over the spatial configuration:
                                   the SCALARS words are stored, and every apply re-interpolates
                                   u_k and forms the SPATIAL mode's data from it with those scalars
                                   (the library keeps a copy of u_k); FP64 or FP32 data */
  HX_STORE_AUTO = 255 /* only where a field says so: the mode is chosen by hx_autotune_storage */
} hx_storage;

/* Arithmetic of hx_apply_tangent and the type of its stored data.
 *   FP64             double vectors, double compute, double data
 *   FP32             float vectors, float compute, float data
 *   FP32_BF16DATA    float vectors and compute, bfloat16 data (FINV_J, TANGENT, SPATIAL)
 *   FP32_FP16DATA    float vectors and compute, binary16 data scaled per cell by a power of
 *                    two (TANGENT only: its words share one magnitude per cell)
 * The linearisation data itself is always computed in FP64 and rounded once when stored. */
typedef enum {
  HX_FP64 = 0,
  HX_FP32 = 1,
  HX_FP32_BF16DATA = 2,
  HX_FP32_FP16DATA = 3
} hx_precision;

/* A general conforming mesh of hexahedra (Section 2: the domain Omega0 and its boundary parts;
 * Section 5: the geometry J0 enters every stored set). All arrays are HOST arrays copied by
 * hx_setup; the caller keeps ownership. */
typedef struct {
  int64_t n_vertices, n_cells;  /* n_cells >= 1; every cell's corners are 8 distinct vertex ids */
  const double* vertices;       /* [n_vertices][3] */
  const int64_t* cells;         /* [n_cells][8] vertex ids, corner a + 2b + 4c at reference corner
                                   (a, b, c) */
  const uint8_t* face_bid;      /* [n_cells][6] or NULL: boundary id of each local face
                                   (-x, +x, -y, +y, -z, +z of the reference cell), 0 = none,
                                   1..31 may be constrained (hx_options.dirichlet_bid_mask) and
                                   carry pressure loads (hx_surface_load) */
  int32_t geom_degree;          /* g in [1, 8]: degree of every cell's map */
  const double* geom_nodes;     /* [n_cells][(g+1)^3][3] or NULL (only for g = 1: the trilinear
                                   map of the vertices): each cell's map at its equispaced points */
  const double* frames;         /* [n_cells][3][3] or NULL: local fibre frames, as for lattices */
} hx_mesh;

/* A structured lattice of hexahedra, the fast case (index arithmetic instead of a node map). */
typedef struct {
  int32_t nx, ny, nz;       /* cells per lattice direction, each >= 1 */
  int32_t periodic;         /* bit d (d = 0,1,2 for x,y,z) set: direction d is periodic */
  const double* vertices;   /* HOST array [V_z][V_y][V_x][3], V_d = n_d (+1 if not periodic),
                               x fastest; copied by hx_setup_lattice; may be NULL when geom_nodes
                               is given */
  uint32_t dirichlet_faces; /* bit f set: face f is constrained, f = 0..5 = -x,+x,-y,+y,-z,+z;
                               bits of periodic directions are ignored */
  const double* frames;     /* HOST array [n_cells][3][3] or NULL: per cell the rows E1, E2, E3 of
                               an orthonormal right-handed local frame (fibre frame of Section 3;
                               cells in lattice order, x fastest); copied by the setup. With frames,
                               the FIBER law's H4, H6, M4, M6 are components in the local frame,
                               H_i = sum_ab H_i[a][b] E_a (x) E_b in each cell; NULL = the global
                               axes. Ignored by the other laws. A frame that is not orthonormal
                               to 1e-8 or not right-handed gives HX_E_ARG. */
  int32_t geom_degree;      /* g in [1, 8] with geom_nodes, else 1 */
  const double* geom_nodes; /* HOST array [n_cells][(g+1)^3][3] or NULL: curved cells, each cell's
                               map at its equispaced points (cells in lattice order); NULL = the
                               trilinear map of the vertices */
} hx_lattice;

/* Material parameters (Section 3). cNH uses mu, lambda with Psi = mu/2 (I1 - 3 - 2 ln J) +
 * lambda ln^2 J. iNH uses mu, kappa with Psi = mu/2 (J^-2/3 I1 - 3) + kappa/4 (J^2 - 1 - 2 ln J).
 * FIBER adds k1, k2 and, for the two families i = 4, 6, the symmetric structure tensor H_i
 * (row-major 3x3) and the mean fibre direction M_i used in the tension switch I*_i > 1
 * (hx_fiber_structure computes both from dispersion parameters). */
typedef struct {
  hx_law law;
  double mu, lambda, kappa, k1, k2;
  double H4[9], H6[9];
  double M4[3], M6[3];
} hx_material;

typedef struct {
  int32_t jpow_newton_iters;   /* FP32 arithmetic: J^-2/3 by this many Newton steps from x0 = 1
                                  (Algorithm 2, Section 4), accurate only near J = 1;
                                  0 = cube root (the default, also with opt == NULL). FP64
                                  always uses the cube root. */
  uint32_t dirichlet_bid_mask; /* hx_setup: bit b set (b = 1..31) = the faces with boundary id b
                                  are constrained (homogeneous Dirichlet data, Problems 2.1/2.2);
                                  bit 0 must be clear; ignored by hx_setup_lattice */
  int32_t reserved[6];         /* must be zero */
} hx_options;

/* Builds a context on a general hexahedral mesh for the residual and the linearised operator of
 * Section 2 (Problem 2.1: find u with r(v, u) = 0 for all v in H^1_0; Problem 2.2: Newton steps
 * with the directional derivative), discretised with Q_p Lagrange elements on the Gauss-Lobatto
 * points and (p+1)^3 Gauss points per cell (Section 6).
 * Numbers the nodes (first-touch order, header preamble), builds the int32 cell -> node map and
 * the node -> element-vector lists of the assembly, and stores J0^-1 and w det J0 of every Gauss
 * point (Section 5: J0 is part of every stored set), FP64 and FP32.
 * p in [1, 6]. opt may be NULL (defaults: no constraints). Errors: HX_E_ARG for NULL arrays, a
 * vertex id out of range or repeated within a cell, non-finite coordinates, g out of [1, 8],
 * bit 0 of the mask, more than 2^31 - 1 nodes or cells * (p+1)^3; HX_E_INVERTED if det J0 <= 0
 * at some Gauss point; HX_E_NOMEM, HX_E_HIP. On success *out owns device memory until hx_destroy,
 * among it the element-vector buffer of 24 * n_cells * (p+1)^3 bytes (rounded up to whole
 * workgroups of cells). The current HIP device at the time of the call is the context's device.
 * General-mesh contexts have no multigrid (hx_mg_create returns HX_E_UNSUPPORTED). */
hx_status hx_setup(const hx_mesh* mesh, int32_t p, const hx_material* mat,
                   const hx_options* opt, hx_ctx* out);

/* The same for a structured lattice (the fast case: nodes by index arithmetic, trilinear
 * geometry formed from the vertices at every Gauss point, or, with geom_nodes, stored per Gauss
 * point like hx_setup's). Checks det J0 > 0 at every Gauss point of every cell (HX_E_INVERTED
 * otherwise); HX_E_ARG also for geom_degree out of [1, 8] or > 1 without geom_nodes. */
hx_status hx_setup_lattice(const hx_lattice* mesh, int32_t p, const hx_material* mat,
                           const hx_options* opt, hx_ctx* out);

/* Frees every device and host resource of the context. NULL is accepted. */
hx_status hx_destroy(hx_ctx ctx);

/* 3 * n_nodes, or -1 for a NULL context. */
int64_t hx_num_dofs(hx_ctx ctx);
int64_t hx_num_nodes(hx_ctx ctx);
int64_t hx_num_cells(hx_ctx ctx);

/* Writes the node positions, HOST array [n_nodes][3]: the map of the node's owning cell at the
 * Gauss-Lobatto point of its local index; the owning cell is, on a lattice, the cell with lattice
 * index min(I / p, n_d - 1) per direction, on a general mesh the cell where the node is first
 * met. */
hx_status hx_node_coords(hx_ctx ctx, double* host_xyz);

/* Writes the constraint mask, HOST array [n_nodes] of 0/1. */
hx_status hx_constrained_mask(hx_ctx ctx, uint8_t* host_mask);

/* r = r~(u): material residual (Section 2) of the displacement u, FP64, device arrays
 * [3][n_nodes]; constrained rows are 0. u and r must not alias. */
hx_status hx_residual(hx_ctx ctx, const double* u, double* r, void* stream);

/* r = r~(u) evaluated over the spatial configuration (Section 2, the residual written with the
 * Kirchhoff stress and the spatial gradient: r_a = int_Omega0 tau : grad phi_a, grad = Grad F^-1,
 * with the Jacobian J_t = J0 + du/dxi of the deformed map). Equal to hx_residual in exact
 * arithmetic; same arguments and errors. */
hx_status hx_residual_spatial(hx_ctx ctx, const double* u, double* r, void* stream);

/* Linearisation update at u (Algorithm 1, "update quadrature point data"): stores the data of
 * the requested mode in the requested storage precision, in the configuration hx_autotune or
 * hx_set_tuning recorded for that mode and precision class (else the default one). The FP64 class (prec == HX_FP64) and
 * the FP32 class (the three FP32 values) are separate slots, so one context can hold an FP64
 * operator and an FP32 operator at once. For the fibre law in the FP32 NONE and FINV_J modes the
 * tension switches (I*_i > 1) are decided here in FP64 and kept (one byte per q-point), so that
 * rounding in the FP32 apply cannot flip them. Waits for the stream; returns HX_E_INVERTED if J <= 0
 * at some q-point and HX_E_NONFINITE on NaN/Inf. The data is kept even on those errors. */
hx_status hx_update_linearization(hx_ctx ctx, const double* u, hx_storage mode,
                                  hx_precision prec, void* stream);

/* dst = K~(u_k) du: the linearised operator of Problem 2.2 (Section 2, the directional derivative
 * (Grad v, Grad du S + F D_u S) of the residual), evaluated matrix-free by sum factorisation
 * (Section 6) from the data of the last linearisation update (Section 5, Algorithm 1), with the
 * slot selected by prec (HX_FP64: double du and dst; any FP32 value: float du and dst, data as
 * last stored in the FP32 slot). du and dst are device arrays [3][n_nodes] owned by the caller
 * and must not alias. Constrained rows: dst = du (identity rows and columns). Allocates nothing;
 * asynchronous on the stream. HX_E_STATE if that slot was never updated; HX_E_ARG for NULL or
 * aliasing pointers or an unknown precision; HX_E_HIP if a launch fails. */
hx_status hx_apply_tangent(hx_ctx ctx, const void* du, void* dst, hx_precision prec,
                           void* stream);

/* The same operator as hx_apply_tangent, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the element
 * vectors go to a static device buffer of the library (64 MiB per GPU, held until the process
 * ends) instead of the context's buffer, and the call allocates nothing, host or device. Limit:
 * 3 * n_cells * (p+1)^3 values of the apply's type (8 bytes for HX_FP64, 4 for the FP32 values;
 * n_cells rounded up to whole workgroups of cells) must fit in 64 MiB, else HX_E_ARG with a
 * message. The buffer is shared by every context on the
 * GPU and keeps the last call's contents (no part of it needs to start at zero): calls of this
 * entry point that overlap in time on one GPU (different streams, or host threads) race. */
hx_status hx_apply_tangent_noalloc(hx_ctx ctx, const void* du, void* dst, hx_precision prec,
                                   void* stream);

/* Autotuner of the storage strategy alone (Section 7.2: which strategy is fastest depends on the
 * hardware, degree and law and has to be measured), in the default configuration (the one the
 * multigrid levels use). For each of NONE, FINV_J, TANGENT and SPATIAL: updates the slot of prec
 * (HX_FP64, HX_FP32 or HX_FP32_BF16DATA) at u, applies once to warm up, then times `reps` applies (1..1000) of a
 * fixed direction with HIP events on the stream. Leaves the slot linearised in the fastest mode,
 * written to *best; ms_per_apply (HOST [4] or NULL) receives the mean time per apply of each mode
 * in that order. Allocates two temporary device vectors and waits for the stream. Errors of the
 * updates (HX_E_INVERTED, ...) are returned as they come. */
hx_status hx_autotune_storage(hx_ctx ctx, const double* u, hx_precision prec, int32_t reps,
                              hx_storage* best, double* ms_per_apply, void* stream);

/* One configuration timed by hx_autotune. */
typedef struct {
  hx_storage mode;
  int32_t variant;              /* cells-per-workgroup variant (0 default, 1 alternative) */
  int32_t cells_per_workgroup;  /* cells each workgroup of the variant processes */
  int32_t nontemporal;          /* 1: the stored data is loaded with the non-temporal hint */
  double ms;                    /* mean time per apply */
} hx_tune_entry;

/* Cells per workgroup of variant v (0 default, 1 alternative) of degree p, or -1. */
int32_t hx_cells_per_workgroup(int32_t p, int32_t variant);

/* Autotuner of the apply's configuration (Section 7.2: the fastest evaluation depends on the
 * hardware, degree and law and has to be measured): for each storage mode (NONE, FINV_J,
 * TANGENT, SPATIAL, SPATIAL_RECOMPUTE, SCALARS, TENSORS, SPATIAL_SCALARS), each cells-per-workgroup variant (two on a lattice of trilinear cells, the
 * default elsewhere; the stored data is laid out per variant) and, for the modes with stored
 * data, both load policies of that data (plain or non-temporal), updates the slot of prec
 * (HX_FP64 or HX_FP32) at u, applies once to warm up and times `reps` applies (1..1000) of a fixed
 * direction with HIP events on the stream (SPATIAL_RECOMPUTE is timed like NONE). Records the
 * fastest configuration of every mode as the
 * context's choice, which later hx_update_linearization calls of that mode and precision class use,
 * and leaves the slot linearised in the overall fastest one (*best). table (HOST, max_entries) or
 * NULL receives every timed configuration, *n_entries (or NULL) their number (at most 28).
 * Allocates two temporary device vectors and waits for the stream. */
hx_status hx_autotune(hx_ctx ctx, const double* u, hx_precision prec, int32_t reps,
                      hx_tune_entry* table, int32_t max_entries, int32_t* n_entries,
                      hx_tune_entry* best, void* stream);

/* Records a configuration for later updates of (precision class of prec, mode) without timing
 * (for a choice read back from a stored table): variant 0 or 1 (1 only on a lattice of trilinear
 * cells), nontemporal -1 (by the data size, the default), 0 or 1. HX_E_ARG otherwise. */
hx_status hx_set_tuning(hx_ctx ctx, hx_precision prec, hx_storage mode, int32_t variant,
                        int32_t nontemporal);

/* Bytes of per-q-point data held by a slot (0 before its first update). */
int64_t hx_linearization_bytes(hx_ctx ctx, hx_precision prec);

/* Host helper (Section 3): structure tensors and mean directions of the two fibre families from
 * the dispersion parameters (a, b), the mean in-plane angle phi (radians) and the local frame
 * E = rows E1 (circumferential), E2 (longitudinal), E3 (radial), row-major 3x3.
 * H33 = 1/(4b) - exp(-2b) / (sqrt(2 pi b) erf(sqrt(2b))), H11/H22 = (1 - H33)/2 (1 +- I1(a)/I0(a));
 * family 4: M1 = cos(phi) E1 + sin(phi) E2, M2 = -sin(phi) E1 + cos(phi) E2, M3 = E3;
 * family 6: the same with -phi; H_i = sum_k H_kk M_k (x) M_k. Outputs are host arrays. */
hx_status hx_fiber_structure(double a, double b, double phi, const double* E,
                             double* H4, double* H6, double* M4, double* M6);

/* Message for the last error on ctx (or of the last failed hx_setup when ctx is NULL). */
/* ------------------------------------------------------------------------------------------
 * p-multigrid preconditioner and Newton-Krylov solve (Section 6 and Algorithm 1).
 * ------------------------------------------------------------------------------------------ */
typedef struct hx_mg_s* hx_mg;

typedef struct {
  int32_t smoother_degree; /* Chebyshev degree of the Jacobi smoother on all but the coarsest
                              level (default 4) */
  int32_t coarse_degree;   /* Chebyshev degree of the approximate coarse solve (default 30) */
  double smoothing_range;  /* smoother interval [lambda_max / range, lambda_max] (default 100); the
                              coarse Chebyshev solve extends it down to the smallest Ritz value */
  int32_t eig_iters;       /* Lanczos (Jacobi-preconditioned CG) steps that estimate the extreme
                              eigenvalues of D^-1 A (default 20) */
  double eig_safety;       /* the estimate is multiplied by this factor (default 1.2) */
  hx_precision precision;  /* HX_FP32: levels apply in FP32 with FP32 stored data (the
                              mixed-precision preconditioner); HX_FP32_BF16DATA: FP32 vectors and
                              arithmetic with bfloat16 stored data of the level mode on all levels
                              but the coarsest (FP32); HX_FP32_FP16DATA: the same with binary16
                              stored tangents (the level mode is then TANGENT); HX_FP64:
                              everything in FP64 */
  int32_t use_graph;       /* 1: one V-cycle is captured into a HIP graph per update */
  hx_storage level_mode;   /* storage mode of the level operators inside the V-cycle: any of
                              the eight modes (default TANGENT) or AUTO (hx_autotune_storage on
                              each level at the first update; the choice is kept). The
                              smoother's D (diagonal or nodal blocks) always comes from a TANGENT
                              update of the level. */
  int32_t coarse_solver;   /* coarsest level: 0 = dense if it has at most 8192 DoFs, else
                              Chebyshev (default); 1 = Chebyshev of coarse_degree; 2 = dense
                              (HX_E_UNSUPPORTED above 32768 DoFs; 20 n^2 bytes of device memory). Dense: the level operator is
                              assembled by probing with 3 k_x k_y k_z coloured vectors (k_d >=
                              2p + 1 colours along direction d for a coarsest degree p, so that
                              no two coupled nodes share a colour), factored by Cholesky
                              (rocSOLVER, FP64) at each update and applied as its explicit
                              inverse. */
  int32_t fuse_smoother;   /* 1 (default): every Chebyshev step after the first, and the residual
                              before the restriction, run in the node kernel of the level apply
                              (no separate pass over the level vectors); 0: separate kernels */
  int32_t smoother_blocks; /* 0: point Jacobi (the inverse of the operator's diagonal); 1 (default):
                              nodal block Jacobi, the inverse of each node's 3x3 block of the
                              operator (the coupling of the three displacement components at the
                              node), formed from the stored tangent like the diagonal; Chebyshev
                              and the Lanczos bounds use the same D^-1 */
} hx_mg_options;

/* Fills *opt with the defaults listed above. */
hx_status hx_mg_default_options(hx_mg_options* opt);

/* Builds a V-cycle over contexts (levels[0] finest). Consecutive levels either share the
 * lattice with a strictly lower degree (polynomial transfer), or both have degree 1 and the
 * coarser lattice has half the cells in some directions and the same cells in the others
 * (transfer in lattice reference space: the coarse trilinear basis at the fine nodes); Dirichlet
 * faces and periodic directions must agree. The contexts stay owned by the caller and must
 * outlive the hierarchy.
 * opt may be NULL (defaults). Levels store the TANGENT mode in the multigrid precision; with
 * HX_FP64 the finest level's FP64 slot is shared with the outer operator. */
hx_status hx_mg_create(const hx_ctx* levels, int32_t n_levels, const hx_mg_options* opt,
                       hx_mg* out);
hx_status hx_mg_destroy(hx_mg mg);
const char* hx_mg_last_error(hx_mg mg);

/* Linearisation of every level at the finest-level displacement u (device FP64 [3][n_nodes]):
 * u is interpolated onto the coarser nodes, each level stores its tangent, the smoother's D^-1
 * (inverse diagonal or inverse nodal blocks) and a lambda_max estimate; the V-cycle is then
 * captured into a graph. Synchronous. */
hx_status hx_mg_update(hx_mg mg, const double* u, void* stream);

/* z = M^-1 r with one V-cycle (pre/post Chebyshev smoothing, restriction by the transpose of the
 * polynomial prolongation). r, z: device [3][n_nodes] of the finest level, float for HX_FP32
 * hierarchies and double for HX_FP64. */
hx_status hx_mg_vcycle(hx_mg mg, const void* r, void* z, void* stream);
int64_t hx_mg_vcycle_count(hx_mg mg);
/* Storage mode the level operators of `level` use (the autotuner's choice with AUTO), or -1 for
 * an invalid level or before the first update. */
int32_t hx_mg_level_mode(hx_mg mg, int32_t level);
double hx_mg_lambda_max(hx_mg mg, int32_t level);

/* Transfers between level `level` (fine) and level + 1 (coarse), device vectors [3][n_nodes]:
 *   kind 0: out_fine += P in_coarse   (P embeds the coarse polynomial space; every fine node is
 *           written once, by its owning cell, so the result is deterministic)
 *   kind 1: out_coarse += P^T in_fine (constrained coarse rows untouched; atomics)
 *   kind 2: out_coarse = the fine field in_fine evaluated at the coarse nodes (FP64 vectors)
 * Kinds 0 and 1 use the hierarchy's precision (float for HX_FP32). Asynchronous. */
hx_status hx_mg_transfer(hx_mg mg, int32_t level, int32_t kind, const void* in, void* out,
                         void* stream);

/* Copies the smoother's D^-1 of level `level` into out (hierarchy precision). Point Jacobi:
 * device [3][n_nodes], the inverse diagonal (1 on constrained rows). Nodal blocks: device
 * [6][n_nodes], the entries (00, 11, 22, 01, 02, 12) of the inverse of each node's symmetric 3x3
 * block (the identity at constrained nodes). */
hx_status hx_mg_inverse_diagonal(hx_mg mg, int32_t level, void* out, void* stream);

typedef struct {
  double newton_rel_tol;  /* per load step: stop when ||r|| <= max(abs, rel * ||r_0||) */
  double newton_abs_tol;
  int32_t max_newton;     /* Newton iterations per load step */
  double krylov_rel_tol;  /* inner flexible CG: ||b - K x|| <= rel * ||b|| */
  int32_t max_krylov;
  int32_t load_steps;     /* the external load is applied in this many equal increments */
  hx_storage outer_mode;  /* storage mode of the FP64 outer operator with an FP32 hierarchy:
                             NONE, FINV_J, TANGENT, SPATIAL or AUTO (hx_autotune at the first
                             linearisation: mode and configuration kept for the solve). An FP64
                             hierarchy shares the
                             finest level's data with the outer operator and ignores it. */
  int32_t verbose;        /* 1: one progress line per Newton iteration on stderr */
  int32_t predictor;      /* 1: each load step after the first starts from the previous converged
                             displacement plus the previous step's increment (secant predictor),
                             unless the new load's residual is not finite there; the step's
                             ||r_0|| is still that of the previous displacement. 0: Newton starts
                             from the previous displacement. */
} hx_newton_opts;

typedef struct {
  int32_t newton_iters, krylov_iters, vcycles, load_steps_done;
  double initial_residual, final_residual, seconds;
  int32_t outer_mode;     /* storage mode the outer FP64 operator used */
} hx_newton_report;

/* Solves r(u) = f_ext (Problem 2.1 with a dead load) by Newton's method with load stepping
 * (Algorithm 1), each step by flexible CG in FP64 on the finest FP64 operator preconditioned by
 * one V-cycle of mg. The CG scalars stay on the device: each iteration (apply, inner products,
 * updates, V-cycle) is one graph launch when mg uses graphs, and the host reads the iteration
 * count and stop flag every 4 iterations (iterations after the stopping one leave the iterate
 * unchanged; report->vcycles counts the V-cycles run, report->krylov_iters the counted ones).
 * u: device FP64 [3][n_nodes], in/out (its constrained entries are the
 * homogeneous Dirichlet data). f_ext: device FP64 [3][n_nodes] or NULL. Synchronous; returns
 * HX_E_NOT_CONVERGED if a load step does not reach its tolerance (u holds the last iterate). */
hx_status hx_newton_solve(hx_mg mg, double* u, const double* f_ext, const hx_newton_opts* opt,
                          hx_newton_report* report, void* stream);

/* Host helper: dead-load pressure (Section 2, Neumann term of the residual):
 * f_(c,a) = -p int phi_a N_c dA with N the outward unit normal of the reference body, over the
 * lattice boundary face `face` (0..5 = -x,+x,-y,+y,-z,+z) of a lattice context, or over every
 * cell face with boundary id `face` (1..255) of a general-mesh context; (p+1)^2 Gauss points per
 * cell face of the cell's map (trilinear or curved). f: HOST array [3][n_nodes], overwritten.
 * HX_E_ARG for a face of a periodic direction or an id out of range. */
hx_status hx_surface_load(hx_ctx ctx, int32_t face, double pressure, double* f);

/* ------------------------------------------------------------------------------------------
 * Forward-stability study of the q-point functions (Section 7.1).
 * ------------------------------------------------------------------------------------------ */
/* For n displacement gradients H and directions G (device FP64 arrays [n][9], row-major 3x3),
 * evaluates the first Piola-Kirchhoff stress P(I + H) and its directional derivative
 * P'(H)[G] = G S + F D_u S[G] of the law in *mat (uniform fibre tensors), in the arithmetic of
 * prec (HX_FP64, or HX_FP32 with H and G rounded to FP32 first):
 *   form 0: the stable forms of Section 4, i.e. the functions the operator kernels evaluate (J - 1
 *           from the invariants of H, E = (H + H^T + H^T H)/2, C^-1 via F^-1, log1p);
 *   form 1: the standard forms of Section 3 (C = F^T F, J = det F, C^-1 by inverting C, ln J and
 *           J^-2/3 from J, E = (C - I)/2).
 * jpow_iters: FP32 J^-2/3 by Algorithm 2 with this many steps (0: cube root), as in hx_options;
 * FP32 exp is the hardware base-2 exponential in both forms. P, dP: device FP64 [n][9].
 * Asynchronous on the stream; HX_E_ARG for invalid arguments. */
hx_status hx_qpoint_eval(const hx_material* mat, int32_t form, hx_precision prec, int32_t jpow_iters,
                         int64_t n, const double* H, const double* G, double* P, double* dP,
                         void* stream);

/* ------------------------------------------------------------------------------------------
 * Device bandwidth and issue-rate probes (not part of the method).
 * ------------------------------------------------------------------------------------------ */
/* STREAM "triad" (McCalpin's memory benchmark): a[i] = b[i] + s * c[i] for 0 <= i < n, FP64
 * device arrays owned by the caller, each 16-byte aligned and not overlapping; moves 24 n bytes.
 * It states the HBM rate a plain streaming kernel sustains on the device, against which the
 * operator's bytes per apply can be read. Asynchronous on the stream; HX_E_ARG for n < 0, a NULL
 * or misaligned array, or n beyond 2^39. */
hx_status hx_stream_triad(int64_t n, double* a, const double* b, const double* c, double s,
                          void* stream);

/* FP64 issue-rate probe: 2048 workgroups of 256 threads, each thread running iters iterations of
 * independent dependency chains. kind 0: vector fused multiply-adds, 8192 flops per wave and
 * iteration (8 chains x 8 steps x 64 lanes x 2); kind 1: 16x16x4 FP64 matrix instructions, the
 * same 8192 flops per wave and iteration (4 chains x 2048); kind 2: both in every wave (16384).
 * Flops per call: 2048 x 4 waves x iters x (8192, 8192 or 16384). Timed, it states the FP64 rate
 * each unit sustains alone and whether the two add up when a wave issues to both, the basis for
 * keeping the 1D contractions of the sum factorisation on the vector units. out: device FP64
 * [2048 * 256] owned by the caller, 8-byte aligned, receives each thread's sum of its chains.
 * Lane l of a wave supplies 1e-3 l to A and 1e-3 to B of every matrix instruction, so each one adds
 * 16 x 1e-3 x sum_l 1e-3 l = 0.032256 to the sum of the wave's accumulator entries whatever the
 * lane layout: over the 64 threads of a wave the matrix chains sum to iters x 0.129024.
 * Asynchronous on the stream; HX_E_ARG for kind outside [0, 2], iters outside [1, 10^6], or a
 * NULL or misaligned out. */
hx_status hx_fp64_pipe_probe(int32_t kind, int64_t iters, double* out, void* stream);

const char* hx_last_error(hx_ctx ctx);
const char* hx_status_string(hx_status s);

#ifdef __cplusplus
}
#endif

#endif /* HX_H */
