/*
 * sasa.h -- C-ABI of the MI355X (gfx950) library for exact analytic solvent
 * accessible surface area with analytic Cartesian derivatives.
 *
 * The library implements the dSASA method (Cao, Hummel, Wang, Simmerling,
 * Coutsias, arXiv 2401.10462):
 *   - every atom is a weighted point (p_i, d_i), d_i = (r_i + probe)^2
 *     (Methods, "dSASA: an analytical method for SASA");
 *   - the dual complex of the weighted Delaunay tetrahedrization restricted to
 *     the balls (Steps 1 and 2; the Laguerre-intersection cells L_i cap B_i);
 *   - its interior / exterior classification (GPU section, extraction of
 *     exterior simplices);
 *   - the per-atom inclusion-exclusion area of Eq. 1 with the vertex, edge and
 *     triangle terms of Eqs. 3, 4 and 6, and the derivatives of Eqs. 2, 5, 7;
 *   - the volumes of the same cells, the molecular-volume gradient and the
 *     per-atom volume VJP (sasa_volume, sasa_volume_backward; the
 *     Discussion's extension to volumes), and the surface's integrated mean
 *     and Gaussian curvatures (sasa_curvature; the Introduction's);
 *   - the paper's sort-based extraction of unique triangles, edges and
 *     vertices, for comparison (sasa_triangles_by_sort,
 *     sasa_edges_vertices_by_sort).
 *
 * Units: lengths in Angstrom, areas in A^2, volumes in A^3, gradients in A^2/A.
 *
 * Memory.  Every data pointer is either host or device memory, as the `mem`
 * argument says; all pointers of one call live in the same space.  The caller
 * owns every input and output buffer; the library neither frees nor keeps them
 * past the call.  Device pointers are used on `hip_stream` (a hipStream_t, or
 * NULL for the default stream); host pointers are staged through the context's
 * device buffers and the call returns after the results are back on the host.
 *
 * Threads.  A context is not thread-safe: use one context per host thread or
 * per stream slot.  Distinct contexts are independent.
 *
 * Errors.  Every call returns SASA_OK (0) or a negative code; no C++
 * exception crosses this boundary.  sasa_strerror() names the code and
 * sasa_last_error() gives the context's last message.
 */
#ifndef SASA_H
#define SASA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SASA_OK = 0,
  SASA_E_INVAL = -1,    /* bad argument: n < 0, NaN/Inf coordinate, radius <= 0, probe < 0, NULL pointer,
                           two atoms of one molecule with the same centre and the same radius */
  SASA_E_NOMEM = -2,    /* device allocation failed */
  SASA_E_DEVICE = -3,   /* HIP runtime error; the context should be destroyed */
  SASA_E_STATE = -4,    /* backward / export without a preceding compute on this context */
  SASA_E_CAPACITY = -5  /* an atom has more overlapping neighbours (512) or cell vertices (128) than
                           the kernels hold (sasa_capacity), or more than 64 K-neighbours or 160
                           K-tetrahedra or exterior K-triangles */
};

typedef enum { SASA_FP64 = 0, SASA_MIXED = 1 } sasa_precision;
/* SASA_FP64 : every step in double precision.
 * SASA_MIXED: the tetrahedrization predicates and all accumulations in double,
 *             the per-simplex area terms and their derivatives in single
 *             precision (Eqs. 3-7 evaluated in float). */

typedef enum { SASA_MEM_HOST = 0, SASA_MEM_DEVICE = 1 } sasa_mem;

enum {
  SASA_FLAG_ASYNC = 1u, /* device-pointer calls return without synchronising the stream; capacity
                           overflow and input errors are then reported by the next sasa_diagnostics */
  SASA_FLAG_TIMING = 2u, /* record HIP events around every stage of a call (stage times in sasa_diag) */
  SASA_FLAG_FRAMES = 4u, /* consecutive calls are frames of one trajectory (same atoms, small moves).
                            The context keeps each atom's power cell (facet neighbours and vertices
                            as plane triples) from the previous call of the same atom count.  A kept
                            cell whose vertices, solved afresh, lie inside every neighbour plane
                            they are not on is the new cell and is not clipped again; any other
                            cell is clipped with the kept facets first.  The cells, the complex and
                            every result are the same as without the flag (up to the summation
                            order of the terms; near-degenerate decisions aside, which sasa_diag
                            counts); a call with another atom count starts without.  Costs 516
                            bytes of device memory per atom. */
  SASA_FLAG_INCREMENTAL = 8u /* consecutive one-molecule calls (sasa_compute, sasa_compute_forces) of
                                the same atom count and probe rebuild only the stars of atoms whose
                                star can have changed: an atom that moved (position or radius,
                                compared bit for bit) and every atom overlapping such an atom at its
                                old or its new place.  The other atoms keep the star, the area and,
                                when this call and the previous one both ask for the gradient, the
                                gradient blocks of the previous call; the gradient sums are always
                                redone.  Every result equals that of a context without the flag bit
                                for bit (a star depends only on the atom and its overlapping
                                neighbours; with SASA_FLAG_FRAMES too, up to the summation order
                                of the terms, as for that flag alone).  When more than a quarter of the atoms moved, every
                                star is rebuilt.  A batch, a failed call or another atom count or
                                probe starts afresh.  Costs 77 bytes of device memory per atom. */
};

/* Opaque context: device buffers, the complex kept from the last compute and
 * the diagnostics of the last call.  Created by sasa_create, freed by
 * sasa_destroy; one per host thread or stream slot. */
typedef struct sasa_context sasa_context;

/* Context options.  There is no tolerance to set: every decision that builds
 * the complex is the exact sign of its predicate, with a symbolic tie rule, so
 * no tangency epsilon exists; the per-atom capacities are fixed
 * (sasa_capacity). */
typedef struct {
  int32_t device;       /* HIP device ordinal */
  int32_t precision;    /* sasa_precision */
  int64_t max_atoms;    /* optional size hint for the first allocation (0: grow on demand); the buffers are
                           sized for max_atoms atoms in up to min(max_atoms, 8192) molecules per call, so
                           calls within that size never reallocate (which would wait for the device) */
  uint32_t flags;       /* SASA_FLAG_* */
  uint32_t reserved;    /* must be 0 */
} sasa_options;

/*
 * Create a context on opt->device (NULL opt: device 0, FP64, synchronous) and
 * store it in *ctx_out (NULL on failure).  SASA_E_INVAL for a bad precision,
 * unknown flag bits or a non-zero reserved field, SASA_E_DEVICE for a missing
 * device, SASA_E_NOMEM if the max_atoms pre-allocation fails.
 */
int sasa_create(const sasa_options* opt, sasa_context** ctx_out);
/* Wait for the context's device work and free it (NULL is ignored). */
void sasa_destroy(sasa_context* ctx);

/*
 * Per-atom SASA of one molecule and the gradient of the molecular SASA
 * (Methods, "dSASA: an analytical method for SASA"): the dual complex K of the
 * weighted points (Steps 1 and 2), its exterior simplices, the area of Eq. 1
 * with the terms of Eqs. 3, 4 and 6, and its gradient, Eq. 2 with Eqs. 5 and 7.
 *   n       number of atoms (0 is allowed and returns at once; at most 100,000,000,
 *           else SASA_E_INVAL)
 *   xyz     n*3 doubles, row-major (x0 y0 z0 x1 ...)
 *   radii   n doubles, van der Waals radii > 0
 *   probe   probe radius >= 0 (1.4 A in the paper)
 *   area    n doubles out: A_i, the exposed area of sphere i (0 for buried or
 *           hidden atoms); may be NULL
 *   dA_dx   n*3 doubles out: d(sum_i A_i)/dp_m; may be NULL
 * The context keeps the dual complex K of this call (indices only) for
 * sasa_backward and sasa_complex_export.  Errors: SASA_E_INVAL (see the codes),
 * SASA_E_CAPACITY (an atom beyond sasa_capacity), SASA_E_NOMEM (buffers could
 * not grow), SASA_E_DEVICE; a failed call keeps no complex.
 */
int sasa_compute(sasa_context* ctx, int64_t n, const double* xyz, const double* radii, double probe,
                 double* area, double* dA_dx, int32_t mem, void* hip_stream);

/*
 * Many molecules in one launch sequence.  Molecule k holds atoms
 * offsets[k] .. offsets[k+1]-1 of xyz / radii / area / dA_dx (offsets has
 * nmol+1 non-decreasing entries, offsets[0] = 0).  Atoms of different molecules
 * never interact; every per-atom result equals the one sasa_compute gives for
 * that molecule alone.
 */
int sasa_compute_batch(sasa_context* ctx, int32_t nmol, const int64_t* offsets, const double* xyz,
                       const double* radii, double probe, double* area, double* dA_dx,
                       int32_t mem, void* hip_stream);

/*
 * Non-polar solvation forces: the nonpolar energy is gamma * SASA with one
 * surface tension gamma for all atoms (Methods, "Theory and estimations for
 * nonpolar solvation"), so F_m = -gamma d(sum_i A_i)/dp_m.  Same as
 * sasa_compute with dA_dx scaled by -gamma in the gradient kernel.
 *   gamma   surface tension (e.g. 0.005 kcal/mol/A^2); forces in its energy unit per A
 *   forces  n*3 doubles out (required)
 */
int sasa_compute_forces(sasa_context* ctx, int64_t n, const double* xyz, const double* radii, double probe,
                        double gamma, double* area, double* forces, int32_t mem, void* hip_stream);

/*
 * Vector-Jacobian product of the last compute through the derivatives of
 * Eq. 2 (Eqs. 5 and 7 for the edge and triangle terms):
 * dL_dx[m] = sum_i dL_dA[i] dA_i/dp_m (n doubles in, n*3 doubles out).  Recomputes the simplex geometry from the kept complex and the
 * coordinates of that compute; the coordinates are the context's own copy, so the
 * caller's input buffers may have changed.  SASA_E_STATE without a kept compute.
 */
int sasa_backward(sasa_context* ctx, const double* dL_dA, double* dL_dx, int32_t mem, void* hip_stream);

/*
 * Volumes of the last compute (the Discussion's extension of the method to
 * volumes and their derivatives on the same Laguerre intersection cells):
 *   volume[i] = volume of B_i ∩ L_i (A^3; sum = volume of the union of the balls)
 *   dV_dx[m]  = d(sum_i volume[i]) / dp_m (n*3 doubles, A^2)
 * From the kept complex and that compute's coordinates: 3 V_i = R_i A_i +
 * sum_j h_ij F_ij over the flat faces of the cell, each face area by
 * inclusion-exclusion over the K-triangles and K-tetrahedra at its edge, and
 * dV/dp_i = -sum_j F_ij (p_j - p_i) / |p_j - p_i|.  Always FP64 (the areas are
 * recomputed in FP64 whatever the context's precision).  The caller owns both
 * output buffers (host or device per mem); the gradient is that of the
 * molecular volume, not a per-atom Jacobian.  SASA_E_STATE without a kept
 * compute, SASA_E_INVAL for NULL outputs.
 */
int sasa_volume(sasa_context* ctx, double* volume, double* dV_dx, int32_t mem, void* hip_stream);

/*
 * Vector-Jacobian product of the per-atom volumes of the last compute:
 *   dL_dx[m] = sum_i dL_dV[i] dV_i/dp_m   (n*3 doubles, FP64)
 * Moving p_j moves only the face (i, j) of cell i and moving p_i moves its
 * sphere and all its faces, so the product comes from each atom's own faces:
 *   dL_dx[m] = sum_j F_mj [(u_m - u_j)(cbar_mj - p_m) - u_m (p_j - p_m)] / d_mj
 * with u = dL_dV, F the face areas and cbar their centroids (first moments
 * by inclusion-exclusion over the K-triangles and K-tetrahedra, as the areas).
 * dL_dV = 1 gives the molecular-volume gradient of sasa_volume.  Buffers and
 * errors as sasa_backward.
 */
int sasa_volume_backward(sasa_context* ctx, const double* dL_dV, double* dL_dx, int32_t mem, void* hip_stream);

/*
 * Curvature measures of the last compute's solvent accessible surface (the
 * Introduction extends the method from areas to volumes and to mean and
 * Gaussian curvatures; the paper gives no formula, these are the standard
 * ones for the piecewise smooth boundary of a union of balls):
 *   mean[i]  n doubles out (host or device per mem; may be NULL): the
 *            integrated mean curvature of atom i's share of the surface (A),
 *            C_i = A_i / R_i - 1/4 sum_j L_ij gamma_ij, with L_ij the exposed
 *            length of the circle where spheres i and j meet (a concave
 *            crease) and gamma_ij the angle between their outward normals
 *            along it; sum_i C_i is the integral of (k1 + k2) / 2 over the
 *            surface, creases included.  The arcs come from the kept complex
 *            by the inclusion-exclusion of sasa_volume; FP64 in both
 *            precisions.
 *   euler    host int64 out (may be NULL): V - E + T - Q of K, the Euler
 *            characteristic of the union of the balls (K is homotopy
 *            equivalent to it), so the integrated Gaussian curvature of the
 *            surface is 4 pi * euler (Gauss-Bonnet).  At exact ties where
 *            more than four cells meet at one point and the stars split the
 *            point differently (a regular octahedron of equal balls), the
 *            counts are not those of one complex and euler can be off; the
 *            per-atom measures (areas, volumes, mean curvature) are not
 *            affected.
 * Synchronous.  SASA_E_STATE without a kept compute, SASA_E_INVAL for a bad
 * mem or both outputs NULL.  Uses the input staging buffers of the context
 * as scratch (the last compute's results and complex stay).
 */
int sasa_curvature(sasa_context* ctx, double* mean, int64_t* euler, int32_t mem, void* hip_stream);

/*
 * Vector-Jacobian product of the per-atom integrated mean curvature of the
 * last compute (sasa_curvature; the Introduction's extension to curvatures):
 *   dL_dx[m] = sum_i dL_dC[i] dC_i/dp_m   (n doubles in, n*3 doubles out, FP64)
 * C_i = A_i / R_i + C_i', where C_i' = -1/4 sum_j L_ij gamma_ij is the crease
 * part.  The first term is the area VJP (Eq. 2) with weights dL_dC[i] / R_i.
 * The exposed share of crease circle ij, theta / 2 pi, is the edge and triangle
 * part of the same inclusion-exclusion as Eq. 1: Phi_ij - sum_t c_t 2
 * phi_ij(T_x).  So C_i' is the Eq. 1 edge and triangle sum with
 * W = (pi / 2) rho gamma in place of the cap areas and no vertex term, and its
 * gradient is Eq. 2 with the same substitution; dW/dd = (pi / 2)
 * (gamma drho/dd + 1).  Buffers and errors as sasa_backward.  Rewrites the
 * context's gradient blocks, so an incremental context starts afresh
 * afterwards.
 */
int sasa_curvature_backward(sasa_context* ctx, const double* dL_dC, double* dL_dx, int32_t mem, void* hip_stream);

/*
 * Sizes of the kept complex K of the last compute (Methods, Steps 1 and 2)
 * and of its exterior part (GPU section, extraction of exterior simplices):
 * counts[0..7] = vertices in K, edges, triangles, tetrahedra, exterior
 * vertices, exterior edges, exterior triangles, atoms.  SASA_E_STATE without
 * a kept compute.
 */
int sasa_complex_counts(sasa_context* ctx, int64_t counts[8]);

/*
 * The unique K-triangles of the last compute and their n_t, found the way the
 * paper's GPU section extracts them (for comparison with the star kernel,
 * which decides n_t per atom): the four faces of every K-tetrahedron are
 * listed, radix-sorted as 63-bit keys and run-length counted (n_t = 1 or 2);
 * K-triangles on no K-tetrahedron (n_t = 0) come from the stars.
 *   tris      3*capacity int32 out (host): ascending atom ids per triangle;
 *             the tetrahedron faces in lexicographic order, then the n_t = 0
 *             triangles
 *   tri_ntet  capacity uint8 out (host): n_t
 *   count     out: number of triangles (= sasa_complex_counts()[2]); with tris
 *             or tri_ntet NULL only the count (and ms) is returned
 *   ms        out (may be NULL): GPU time of the extraction (emit, sort,
 *             count, unpack) on the null stream
 * Allocates its work buffers on first use.  SASA_E_CAPACITY if count >
 * capacity, SASA_E_INVAL for 2^21 atoms or more, SASA_E_STATE without a kept
 * compute.
 */
int sasa_triangles_by_sort(sasa_context* ctx, int32_t* tris, uint8_t* tri_ntet, int64_t capacity, int64_t* count,
                           float* ms);

/*
 * The other half of that extraction (GPU section, extraction of exterior
 * simplices): the unique K-edges and K-vertices of the last compute and their
 * exterior flags, found by the same lexicographic sorts one dimension down.
 * Every unique triangle (sasa_triangles_by_sort) lists its three edges with its
 * exterior flag (n_t <= 1), and every K-edge is listed once more from the star
 * of its lower atom; the candidates are radix-sorted and each run's flags
 * combined: an edge is exterior iff it lies on an exterior triangle or on
 * none.  Every unique edge then lists its two atoms with its flag, every atom
 * in K once more, and a vertex is exterior iff it has an exterior edge or none.
 * For comparison with the star kernel's per-atom classification.
 *   edges      2*edge_capacity int32 out (host): ascending atom ids per edge,
 *              in lexicographic order
 *   edge_ext   edge_capacity uint8 out (host): 1 if the edge is exterior
 *   edge_count out: number of K-edges (= sasa_complex_counts()[1])
 *   verts      vert_capacity int32 out (host): the atoms in K, ascending
 *   vert_ext   vert_capacity uint8 out (host): 1 if the vertex is exterior
 *   vert_count out: number of K-vertices (= sasa_complex_counts()[0])
 *   ms         out (may be NULL): GPU time of the whole extraction (triangles,
 *              edges and vertices) on the null stream
 * With all four output arrays NULL only the counts (and ms) are returned; give
 * all four or none.  Allocates its work buffers on first use.
 * SASA_E_CAPACITY if a count exceeds its capacity, SASA_E_INVAL for 2^21 atoms
 * or more, SASA_E_STATE without a kept compute, SASA_E_DEVICE if the sorted
 * counts disagree with the complex's counters.
 */
int sasa_edges_vertices_by_sort(sasa_context* ctx, int32_t* edges, uint8_t* edge_ext, int64_t edge_capacity,
                                int64_t* edge_count, int32_t* verts, uint8_t* vert_ext, int64_t vert_capacity,
                                int64_t* vert_count, float* ms);

/*
 * Copy the kept complex K of the last compute (Methods, Steps 1 and 2; the
 * exterior flags and n_t of the GPU section's classification) to host arrays
 * sized by sasa_complex_counts, in canonical order: each simplex once, its
 * atom indices ascending (batch-global), the tuples sorted lexicographically.
 *   edges (E*2), tris (T*3), tri_ntet (T: number of K-tetrahedra on the
 *   triangle, in the order of tris), tets (Q*4), vert_flags (n: bit0 in K,
 *   bit1 exterior).
 * Any pointer may be NULL to skip that list.  Synchronous (null stream).
 * SASA_E_STATE without a kept compute, SASA_E_NOMEM, SASA_E_DEVICE.
 */
int sasa_complex_export(sasa_context* ctx, int32_t* edges, int32_t* tris, uint8_t* tri_ntet, int32_t* tets,
                        uint8_t* vert_flags);

/*
 * Diagnostics of the last call (not an operation of the method: sizes, work
 * counts and errors of the kernels; fills as many bytes as given, up to the
 * struct, so an older, shorter struct stays valid).
 * The size and work counts of a compute (and sasa_complex_counts) are summed
 * from per-atom records on the device the first time they are asked for after
 * that compute: one small launch on the call's stream and a synchronisation,
 * which a compute itself does not spend.
 */
typedef struct {
  int64_t n_atoms;
  int64_t n_mol;
  int64_t max_neighbours;     /* largest overlapping-neighbour count of any atom */
  int64_t max_cell_vertices;  /* largest polytope size met while clipping */
  int64_t near_ties;          /* clipping side tests within their FP64 rounding bound, decided exactly */
  int64_t lost_pairs;         /* K-edges seen from one side only (near-degenerate inputs) */
  int64_t capacity_retries;   /* always 0: the per-atom capacities are fixed, and an atom beyond
                                 them ends the call with SASA_E_CAPACITY (no retry) */
  int64_t input_errors;       /* NaN/Inf coordinates, radii <= 0 or equal coincident atoms seen by the device */
  int64_t overflow;           /* atoms beyond the kernels' neighbour / vertex capacity */
  double ms_total;            /* wall time of the last synchronous call */
  /* stage times of the last call (SASA_FLAG_TIMING; HIP events on the call's stream) */
  double ms_cells;            /* weights, per-molecule cell grid, scan, scatter */
  double ms_star;             /* per-atom power-cell clipping and the star in K (fast pass) */
  double ms_star_wide;        /* the star's second pass (large cells; exact side tests) */
  double ms_terms;            /* Eq. 1 area terms (and gradient blocks) */
  double ms_gather;           /* segmented gradient sums */
  /* algorithmic work of the last call's star kernel */
  int64_t plane_tests;        /* (vertex, plane) side tests while clipping */
  int64_t new_vertices;       /* cell vertices created (three-plane solves) */
  int64_t candidates;         /* neighbour-candidate distance tests */
  int64_t planes_used;        /* radical planes visited by the clipping loops (sum over atoms) */
  int64_t max_planes_used;    /* ... largest for one atom */
  int64_t atoms_over_64_planes; /* atoms whose clipping visited more than 64 planes */
  int64_t reused_cells;       /* SASA_FLAG_FRAMES: atoms whose previous-frame cell was verified and kept */
  int64_t second_pass_atoms;  /* atoms the fast star pass left to the second pass (cells past 64
                                 vertices, or a side test within its rounding bound) */
  int64_t moved_atoms;        /* SASA_FLAG_INCREMENTAL: atoms whose position or radius changed since
                                 the previous call (all atoms when the call started afresh) */
  int64_t skipped_atoms;      /* SASA_FLAG_INCREMENTAL: atoms whose star was kept from the previous call */
} sasa_diag;
int sasa_diagnostics(sasa_context* ctx, sasa_diag* out, int64_t size);

/*
 * Error status of the last call: for a SASA_FLAG_ASYNC call, waits for its
 * stream and returns SASA_E_CAPACITY / SASA_E_INVAL as sasa_diagnostics would,
 * without summing the diagnostics counts; SASA_OK otherwise.
 */
int sasa_status(sasa_context* ctx);

/*
 * Device bytes a context needs for a call of n atoms in total (all molecules of
 * a batch): the admission model of a server that packs requests by HBM
 * footprint.  The same for both precisions (the buffers do not depend on
 * them); SASA_FLAG_FRAMES adds 516 and SASA_FLAG_INCREMENTAL 77 bytes per atom,
 * which this figure leaves out.  Host-pointer calls add no device memory
 * beyond it.  SASA_E_INVAL for n < 0 or a NULL bytes.
 */
int sasa_footprint(int64_t n, int64_t* bytes);

/* Fixed per-atom kernel capacities (those of the second pass, which takes every atom beyond the
 * first's): [0] overlapping neighbours, [1] cell vertices. */
void sasa_capacity(int64_t caps[2]);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): sasa_compute
 * of one molecule of at most SASA_NOALLOC_MAX_ATOMS atoms, all work space in
 * one fixed 16 MiB array of the library's device code (each GPU the library
 * runs on holds it until the process ends).  No context; nothing is kept, so
 * there is no sasa_backward or export afterwards.
 *   device      HIP ordinal (made current for the call, restored after)
 *   xyz, radii  device pointers, as in sasa_compute
 *   area        n doubles out (device) or NULL;  dA_dx n*3 doubles out (device) or NULL
 *   precision   SASA_FP64 or SASA_MIXED;  hip_stream: the caller's stream (NULL: default)
 * Synchronous: waits for the stream and returns SASA_E_INVAL (as sasa_compute,
 * also for n > SASA_NOALLOC_MAX_ATOMS), SASA_E_CAPACITY or SASA_E_DEVICE.  It
 * calls no allocator.  Every call on one GPU uses the same array: calls that
 * overlap on one GPU (other threads, other streams) race and must be
 * serialised by the caller.
 */
#define SASA_NOALLOC_MAX_ATOMS 4096
int sasa_compute_noalloc(int device, int64_t n, const double* xyz, const double* radii, double probe,
                         double* area, double* dA_dx, int precision, void* hip_stream);

const char* sasa_strerror(int32_t code);
const char* sasa_last_error(sasa_context* ctx);

#ifdef __cplusplus
}
#endif
#endif
