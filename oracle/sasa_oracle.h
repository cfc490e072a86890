/*
 * sasa_oracle.h -- plain FP64 CPU reference of the dSASA hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load or call this library; the
 * product path never does.  It shares no code with the HIP library.
 *
 * What it computes (Cao, Hummel, Wang, Simmerling, Coutsias, "Exact analytical
 * algorithm for solvent accessible surface area and derivatives in implicit
 * solvent molecular simulations on GPUs", arXiv 2401.10462):
 *   - weighted points (p_i, w_i), w_i = (r_i + probe)^2       (Methods, dSASA)
 *   - the alpha = 0 dual complex K of the weighted Delaunay tetrahedrization,
 *     decided simplex by simplex from its definition: the restricted
 *     Laguerre-intersection cells L_i cap B_i of the simplex's atoms share a
 *     point                                          (Steps 1-2, Laguerre cell),
 *     by exact predicates with ties broken by a symbolic perturbation of the
 *     weights (predicates.h), so that co-spherical inputs get one consistent
 *     complex
 *   - the interior / exterior classification of K           (GPU section,
 *     "Extraction of exterior simplices")
 *   - per-atom SASA by the inclusion-exclusion sum, Eq. 1, with the vertex,
 *     edge and triangle terms of Eqs. 3, 4 and 6
 *   - per-atom Cartesian derivatives, Eq. 2 (with Eqs. 3, 5, 7), evaluated by
 *     forward-mode dual numbers over the same formulas with K held fixed.
 *
 * All lengths in Angstrom, areas in A^2, gradients in A^2/A.
 * Every function returns / fills plain arrays owned by the caller.
 */
#ifndef SASA_ORACLE_H
#define SASA_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Opaque result of one oracle run. */
typedef struct oracle_result oracle_result;

/* Run the whole reference on n atoms (xyz: n*3 row-major, radii: n van der
 * Waals radii > 0, probe >= 0).  Returns NULL on invalid input, which
 * includes two atoms with the same centre and the same radius. */
oracle_result* oracle_run(int64_t n, const double* xyz, const double* radii, double probe);
void oracle_free(oracle_result* r);

/* Counts.  what: 0 = vertices in K, 1 = edges in K, 2 = triangles in K,
 * 3 = tetrahedra in K, 4 = exterior vertices, 5 = exterior edges,
 * 6 = exterior triangles, 7 = non-zero (atom, atom) blocks of the Jacobian,
 * 8 = predicates the FP64 filter left to exact arithmetic,
 * 9 = exact ties decided by the symbolic perturbation of the weights,
 * 10 = candidate simplices with coplanar / collinear / coincident centres
 * (never in K) skipped. */
int64_t oracle_count(const oracle_result* r, int what);

/* Per-atom SASA A_i (n values). */
void oracle_area(const oracle_result* r, double* area);
/* d(sum_i A_i)/dp_m (n*3 values). */
void oracle_dadx(const oracle_result* r, double* g);
/* sum_i u_i dA_i/dp_m (n*3 values). */
void oracle_vjp(const oracle_result* r, const double* u, double* g);
/* Sparse Jacobian blocks J[i][m] = dA_i/dp_m, COO over count(7) entries. */
void oracle_jacobian(const oracle_result* r, int32_t* rows, int32_t* cols, double* vals3);
/* K, every simplex once with ascending vertex indices, lexicographically sorted. */
void oracle_vertices(const oracle_result* r, uint8_t* in_k, uint8_t* exterior);
void oracle_edges(const oracle_result* r, int32_t* e2, uint8_t* exterior);
void oracle_triangles(const oracle_result* r, int32_t* t3, uint8_t* n_tet, uint8_t* exterior);
void oracle_tetrahedra(const oracle_result* r, int32_t* t4);

/* Single formula pieces, exposed so that tests can pin each one to a closed form.
 * Points are 3-vectors.  Results are the normalised quantities of the paper. */
double oracle_solid_angle(const double* pi, const double* pj, const double* pk, const double* pl);
double oracle_dihedral(const double* pi, const double* pj, const double* pk, const double* pl);
double oracle_cap_area(const double* pi, double Ri, const double* pj, double Rj);
double oracle_triple_term(const double* pi, double Ri, const double* pj, double Rj,
                          const double* pk, double Rk);

#ifdef __cplusplus
}
#endif
#endif
