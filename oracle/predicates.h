// predicates.h -- exact, symbolically perturbed predicates of the oracle's
// dual-complex decisions (TEST INFRASTRUCTURE ONLY, see sasa_oracle.h).
//
// Every membership decision of the alpha = 0 dual complex K (Methods, Steps
// 1-2: the restricted Laguerre cells of a simplex's atoms share a point inside
// the balls) reduces to the sign of a polynomial in the input doubles:
//   * orientation of four centres and collinearity of three (positions only);
//   * the "size" of a simplex: the power pi_i(y) of its orthocentre y, the
//     point of its Laguerre face closest to the atoms' centres;
//   * the "side" of another atom m at that orthocentre: pi_m(y) - pi_i(y).
// Each polynomial is first evaluated in FP64 together with a running bound on
// its rounding error; when the bound does not separate the value from zero
// it is evaluated again in exact dyadic (big-integer times power of two)
// arithmetic from the same doubles.
//
// The weighted Delaunay tetrahedrization is not unique when weighted points
// are co-spherical (ideal rings, lattices); the method (and Eq. 1) needs one
// consistent complex.  Exact zeros of the size and side predicates are
// decided by Simulation of Simplicity (Edelsbrunner and Muecke, ACM TOG 1990)
// applied to the weights only: w_q becomes w_q + eps^(1 + q/(n+1)) for atom
// index q, eps -> 0+.  Size and side predicates are polynomials of degree at
// most two in the weights, so their perturbed sign is the sign of the value
// if it is non-zero, else that of the first non-zero partial derivative with
// respect to a weight, atoms taken in ascending index order.  The side
// predicates have the partial -(positive factor) for the tested atom m and
// the size predicates partials summing to minus a positive factor, so every
// perturbed sign is non-zero.  Positions are not perturbed: flat
// tetrahedra and collinear triangles are never in K (their atoms' radical
// planes meet in no single point) and are skipped outright.
//
// Weights are w_q = R_q^2 computed exactly from the double R_q = r_q + probe.
#ifndef SASA_ORACLE_PREDICATES_H
#define SASA_ORACLE_PREDICATES_H
#include <stdint.h>

#include <new>

namespace oracle_pred {

struct Atom {
  double x, y, z;  // centre
  double R;        // probe-inflated radius; the weight is R^2, exactly
  int id;          // index: the symbolic perturbation's order
};

struct Stats {
  int64_t exact = 0;  // predicates the FP64 filter left undecided
  int64_t sos = 0;    // exact zeros decided by the symbolic perturbation
};

// Sign of det[p_j - p_i; p_k - p_i; p_l - p_i] (exact, unperturbed).
int orient(const Atom& i, const Atom& j, const Atom& k, const Atom& l, Stats& st);
// True iff p_i, p_j, p_k are collinear or two of them coincide (exact).
bool collinear(const Atom& i, const Atom& j, const Atom& k, Stats& st);

// Perturbed sign of the power of the orthocentre of the simplex (< 0: inside
// the balls).  Never 0.  Requires a non-degenerate simplex.
int tet_size(const Atom& i, const Atom& j, const Atom& k, const Atom& l, Stats& st);
int tri_size(const Atom& i, const Atom& j, const Atom& k, Stats& st);
int edge_size(const Atom& i, const Atom& j, Stats& st);

// Perturbed sign of pi_m(y) - pi_i(y) at the simplex's orthocentre y
// (> 0: atom m does not cut y away from the simplex's Laguerre face).
// Never 0.  Requires a non-degenerate simplex and m not one of its atoms.
int tet_side(const Atom& i, const Atom& j, const Atom& k, const Atom& l, const Atom& m, Stats& st);
int tri_side(const Atom& i, const Atom& j, const Atom& k, const Atom& m, Stats& st);
int edge_side(const Atom& i, const Atom& j, const Atom& m, Stats& st);
int vertex_side(const Atom& i, const Atom& m, Stats& st);

// Exact sign of a + b*c - d*e (the building block is exercised on its own by
// the tests of the exact arithmetic).
int exact_sign_test(double a, double b, double c, double d, double e);

// The same decisions with the FP64 data of atom i's neighbours and of each
// simplex built once and reused for every tested atom m (the exact path,
// rare, rebuilds what it needs).  Simplices and tested atoms are given as
// positions in the neighbour list of the Base.
struct BaseFlt;
struct TetFlt;
struct TriFlt;
struct EdgeFlt;
class Base {
 public:
  Base(const Atom* atoms, int i, const int* nb, int nnb, Stats& st);
  ~Base();
  const Atom& atom(int q) const { return q < 0 ? atoms_[i_] : atoms_[nb_[q]]; }
  const Atom* atoms_;
  int i_;
  const int* nb_;
  Stats& st_;
  BaseFlt* f_;
};
class TetTest {
 public:
  TetTest(Base& b, int j, int k, int l);  // positions in b's neighbour list
  ~TetTest();
  int orient() const { return sd_; }  // exact sign of the orientation (0: flat)
  int size();                         // as tet_size
  int side(int m);                    // as tet_side (m a position in the list)
 private:
  Base& b_;
  int j_, k_, l_;
  TetFlt* f_;
  int sd_;
  alignas(double) unsigned char buf_[512];  // holds *f_
};
class TriTest {
 public:
  TriTest(Base& b, int j, int k);
  ~TriTest();
  int size();
  int side(int m);
 private:
  Base& b_;
  int j_, k_;
  TriFlt* f_;
  alignas(double) unsigned char buf_[512];
};
class EdgeTest {
 public:
  EdgeTest(Base& b, int j);
  ~EdgeTest();
  int size();
  int side(int m);
 private:
  Base& b_;
  int j_;
  EdgeFlt* f_;
  alignas(double) unsigned char buf_[256];
};

}  // namespace oracle_pred
#endif
