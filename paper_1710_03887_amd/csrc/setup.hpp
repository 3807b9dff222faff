// Host-side FP64 setup of the nodal DG discretization: reference nodes,
// orthonormal-basis operators, affine element geometry and face matching.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace dg {

struct RefOps {
  int N = 0, Np = 0, Nfp = 0;
  std::vector<double> rst;   // [Np][3]
  std::vector<double> Dr, Ds, Dt;  // [Np][Np] row-major
  std::vector<double> LIFT;  // [Np][4*Nfp]
  std::vector<int32_t> Fmask;  // [4][Nfp]
  // nbr_node[((f*4 + f2)*6 + o)*Nfp + i] = volume node of the neighbour that
  // coincides with node i of my face f, when the neighbour's face is f2 and
  // o is the orientation code of the shared vertex triple.
  std::vector<uint8_t> nbr_node;
  std::vector<double> Vinv;  // [Np][Np] inverse of V[n][m] = psi_m(node n)
};

struct HostMesh {
  int64_t K = 0;
  std::vector<double> xyz;       // [K][4][3] after orientation fix
  std::vector<int64_t> EToV;     // [K][4]
  std::vector<int8_t> bc;        // [K][4]
  std::vector<double> drst_dx;   // [K][3][3]
  std::vector<double> J;         // [K]
  std::vector<double> nrm;       // [K][4][3]
  std::vector<double> Fscale;    // [K][4]
  std::vector<int32_t> EToE;     // [K][4]  neighbour element or -1
  std::vector<uint8_t> EToF;     // [K][4]  neighbour face
  std::vector<uint8_t> orient;   // [K][4]  orientation code 0..5
};

// Builds reference operators for order N.  Returns "" or an error message.
std::string build_reference(int N, RefOps& ops);

// Orientation, geometry and connectivity.  Returns "" or an error message.
std::string build_mesh(const RefOps& ops, int64_t K, const double* xyz,
                       const int64_t* EToV, const int8_t* bc, HostMesh& mesh);

// Physical node coordinates [K][Np][3].
void node_coordinates(const RefOps& ops, const HostMesh& mesh, double* out);

// Neighbour node map [K][4][Nfp] (k'*Np + node, or -1).
void neighbour_map(const RefOps& ops, const HostMesh& mesh, int64_t* out);

// Operators of the weak form with Gauss quadrature (Appendix A: volume
// integrals with a rule exact to degree 2N, face integrals exact to degree
// 2N + 1), acting on the nodal values of the order-N nodes:
//   dq/dt = sum_a Dw_a Fc_a(q at the volume points)
//           - sum_f Fscale_f Lq_f (F* . n)(q at the face points of f),
// Fc_a the contravariant fluxes.  Rules: inside, the collapsed-coordinate
// Gauss-Jacobi product with N + 1 points per direction; on faces Radon's
// symmetric seven-point rule (degree 5, N <= 2).
struct QuadOps {
  int N = 0, Np = 0, Nq = 0, Nfq = 0;
  std::vector<double> Bv;   // [Nq][Np]     nodal values -> volume points
  std::vector<double> Dw;   // [3][Np][Nq]  M^-1 (d l_i / d r_a)(x_q) w_q
  std::vector<double> Bf;   // [4][Nfq][Np] nodal values -> face points of face f
  std::vector<double> Lq;   // [4][Np][Nfq] M^-1 l_i(x_fq) w_fq
  // [((f*4 + f2)*6 + o)][Nfq][Np]: the neighbour's nodal values -> my face
  // points, when its face is f2 and o the orientation code
  std::vector<double> Bnb;
  std::vector<double> xq, wq;     // volume points [Nq][3] (reference) and weights
  std::vector<double> xf, wf;     // face points [4][Nfq][3] (reference) and weights [Nfq]
};

std::string build_quadrature(const RefOps& ops, QuadOps& q);

// Curved (isoparametric) elements (Section 3 names curved boundary faces as
// the remedy for reflections from flat ones): each element's map is the degree-N
// polynomial through the given physical positions of its nodes x [K][Np][3]
// (node order of ops.rst).  An element is curved when one of its nodes lies
// farther than tol times its longest edge from the straight-sided position.
// For each curved element (ascending ids in `elems`), at every node:
//   vg[(c*Np + n)*9 + a*3 + d] = d r_a / d x_d  (inverse of [Dr x, Ds x, Dt x]),
// and at every face node (face-major, Fmask order):
//   sg[(c*4*Nfp + f*Nfp + i)*4 + 0..2] = outward unit normal, [3] = sJ / J,
// the normal being the gradient of the face's reference coordinate
// (-grad t, -grad s, grad(r+s+t), -grad r for faces 0..3).
// Fails when a node's Jacobian is not positive or the nodes that two
// elements share on a face do not coincide (to tol times the edge length).
std::string curved_geometry(const RefOps& ops, const HostMesh& mesh, const double* x, double tol,
                            std::vector<int64_t>& elems, std::vector<float>& vg,
                            std::vector<float>& sg);
// Element containing the physical point x: the element whose smallest
// barycentric coordinate at x is largest (first such element on ties), or -1
// when that coordinate is below -tol (the point lies outside the mesh).
// rst receives the point's reference coordinates in that element.
int64_t locate_point(const HostMesh& mesh, const double x[3], double tol, double rst[3]);

// Reference coordinates of the physical point x in an element whose map is
// the degree-N polynomial through its node positions xe [Np][3]: Newton's
// method on x(r) = sum_i l_i(r) xe_i from the starting point rst (updated in
// place).  Returns false when it does not converge (|step| <= 1e-13 within
// 50 iterations) or meets a singular Jacobian.
bool invert_element_map(const RefOps& ops, const double* xe, const double x[3], double rst[3]);
// Element containing x when some elements are curved (curved: their ids,
// ascending; xc: their node positions [n][Np][3] in that order).  A point
// whose straight-sided element is straight is located as by locate_point.
// Otherwise the curved elements whose straight-sided images lie near x
// (smallest barycentric coordinate >= -0.5) have their maps inverted, nearest
// first, and the one whose reference point has the largest smallest
// barycentric coordinate is taken if that coordinate is >= -tol: a point
// between a chord and a face bent outward, or beyond a curved face that moved
// into its straight-sided element, lands in the element whose curved image
// holds it.  Returns the element, -1 when no element holds the point, or -2
// when the point lies in a curved element's straight-sided image and no map
// that could hold it inverts.
int64_t locate_point_curved(const RefOps& ops, const HostMesh& mesh,
                            const std::vector<int64_t>& curved, const double* xc,
                            const double x[3], double tol, double rst[3]);
// Nodal interpolation weights w[i] = l_i(r, s, t) of the order-N nodal basis
// at a reference point: the polynomial through nodal values u_i takes the
// value sum_i w[i] u_i there.
void interpolation_weights(const RefOps& ops, const double rst[3], double* w);

}  // namespace dg
