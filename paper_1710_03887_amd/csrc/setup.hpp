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

// Element containing the physical point x: the element whose smallest
// barycentric coordinate at x is largest (first such element on ties), or -1
// when that coordinate is below -tol (the point lies outside the mesh).
// rst receives the point's reference coordinates in that element.
int64_t locate_point(const HostMesh& mesh, const double x[3], double tol, double rst[3]);

// Nodal interpolation weights w[i] = l_i(r, s, t) of the order-N nodal basis
// at a reference point: the polynomial through nodal values u_i takes the
// value sum_i w[i] u_i there.
void interpolation_weights(const RefOps& ops, const double rst[3], double* w);

}  // namespace dg
