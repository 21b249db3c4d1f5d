// Tetrahedral meshes for the three-dimensional form of the scheme (the paper's Conclusion:
// tetrahedra, E and j on edges, B on faces, n on nodes), shared by the host builder (tet.cpp)
// and the device stepping (tet.hip).
#pragma once

#include <cstdint>
#include <vector>

#include "internal.hpp"

namespace tyee {

// Host mesh in canonical numbering: nodes as given, edges by (lower, higher) node id, faces by
// their sorted node triples (a, b, c), tetrahedra as given (reoriented to positive volume).
// A face's unit normal follows a -> b -> c by the right-hand rule; its edges are (a, b), (b, c)
// and (a, c), which that circuit runs along, along and against.  The box's walls are perfect
// conductors: a face with one tetrahedron is a wall face, an edge of a wall face a wall edge.
struct TetMesh {
    int64_t nv = 0, ne = 0, nf = 0, nt = 0, n_inner_edge = 0, n_inner_face = 0;
    std::vector<double> xyz;            // [nv][3]
    std::vector<int32_t> tet;           // [nt][4], det[b - a, c - a, d - a] > 0
    std::vector<int32_t> edge;          // [ne][2]
    std::vector<int32_t> face;          // [nf][3]
    std::vector<int32_t> face_edge;     // [nf][3]: (a, b), (b, c), (a, c)
    std::vector<int32_t> front, back;   // [nf]: the tetrahedron on the +normal / -normal side, -1 if none
    std::vector<uint8_t> inner_edge, inner_face;
    std::vector<double> elen, dual_area;   // [ne]; dual_area (the Voronoi polygon) 0 on wall edges
    std::vector<double> farea, d;          // [nf]; d = (C_front - C_back) . normal, 0 on wall faces
    std::vector<double> normal;            // [nf][3]
    std::vector<double> C;                 // [nt][3] circumcentres
    // inner edge -> the faces around it, each as f (the face's circuit runs along the edge) or
    // ~f (against), in ascending face id; wall edges have empty rows
    std::vector<int64_t> ef_off;        // [ne + 1]
    std::vector<int32_t> ef;
};

int build_tet(const double *xyz, int64_t nv, const int32_t *tets, int64_t nt, TetMesh &m);
// Largest eigenvalue of K = -curl_B curl_E on the inner edges (FP64 power iteration in the
// energy weights A*_e |e|).
int tet_power(const TetMesh &m, int64_t max_iter, double rtol, uint64_t seed, double *lambda, int64_t *iters);

}  // namespace tyee

struct tyee_tet {
    tyee::TetMesh m;
};
