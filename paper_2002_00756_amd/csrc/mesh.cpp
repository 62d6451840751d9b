// Cubed-sphere column mesh and its horizontal 2x2 hierarchy (host side).
//
// The paper coarsens the mesh horizontally only, each coarse cell being the
// union of 2x2 fine cells (Section 3.6), and runs on cubed-sphere meshes of
// 6 x N x N columns (Section 5.1). The topology is built here from integer
// geometry on the cube [0, 2N]^3: panel p has outward normal n, origin O and
// in-panel axes a (E, index i) and b (N, index j); cell (p,i,j) is centred at
// O + (2i+1)a + (2j+1)b. A step off the panel goes to the edge and one unit
// down the adjacent face, the one whose normal is the step direction.
#include "mesh.hpp"

#include <array>
#include <cstdint>

namespace hh {
namespace {

struct Vec3 {
    int64_t x, y, z;
};
inline Vec3 operator+(Vec3 u, Vec3 v) { return {u.x + v.x, u.y + v.y, u.z + v.z}; }
inline Vec3 operator-(Vec3 u, Vec3 v) { return {u.x - v.x, u.y - v.y, u.z - v.z}; }
inline Vec3 operator*(int64_t s, Vec3 v) { return {s * v.x, s * v.y, s * v.z}; }
inline Vec3 operator-(Vec3 v) { return {-v.x, -v.y, -v.z}; }
inline int64_t dot(Vec3 u, Vec3 v) { return u.x * v.x + u.y * v.y + u.z * v.z; }
inline bool same(Vec3 u, Vec3 v) { return u.x == v.x && u.y == v.y && u.z == v.z; }

struct Panel {
    Vec3 normal, origin_unit, east, north;  // origin in units of 2N
};

// p0 +x, p1 +y, p2 -x, p3 -y, p4 +z, p5 -z
const std::array<Panel, 6> kPanels = {{
    {{1, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {1, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, 1, 1}, {0, 0, -1}, {0, -1, 0}},
    {{0, -1, 0}, {0, 0, 1}, {0, 0, -1}, {1, 0, 0}},
    {{0, 0, 1}, {1, 1, 1}, {-1, 0, 0}, {0, -1, 0}},
    {{0, 0, -1}, {0, 0, 0}, {0, 1, 0}, {1, 0, 0}},
}};

int panel_with_normal(Vec3 n) {
    for (int q = 0; q < 6; ++q)
        if (same(kPanels[q].normal, n)) return q;
    return -1;
}

}  // namespace

void build_neighbours(int N, int32_t* nbr) {
    const int64_t M = 2 * int64_t(N);
    const int64_t ncol = 6 * int64_t(N) * N;
    for (int p = 0; p < 6; ++p) {
        const Panel& P = kPanels[p];
        const Vec3 O = M * P.origin_unit;
        const Vec3 steps[4] = {P.east, -P.east, P.north, -P.north};
        const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
        int target[4];
        for (int d = 0; d < 4; ++d) target[d] = panel_with_normal(steps[d]);
        for (int j = 0; j < N; ++j) {
            for (int i = 0; i < N; ++i) {
                const int64_t c = int64_t(p) * N * N + int64_t(j) * N + i;
                const Vec3 centre = O + (2 * i + 1) * P.east + (2 * j + 1) * P.north;
                for (int d = 0; d < 4; ++d) {
                    const int i2 = i + di[d], j2 = j + dj[d];
                    int64_t n;
                    if (i2 >= 0 && i2 < N && j2 >= 0 && j2 < N) {
                        n = int64_t(p) * N * N + int64_t(j2) * N + i2;
                    } else {
                        const Panel& Q = kPanels[target[d]];
                        const Vec3 rel = centre + steps[d] - P.normal - M * Q.origin_unit;
                        const int64_t ia = (dot(rel, Q.east) - 1) / 2;
                        const int64_t jb = (dot(rel, Q.north) - 1) / 2;
                        n = int64_t(target[d]) * N * N + jb * N + ia;
                    }
                    nbr[d * ncol + c] = int32_t(n);
                }
            }
        }
    }
}

void build_face_table(int N, const int32_t* nbr, int32_t* ftab) {
    const int64_t ncol = 6 * int64_t(N) * N;
    for (int64_t c = 0; c < ncol; ++c) {
        ftab[0 * ncol + c] = int32_t(c);          // E: own face, slot 0
        ftab[2 * ncol + c] = int32_t(ncol + c);   // N: own face, slot 1
        for (int d : {1, 3}) {                    // W, S: the neighbour's face
            const int64_t o = nbr[d * ncol + c];
            const bool east_of_owner = nbr[0 * ncol + o] == c;
            ftab[d * ncol + c] = int32_t(east_of_owner ? o : ncol + o);
        }
    }
}

void build_parent(int N, int32_t* parent) {
    const int64_t Nc = N / 2;
    for (int p = 0; p < 6; ++p)
        for (int j = 0; j < N; ++j)
            for (int i = 0; i < N; ++i)
                parent[int64_t(p) * N * N + int64_t(j) * N + i] =
                    int32_t(p * Nc * Nc + (j / 2) * Nc + (i / 2));
}

void build_children(int Nc, int32_t* child) {
    const int64_t Nf = 2 * int64_t(Nc);
    const int64_t ncc = 6 * int64_t(Nc) * Nc;
    for (int p = 0; p < 6; ++p)
        for (int J = 0; J < Nc; ++J)
            for (int I = 0; I < Nc; ++I) {
                const int64_t C = int64_t(p) * Nc * Nc + int64_t(J) * Nc + I;
                for (int s = 0; s < 4; ++s) {
                    const int64_t di = s & 1, dj = s >> 1;  // (0,0),(1,0),(0,1),(1,1)
                    child[s * ncc + C] =
                        int32_t(p * Nf * Nf + (2 * J + dj) * Nf + (2 * I + di));
                }
            }
}

}  // namespace hh
