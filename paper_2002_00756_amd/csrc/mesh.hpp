// Host-side cubed-sphere mesh tables (see mesh.cpp).
#pragma once
#include <cstdint>

namespace hh {

// nbr[4][6N^2]: neighbour column in directions E, W, N, S.
void build_neighbours(int N, int32_t* nbr);
// ftab[4][6N^2]: stored face (slot*ncol + owner) behind each direction.
void build_face_table(int N, const int32_t* nbr, int32_t* ftab);
// parent[6N^2]: column of C<N/2> containing each column of C<N> (N even).
void build_parent(int N, int32_t* parent);
// child[4][6Nc^2]: children (0,0),(1,0),(0,1),(1,1) of each column of C<Nc> in C<2Nc>.
void build_children(int Nc, int32_t* child);

}  // namespace hh
