// Marching-cubes case table (host side), derived at first use from a face
// rule instead of being tabulated by hand.
//
// A cube of the grid has corners c = x + 2y + 4z (x, y, z in {0, 1}) and 12
// edges; edge e = 4 a + (the two other coordinates of its lower end, as a
// 2-bit number in axis order) runs along axis a from that lower end.  For a
// configuration of inside (1) and outside (0) corners the surface meets every
// edge whose ends differ.  On each face the crossing points are joined by
// segments: two crossings by one segment; four (inside corners diagonal) by
// two segments, each cutting off one inside corner -- a choice that depends
// on the face's corners only, so the two cubes sharing a face draw the same
// segments and the mesh is watertight.  The segments of the six faces form
// closed loops (each crossing edge lies on two faces); each loop is oriented
// so that its normal points from the inside ends of its edges to the outside
// ends, started at its smallest edge and split into a fan of triangles from
// there.
#pragma once

#include <array>
#include <cstdint>

namespace eses {

struct McTable {
    // per configuration: number of triangles and their edge triples
    uint8_t ntri[256];
    int8_t tri[256][12][3];
};

// Corner of a cube edge: edge e = 4a + r runs along axis a from the corner
// whose other two coordinates are the bits of r (lower bit first in axis order).
inline int mc_edge_corner(int e, int end) {
    const int a = e / 4, r = e % 4;
    int xyz[3] = {0, 0, 0};
    int q = 0;
    for (int b = 0; b < 3; ++b) {
        if (b == a) continue;
        xyz[b] = (r >> q) & 1;
        ++q;
    }
    xyz[a] = end;
    return xyz[0] + 2 * xyz[1] + 4 * xyz[2];
}

const McTable &mc_table();

}  // namespace eses
