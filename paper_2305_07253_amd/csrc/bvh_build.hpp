// Host-side BVH construction shared by the C API (internal header).
#pragma once

#include <cstdint>
#include <vector>

namespace hyb {

// Child reference stored in a node and on the traversal stack:
//   ref >= 0  internal node index
//   ref <  0  leaf: ~ref = (first_triangle << 3) | count, count <= 7
constexpr int kLeafMax = 4;
constexpr int kMaxDepth = 64;
constexpr int32_t kEmptyRef = ~0;  // a leaf with no triangles

// Flattened BVH2 in the device layout.
//   nodes: 16 floats (64 bytes, four float4) per internal node:
//     [0..3]   left  child: lo.x hi.x lo.y hi.y
//     [4..7]   right child: lo.x hi.x lo.y hi.y
//     [8..11]  lo.z hi.z of the left child, lo.z hi.z of the right child
//     [12..13] child references (int32 bits), [14..15] unused
//   tris: 12 floats (48 bytes, three float4) per triangle in leaf order:
//     v0.xyz + original triangle id (int32 bits), v1.xyz + 0, v2.xyz + 0
struct BvhHost {
    std::vector<float> nodes;
    std::vector<float> tris;
    int32_t depth = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // mesh bounds
};

// Binned-SAH build; returns 0 on success, 1 for invalid input, 4 when the
// tree would be deeper than kMaxDepth.
int build_bvh_host(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, BvhHost* out);

}  // namespace hyb
