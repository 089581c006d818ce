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
constexpr int kStackDepth4 = 96;  // traversal stack entries per lane for nodes4
constexpr int32_t kEmptyRef = ~0;  // a leaf with no triangles

// Flattened BVH2 in the device layout.
//   nodes: 16 floats (64 bytes, four float4) per internal node:
//     [0..3]   left  child: lo.x hi.x lo.y hi.y
//     [4..7]   right child: lo.x hi.x lo.y hi.y
//     [8..11]  lo.z hi.z of the left child, lo.z hi.z of the right child
//     [12..13] child references (int32 bits), [14..15] unused
//   tris: 12 floats (48 bytes, three float4) per triangle in leaf order:
//     v0.xyz + original triangle id (int32 bits), v1.xyz + 0, v2.xyz + 0
//   nodes4: the same tree collapsed to four children per node, 32 floats (128
//     bytes, eight float4) per internal node, children c = 0..3 in columns:
//     [0..3] lo.x  [4..7] hi.x  [8..11] lo.y  [12..15] hi.y  [16..19] lo.z
//     [20..23] hi.z  [24..27] child references (int32 bits)  [28..31] unused;
//     missing children have kEmptyRef and a box far outside the scene.
struct BvhHost {
    std::vector<float> nodes;
    std::vector<float> nodes4;
    int32_t depth4 = 0;
    int32_t stack4 = 0;  // most stack entries a nodes4 traversal can hold
    // Traversal entry points: levels l = 0 .. entry_levels-1.  Level l cuts
    // the cube of entry_res voxels of side entry_size (origin entry_lo) into
    // 2 (entry_res >> l) half-cells of side entry_size << l / 2 per axis and
    // stores one entry per window of 2 x 2 x 2 neighbouring half-cells,
    // (2 (entry_res >> l) - 1)^3 windows, x fastest, levels concatenated
    // finest first.  A window's entry is the lowest common ancestor (a nodes4
    // index, or a leaf reference) of every leaf whose box overlaps the window
    // grown by a small margin, or kEmptyRef when none does.  A segment inside
    // one window can only hit triangles under its entry; any segment less
    // than half a cell long per axis lies in some window of that level (the
    // windows overlap by half their side).  entry_res == 0: none.
    std::vector<int32_t> entry;
    int32_t entry_res = 0, entry_levels = 0;
    float entry_lo[3] = {0, 0, 0}, entry_size = 0.0f;
    std::vector<float> tris;
    int32_t depth = 0;
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // mesh bounds
};

// Binned-SAH build; returns 0 on success, 1 for invalid input, 4 when the
// tree would be deeper than kMaxDepth or its nodes4 traversal could need more
// than kStackDepth4 stack entries.
int build_bvh_host(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, BvhHost* out);

}  // namespace hyb
