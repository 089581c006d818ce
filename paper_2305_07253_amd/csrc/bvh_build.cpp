// Binned-SAH BVH2 construction on the host (Wald, "On fast construction of
// SAH-based bounding volume hierarchies", 2007: 32 bins per axis over the
// centroid bounds), flattened into 64-byte two-child nodes (read by the
// distance-field build's nearest-triangle queries), collapsed into 128-byte
// four-wide nodes that the trace traversal reads with seven 16-byte loads, and
// the pyramid of traversal entry points.
#include "bvh_build.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

namespace hyb {
namespace {

constexpr int kBins = 32;
constexpr float kTraversalCost = 1.0f;
constexpr float kTriangleCost = 1.0f;

struct Box {
    float lo[3], hi[3];
    void reset() {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::numeric_limits<float>::infinity();
            hi[a] = -std::numeric_limits<float>::infinity();
        }
    }
    void grow(const Box& b) {
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.lo[a]);
            hi[a] = std::max(hi[a], b.hi[a]);
        }
    }
    float area() const {
        float e[3];
        for (int a = 0; a < 3; ++a) e[a] = std::max(0.0f, hi[a] - lo[a]);
        return 2.0f * (e[0] * e[1] + e[1] * e[2] + e[2] * e[0]);
    }
};

struct Prim {
    Box box;
    float c[3];
};

struct TmpNode {
    Box box;
    int child[2] = {-1, -1};  // indices into the temporary node array
    int first = 0, count = 0; // leaf range in the index array (count > 0 => leaf)
};

struct Builder {
    const std::vector<Prim>& prims;
    std::vector<int> idx;
    std::vector<TmpNode> nodes;
    int max_depth = 0;

    explicit Builder(const std::vector<Prim>& p) : prims(p), idx(p.size()) {
        for (size_t i = 0; i < p.size(); ++i) idx[i] = static_cast<int>(i);
    }

    int make_leaf(const Box& b, int first, int count) {
        TmpNode n;
        n.box = b;
        n.first = first;
        n.count = count;
        nodes.push_back(n);
        return static_cast<int>(nodes.size()) - 1;
    }

    // Builds the subtree over idx[first, first+count); returns its node index.
    int build(int first, int count, int depth) {
        max_depth = std::max(max_depth, depth);
        Box bounds, cbounds;
        bounds.reset();
        cbounds.reset();
        for (int i = first; i < first + count; ++i) {
            const Prim& p = prims[idx[i]];
            bounds.grow(p.box);
            Box c;
            for (int a = 0; a < 3; ++a) c.lo[a] = c.hi[a] = p.c[a];
            cbounds.grow(c);
        }
        if (count == 1) return make_leaf(bounds, first, count);

        // SAH sweep over the bins of every axis with a nonzero centroid extent.
        float best_cost = std::numeric_limits<float>::infinity();
        int best_axis = -1, best_split = -1;
        const float parent_area = bounds.area();
        for (int a = 0; a < 3; ++a) {
            const float ext = cbounds.hi[a] - cbounds.lo[a];
            if (!(ext > 0.0f)) continue;
            const float scale = kBins / ext;
            int cnt[kBins] = {};
            Box bb[kBins];
            for (int b = 0; b < kBins; ++b) bb[b].reset();
            for (int i = first; i < first + count; ++i) {
                const Prim& p = prims[idx[i]];
                int b = std::min(kBins - 1, static_cast<int>((p.c[a] - cbounds.lo[a]) * scale));
                cnt[b]++;
                bb[b].grow(p.box);
            }
            float right_area[kBins];
            int right_cnt[kBins];
            Box acc;
            acc.reset();
            int n = 0;
            for (int b = kBins - 1; b > 0; --b) {
                acc.grow(bb[b]);
                n += cnt[b];
                right_area[b] = acc.area();
                right_cnt[b] = n;
            }
            acc.reset();
            n = 0;
            for (int b = 0; b < kBins - 1; ++b) {
                acc.grow(bb[b]);
                n += cnt[b];
                if (n == 0 || right_cnt[b + 1] == 0) continue;
                float cost = kTraversalCost +
                             kTriangleCost * (acc.area() * n + right_area[b + 1] * right_cnt[b + 1]) /
                                 std::max(parent_area, 1e-30f);
                if (cost < best_cost) {
                    best_cost = cost;
                    best_axis = a;
                    best_split = b;
                }
            }
        }

        const float leaf_cost = kTriangleCost * count;
        if (count <= kLeafMax && leaf_cost <= best_cost) return make_leaf(bounds, first, count);

        int mid;
        if (best_axis < 0) {
            mid = first + count / 2;  // all centroids coincide: split by position in the list
        } else {
            const float ext = cbounds.hi[best_axis] - cbounds.lo[best_axis];
            const float scale = kBins / ext;
            const float lo = cbounds.lo[best_axis];
            int* m = std::partition(idx.data() + first, idx.data() + first + count, [&](int i) {
                int b = std::min(kBins - 1, static_cast<int>((prims[i].c[best_axis] - lo) * scale));
                return b <= best_split;
            });
            mid = static_cast<int>(m - idx.data());
            if (mid == first || mid == first + count) mid = first + count / 2;
        }
        TmpNode inner;
        inner.box = bounds;
        nodes.push_back(inner);
        int self = static_cast<int>(nodes.size()) - 1;
        int l = build(first, mid - first, depth + 1);
        int r = build(mid, first + count - mid, depth + 1);
        nodes[self].child[0] = l;
        nodes[self].child[1] = r;
        return self;
    }
};

inline float bits_as_float(int32_t v) {
    float f;
    std::memcpy(&f, &v, 4);
    return f;
}

constexpr int kEntryRes = 64;

// Entry points of BvhHost (see the header): the finest level by a box query
// per voxel, the coarser ones as the common ancestor of their 8 children.
void build_entries(BvhHost* out) {
    out->entry.clear();
    out->entry_res = 0;
    out->entry_levels = 0;
    const size_t n4 = out->nodes4.size() / 32;
    float ext = 0.0f;
    for (int a = 0; a < 3; ++a) ext = std::max(ext, out->hi[a] - out->lo[a]);
    if (n4 == 0 || !(ext > 0.0f)) return;
    const float* nd = out->nodes4.data();
    auto ref_of = [&](size_t node, int c) {
        int32_t r;
        std::memcpy(&r, nd + 32 * node + 24 + c, 4);
        return r;
    };
    // parents and depths of nodes and leaves
    // a leaf is identified by its first triangle, (~ref) >> 3
    std::vector<int32_t> parent(n4, -1), depth(n4, 0), leaf_parent(out->tris.size() / 12 + 1, -1);
    for (size_t i = 0; i < n4; ++i)  // children come after their parent in the array
        for (int c = 0; c < 4; ++c) {
            const int32_t r = ref_of(i, c);
            if (r == kEmptyRef) continue;
            if (r >= 0) {
                parent[r] = static_cast<int32_t>(i);
                depth[r] = depth[i] + 1;
            } else {
                leaf_parent[(~r) >> 3] = static_cast<int32_t>(i);
            }
        }
    auto depth_of = [&](int32_t r) { return r >= 0 ? depth[r] : depth[leaf_parent[(~r) >> 3]] + 1; };
    auto up = [&](int32_t r) { return r >= 0 ? parent[r] : leaf_parent[(~r) >> 3]; };
    auto lca = [&](int32_t a, int32_t b) {
        if (a == kEmptyRef) return b;
        if (b == kEmptyRef) return a;
        int da = depth_of(a), db = depth_of(b);
        while (da > db) { a = up(a); --da; }
        while (db > da) { b = up(b); --db; }
        while (a != b) { a = up(a); b = up(b); }
        return a;
    };

    const int E = kEntryRes;
    const float size = ext / static_cast<float>(E) * (1.0f + 1e-4f);
    for (int a = 0; a < 3; ++a) out->entry_lo[a] = out->lo[a] - 0.5f * (size * E - (out->hi[a] - out->lo[a]));
    out->entry_size = size;
    int levels = 0;
    size_t total = 0;
    for (int e = E; e >= 1; e >>= 1) {
        const size_t w = static_cast<size_t>(2 * e - 1);
        total += w * w * w;
        ++levels;
    }
    out->entry.assign(total, kEmptyRef);
    // every leaf joins each finest half-cell its box overlaps, the box grown
    // by a margin (FP32 rounding of segment end points is far below it)
    int H = 2 * E;
    const double half = 0.5 * static_cast<double>(size);
    std::vector<int32_t> cells(static_cast<size_t>(H) * H * H, kEmptyRef);
    const double margin = 1e-3 * size;
    for (size_t i = 0; i < n4; ++i)
        for (int c = 0; c < 4; ++c) {
            const int32_t r = ref_of(i, c);
            if (r == kEmptyRef || r >= 0) continue;
            const float* q = nd + 32 * i;
            int v0[3], v1[3];
            for (int a = 0; a < 3; ++a) {
                const double qlo = q[8 * a + c], qhi = q[8 * a + 4 + c];
                const double slack = margin + 1e-6 * (1.0 + std::max(std::fabs(qlo), std::fabs(qhi)));
                const double u0 = (qlo - slack - out->entry_lo[a]) / half, u1 = (qhi + slack - out->entry_lo[a]) / half;
                v0[a] = static_cast<int>(std::floor(std::min(std::max(u0, 0.0), H - 1.0)));
                v1[a] = static_cast<int>(std::floor(std::min(std::max(u1, 0.0), H - 1.0)));
            }
            for (int z = v0[2]; z <= v1[2]; ++z)
                for (int y = v0[1]; y <= v1[1]; ++y)
                    for (int x = v0[0]; x <= v1[0]; ++x) {
                        int32_t& slot = cells[x + static_cast<size_t>(H) * (y + static_cast<size_t>(H) * z)];
                        slot = lca(slot, r);
                    }
        }
    size_t off = 0;
    for (int l = 0; l < levels; ++l) {
        // windows of 2 x 2 x 2 half-cells of this level
        const int W = H - 1;
        for (int z = 0; z < W; ++z)
            for (int y = 0; y < W; ++y)
                for (int x = 0; x < W; ++x) {
                    int32_t acc = kEmptyRef;
                    for (int c = 0; c < 8; ++c) {
                        const int cx = x + (c & 1), cy = y + ((c >> 1) & 1), cz = z + (c >> 2);
                        acc = lca(acc, cells[cx + static_cast<size_t>(H) * (cy + static_cast<size_t>(H) * cz)]);
                    }
                    out->entry[off + x + static_cast<size_t>(W) * (y + static_cast<size_t>(W) * z)] = acc;
                }
        off += static_cast<size_t>(W) * W * W;
        if (l + 1 == levels) break;
        // the next level's half-cells: 2 x 2 x 2 of this level's
        const int h = H / 2;
        std::vector<int32_t> up(static_cast<size_t>(h) * h * h, kEmptyRef);
        for (int z = 0; z < h; ++z)
            for (int y = 0; y < h; ++y)
                for (int x = 0; x < h; ++x) {
                    int32_t acc = kEmptyRef;
                    for (int c = 0; c < 8; ++c) {
                        const int cx = 2 * x + (c & 1), cy = 2 * y + ((c >> 1) & 1), cz = 2 * z + (c >> 2);
                        acc = lca(acc, cells[cx + static_cast<size_t>(H) * (cy + static_cast<size_t>(H) * cz)]);
                    }
                    up[x + static_cast<size_t>(h) * (y + static_cast<size_t>(h) * z)] = acc;
                }
        cells.swap(up);
        H = h;
    }
    out->entry_res = E;
    out->entry_levels = levels;
}

}  // namespace

int build_bvh_host(const float* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, BvhHost* out) {
    if (n_verts < 0 || n_tris < 0 || (n_verts > 0 && !verts) || (n_tris > 0 && !tris) || !out) return 1;
    if (n_tris > (int64_t(1) << 28)) return 4;
    for (int64_t i = 0; i < 3 * n_verts; ++i)
        if (!std::isfinite(verts[i])) return 1;
    for (int64_t i = 0; i < 3 * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return 1;

    std::vector<Prim> prims(static_cast<size_t>(n_tris));
    Box all;
    all.reset();
    for (int64_t t = 0; t < n_tris; ++t) {
        Prim& p = prims[t];
        p.box.reset();
        for (int k = 0; k < 3; ++k) {
            const float* v = verts + 3 * static_cast<int64_t>(tris[3 * t + k]);
            Box pt;
            for (int a = 0; a < 3; ++a) pt.lo[a] = pt.hi[a] = v[a];
            p.box.grow(pt);
        }
        for (int a = 0; a < 3; ++a) p.c[a] = 0.5f * (p.box.lo[a] + p.box.hi[a]);
        all.grow(p.box);
    }
    for (int a = 0; a < 3; ++a) {
        out->lo[a] = n_tris ? all.lo[a] : 0.0f;
        out->hi[a] = n_tris ? all.hi[a] : 0.0f;
    }

    Builder b(prims);
    int root = -1;
    if (n_tris > 0) root = b.build(0, static_cast<int>(n_tris), 1);
    if (b.max_depth > kMaxDepth) return 4;

    // Flatten depth-first: internal nodes get consecutive output indices, leaves
    // become references into the leaf-ordered triangle array.
    out->nodes.clear();
    out->tris.assign(static_cast<size_t>(12 * n_tris), 0.0f);
    int64_t tri_cursor = 0;
    auto leaf_ref = [&](const TmpNode& n) -> int32_t {
        int32_t first = static_cast<int32_t>(tri_cursor);
        for (int i = 0; i < n.count; ++i) {
            int t = b.idx[n.first + i];
            float* dst = out->tris.data() + 12 * tri_cursor;
            for (int k = 0; k < 3; ++k) {
                const float* v = verts + 3 * static_cast<int64_t>(tris[3 * static_cast<int64_t>(t) + k]);
                dst[4 * k + 0] = v[0];
                dst[4 * k + 1] = v[1];
                dst[4 * k + 2] = v[2];
                dst[4 * k + 3] = k == 0 ? bits_as_float(t) : 0.0f;
            }
            ++tri_cursor;
        }
        return ~((first << 3) | n.count);
    };
    std::vector<int32_t> leaf_refs(b.nodes.size(), 0);
    std::vector<char> leaf_done(b.nodes.size(), 0);
    auto leaf_of = [&](int tn) -> int32_t {  // each leaf's triangles are written once
        if (!leaf_done[tn]) {
            leaf_refs[tn] = leaf_ref(b.nodes[tn]);
            leaf_done[tn] = 1;
        }
        return leaf_refs[tn];
    };
    const float far = 1e30f;
    Box empty_box;
    for (int a = 0; a < 3; ++a) empty_box.lo[a] = empty_box.hi[a] = far;

    // emit(node): writes the internal node and returns its output index
    std::vector<std::pair<int, int>> todo;  // (tmp node, output slot)
    auto alloc = [&]() {
        out->nodes.resize(out->nodes.size() + 16, 0.0f);
        return static_cast<int32_t>(out->nodes.size() / 16 - 1);
    };
    auto write_children = [&](int32_t slot, const Box& l, int32_t lref, const Box& r, int32_t rref) {
        float* n = out->nodes.data() + 16 * static_cast<size_t>(slot);
        n[0] = l.lo[0]; n[1] = l.hi[0]; n[2] = l.lo[1]; n[3] = l.hi[1];
        n[4] = r.lo[0]; n[5] = r.hi[0]; n[6] = r.lo[1]; n[7] = r.hi[1];
        n[8] = l.lo[2]; n[9] = l.hi[2]; n[10] = r.lo[2]; n[11] = r.hi[2];
        n[12] = bits_as_float(lref); n[13] = bits_as_float(rref); n[14] = 0.0f; n[15] = 0.0f;
    };

    // BVH4 for the trace kernels: each node takes the children of its BVH2
    // node and replaces the inner child of largest surface area by that
    // child's two children until it has four (or only leaves are left).
    auto emit4 = [&]() {
        out->nodes4.clear();
        auto alloc4 = [&]() {
            out->nodes4.resize(out->nodes4.size() + 32, 0.0f);
            return static_cast<int32_t>(out->nodes4.size() / 32 - 1);
        };
        auto write4 = [&](int32_t slot, const int* kids, int nk) {
            float* q = out->nodes4.data() + 32 * static_cast<size_t>(slot);
            for (int c = 0; c < 4; ++c) {
                const Box& bx = c < nk ? b.nodes[kids[c]].box : empty_box;
                q[0 + c] = bx.lo[0]; q[4 + c] = bx.hi[0];
                q[8 + c] = bx.lo[1]; q[12 + c] = bx.hi[1];
                q[16 + c] = bx.lo[2]; q[20 + c] = bx.hi[2];
            }
        };
        out->depth4 = 1;
        out->stack4 = 0;
        if (root < 0 || b.nodes[root].count > 0) {
            int32_t s = alloc4();
            int kid = root;
            write4(s, &kid, root < 0 ? 0 : 1);
            float* q = out->nodes4.data() + 32 * static_cast<size_t>(s);
            for (int c = 0; c < 4; ++c) q[24 + c] = bits_as_float(c == 0 && root >= 0 ? leaf_of(root) : kEmptyRef);
            return;
        }
        // `pushed`: stack entries a traversal can hold on arrival at the node
        // (the nearer-first order pushes the other hit children of every
        // ancestor), so its maximum bounds the traversal stack.
        struct Item { int tn; int32_t slot; int depth; int pushed; };
        std::vector<Item> st;
        st.push_back({root, alloc4(), 1, 0});
        while (!st.empty()) {
            const Item it = st.back();
            st.pop_back();
            out->depth4 = std::max(out->depth4, it.depth);
            int kids[4] = {b.nodes[it.tn].child[0], b.nodes[it.tn].child[1], -1, -1};
            int nk = 2;
            while (nk < 4) {
                int best = -1;
                float best_area = -1.0f;
                for (int c = 0; c < nk; ++c) {
                    const TmpNode& ch = b.nodes[kids[c]];
                    if (ch.count == 0 && ch.box.area() > best_area) {
                        best_area = ch.box.area();
                        best = c;
                    }
                }
                if (best < 0) break;
                const TmpNode& ch = b.nodes[kids[best]];
                kids[best] = ch.child[0];
                kids[nk++] = ch.child[1];
            }
            write4(it.slot, kids, nk);
            out->stack4 = std::max(out->stack4, it.pushed + nk - 1);
            int32_t refs[4] = {kEmptyRef, kEmptyRef, kEmptyRef, kEmptyRef};
            Item pending[4];
            int np = 0;
            for (int c = 0; c < nk; ++c) {
                if (b.nodes[kids[c]].count > 0) {
                    refs[c] = leaf_of(kids[c]);
                } else {
                    refs[c] = alloc4();
                    pending[np++] = {kids[c], refs[c], it.depth + 1, it.pushed + nk - 1};
                }
            }
            float* q = out->nodes4.data() + 32 * static_cast<size_t>(it.slot);
            for (int c = 0; c < 4; ++c) q[24 + c] = bits_as_float(refs[c]);
            for (int c = np - 1; c >= 0; --c) st.push_back(pending[c]);
        }
    };

    if (root < 0) {
        int32_t s = alloc();
        write_children(s, empty_box, kEmptyRef, empty_box, kEmptyRef);
        out->depth = 1;
        emit4();
        build_entries(out);
        return 0;
    }
    if (b.nodes[root].count > 0) {
        int32_t s = alloc();
        int32_t lr = leaf_of(root);
        write_children(s, b.nodes[root].box, lr, empty_box, kEmptyRef);
        out->depth = 1;
        emit4();
        build_entries(out);
        return 0;
    }
    // iterative pre-order so the left child usually follows its parent in memory
    std::vector<std::pair<int, int32_t>> stack;
    stack.push_back({root, alloc()});
    while (!stack.empty()) {
        auto [tn, slot] = stack.back();
        stack.pop_back();
        const TmpNode& n = b.nodes[tn];
        int32_t refs[2];
        int32_t pending_slot[2] = {-1, -1};
        for (int c = 0; c < 2; ++c) {
            const TmpNode& ch = b.nodes[n.child[c]];
            if (ch.count > 0) {
                refs[c] = leaf_of(n.child[c]);
            } else {
                pending_slot[c] = alloc();
                refs[c] = pending_slot[c];
            }
        }
        write_children(slot, b.nodes[n.child[0]].box, refs[0], b.nodes[n.child[1]].box, refs[1]);
        for (int c = 1; c >= 0; --c)
            if (pending_slot[c] >= 0) stack.push_back({n.child[c], pending_slot[c]});
    }
    out->depth = b.max_depth;
    emit4();
    if (out->stack4 > kStackDepth4) return 4;
    build_entries(out);
    return 0;
}

}  // namespace hyb
