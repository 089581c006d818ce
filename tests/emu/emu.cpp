// CPU emulation of the library's kernels: runs the exact per-ray trace body and
// per-node distance-field body on the host, so tests can compare the kernel
// logic with the oracle (and run it under AddressSanitizer) without a GPU.
//
//   emu <input.bin> <output.bin>
//
// input:  int64 hdr[8] = {what, n_rays, n_verts, n_tris, N, ray_arrays, mode, fmt}
//         ray_arrays: bit 0 per-ray tmin follows, bit 1 per-ray tmax follows
//         float par[8] = {tmax, tau, lo_x, lo_y, lo_z, h, flag, tau_end}
//         flag: exterior solid (what 1) / certified 1-Lipschitz samples (what 0)
//         verts f32[3 n_verts], tris i32[3 n_tris],
//         grid (what 0, N > 0): f32[N^3] dequantized values, then the stored
//           f16 values [N^3] for fmt 1 and 3 (fmt 3: laid out in the two-cell
//           bricks of large grids), the f32 block scales [nb^3] (blocks of 8^3
//           cells) for fmt 2, all x fastest (the emulator lays them out in
//           bricks; an I8 cell holds its corners' dequantized values over
//           the scale of its block, then that scale),
//         rays f32[6 n_rays] (SoA rows), tmin f32[n_rays], tmax f32[n_rays]
// what 0 (trace): output t f32[n], prim i32[n], u f32[n], v f32[n], counts i32[3n]
// what 1 (sdf):   output f32[N^3] signed distances of the grid nodes
// what 3 (block order): hdr[1] = blocks nb, hdr[4] = run; output u32[nb], the
//                 block each workgroup of a trace launch processes
// what 2 (grad):  input as what 0 plus t_hit f32[n_rays] after the ray arrays;
//                 output per ray i64[8] node indices (-1: no contribution) and
//                 f32[8] d t / d sample
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "bvh_build.hpp"
#include "hyb_device.hpp"
#include "sdf_device.hpp"

template <class T>
static std::vector<T> rd(FILE* f, size_t n) {
    std::vector<T> v(n);
    if (n && fread(v.data(), sizeof(T), n, f) != n) {
        fprintf(stderr, "short read\n");
        exit(2);
    }
    return v;
}

int main(int argc, char** argv) {
    if (argc != 3) return 2;
    FILE* f = fopen(argv[1], "rb");
    if (!f) return 2;
    auto hdr = rd<long long>(f, 8);
    auto par = rd<float>(f, 8);
    if (hdr[0] == 3) {
        fclose(f);
        const uint32_t nb = (uint32_t)hdr[1], run = (uint32_t)hdr[4];
        std::vector<uint32_t> order(nb);
        for (uint32_t b = 0; b < nb; ++b) order[b] = hyb::xcd_block(b, nb, run);
        FILE* o = fopen(argv[2], "wb");
        if (!o || fwrite(order.data(), sizeof(uint32_t), nb, o) != nb) return 2;
        fclose(o);
        return 0;
    }
    const long long what = hdr[0], n = hdr[1], nv = hdr[2], nt = hdr[3], N = hdr[4], has_tmin = hdr[5], mode = hdr[6];
    const int fmt = (int)hdr[7];
    const long long nb = N > 1 ? hyb::i8_blocks((int)N) : 0;
    auto verts = rd<float>(f, 3 * nv);
    auto tris = rd<int32_t>(f, 3 * nt);
    std::vector<float> grid = what != 1 && N > 0 ? rd<float>(f, N * N * N) : std::vector<float>();
    std::vector<_Float16> g16 = what == 0 && N > 0 && (fmt == 1 || fmt == 3) ? rd<_Float16>(f, N * N * N) : std::vector<_Float16>();
    std::vector<float> scales = what == 0 && N > 0 && fmt == 2 ? rd<float>(f, nb * nb * nb) : std::vector<float>();
    auto rays = rd<float>(f, 6 * n);
    auto tmin = (has_tmin & 1) ? rd<float>(f, n) : std::vector<float>();
    auto tmaxr = (has_tmin & 2) ? rd<float>(f, n) : std::vector<float>();
    auto thit = what == 2 ? rd<float>(f, n) : std::vector<float>();
    fclose(f);

    hyb::BvhHost bvh;
    int rc = hyb::build_bvh_host(verts.data(), nv, tris.data(), nt, &bvh);
    if (rc) {
        fprintf(stderr, "bvh build failed %d\n", rc);
        return 3;
    }
    // exact-size device-layout buffers so the sanitizer sees any overrun
    std::vector<float4> nodes(bvh.nodes.size() / 4), nodes4(bvh.nodes4.size() / 4), tri4(bvh.tris.size() / 4);
    for (size_t i = 0; i < nodes.size(); ++i)
        nodes[i] = make_float4(bvh.nodes[4 * i], bvh.nodes[4 * i + 1], bvh.nodes[4 * i + 2], bvh.nodes[4 * i + 3]);
    for (size_t i = 0; i < nodes4.size(); ++i)
        nodes4[i] = make_float4(bvh.nodes4[4 * i], bvh.nodes4[4 * i + 1], bvh.nodes4[4 * i + 2], bvh.nodes4[4 * i + 3]);
    for (size_t i = 0; i < tri4.size(); ++i)
        tri4[i] = make_float4(bvh.tris[4 * i], bvh.tris[4 * i + 1], bvh.tris[4 * i + 2], bvh.tris[4 * i + 3]);

    FILE* o = fopen(argv[2], "wb");
    if (!o) return 2;
    if (what == 1) {
        std::vector<float> out(N * N * N);
        for (long long id = 0; id < N * N * N; ++id) {
            const long long i = id % N, j = (id / N) % N, k = id / (N * N);
            hyb::D3 p = hyb::d3((double)par[2] + (double)i * (double)par[5], (double)par[3] + (double)j * (double)par[5],
                                (double)par[4] + (double)k * (double)par[5]);
            out[id] = (float)hyb::sdf_node_value(tri4.empty() ? nullptr : nodes.data(), tri4.data(), p, (int)par[6]);
        }
        fwrite(out.data(), 4, out.size(), o);
        fclose(o);
        return 0;
    }
    float L = 0.0f, slope[3] = {0.0f, 0.0f, 0.0f};
    const float inv_h = 1.0f / par[5];
    for (long long k = 0; k + 1 < N; ++k)
        for (long long j = 0; j + 1 < N; ++j)
            for (long long i = 0; i + 1 < N; ++i) {
                const float* p = grid.data() + i + N * (j + N * k);
                const float c[8] = {p[0], p[1], p[N], p[N + 1], p[N * N], p[N * N + 1], p[N * N + N], p[N * N + N + 1]};
                L = fmaxf(L, hyb::cell_lipschitz(c, inv_h));
                float s[3];
                hyb::cell_slopes(c, inv_h, s);
                for (int a = 0; a < 3; ++a) slope[a] = fmaxf(slope[a], s[a]);
            }
    L = hyb::finish_lipschitz(L);
    for (int a = 0; a < 3; ++a) slope[a] = hyb::finish_slope(slope[a]);

    // the kernels read the samples in the format's bricked layout (exact-size
    // buffers, so the sanitizer sees any read past the storage); the FP32
    // copy also serves the backward body
    const size_t n32 = N > 0 ? (size_t)hyb::Brick<hyb::kF32>::storage((int)N) : 0;
    const size_t n16 = N > 0 ? (size_t)(fmt == 3 ? hyb::Brick<hyb::kF16B2>::storage((int)N)
                                                 : hyb::Brick<hyb::kF16>::storage((int)N)) : 0;
    const size_t n8 = N > 0 ? (size_t)hyb::Brick<hyb::kI8>::storage((int)N) : 0;
    std::vector<float> b32(grid.empty() ? 0 : n32, 0.0f);
    std::vector<_Float16> b16(g16.empty() ? 0 : n16, (_Float16)0.0f);
    std::vector<int8_t> b8(scales.empty() ? 0 : n8, 0);
    int i, j, k;
    for (size_t s = 0; s < b32.size(); ++s)
        if (hyb::Brick<hyb::kF32>::slot_node((int64_t)s, (int)N, i, j, k)) b32[s] = grid.at(i + N * (j + N * (long long)k));
    for (size_t s = 0; s < b16.size(); ++s)
        if (fmt == 3 ? hyb::Brick<hyb::kF16B2>::slot_node((int64_t)s, (int)N, i, j, k)
                     : hyb::Brick<hyb::kF16>::slot_node((int64_t)s, (int)N, i, j, k))
            b16[s] = g16.at(i + N * (j + N * (long long)k));
    for (size_t s = 0; s < b8.size(); ++s) {
        const long long b = (long long)s / hyb::Brick<hyb::kI8>::kStride, nc = N - 1;
        const int r = (int)((long long)s - b * hyb::Brick<hyb::kI8>::kStride);
        const long long ci = b % nc, cj = (b / nc) % nc, ck = b / (nc * nc);
        const float sc = scales.at(ci / 8 + nb * (cj / 8 + nb * (ck / 8)));
        if (r >= hyb::Brick<hyb::kI8>::kNodes) {  // the cell's scale after its codes
            uint32_t bits;
            std::memcpy(&bits, &sc, 4);
            b8[s] = (int8_t)(uint8_t)(bits >> (8 * (r - hyb::Brick<hyb::kI8>::kNodes)));
        } else if (hyb::Brick<hyb::kI8>::slot_node((int64_t)s, (int)N, i, j, k)) {
            const float q = grid.at(i + N * (j + N * (long long)k)) / sc;
            if (!(q == (float)(int)q && q >= -127.0f && q <= 127.0f)) return 5;  // not a code of this block
            b8[s] = (int8_t)q;
        }
    }

    std::vector<float> t(n), u(n), v(n);
    std::vector<int32_t> prim(n), counts(3 * n);
    hyb::TraceArgs a{};
    a.ox = rays.data(); a.oy = rays.data() + n; a.oz = rays.data() + 2 * n;
    a.dx = rays.data() + 3 * n; a.dy = rays.data() + 4 * n; a.dz = rays.data() + 5 * n;
    a.tmin = (has_tmin & 1) ? tmin.data() : nullptr;
    a.tmax_ray = (has_tmin & 2) ? tmaxr.data() : nullptr;
    a.tau_end = par[7];
    a.t = t.data(); a.prim = prim.data(); a.u = u.data(); a.v = v.data(); a.counts = counts.data();
    a.nodes = nodes4.data();
    a.entry = bvh.entry_res ? bvh.entry.data() : nullptr;
    a.entry_lo_x = bvh.entry_lo[0];
    a.entry_lo_y = bvh.entry_lo[1];
    a.entry_lo_z = bvh.entry_lo[2];
    a.entry_inv = bvh.entry_res ? 1.0f / bvh.entry_size : 0.0f;
    a.entry_res = bvh.entry_res;
    a.entry_levels = bvh.entry_levels;
    a.tris = tri4.data();
    a.sdf = grid.empty() ? nullptr
            : (fmt == 1 || fmt == 3 ? static_cast<const void*>(b16.data())
                        : (fmt == 2 ? static_cast<const void*>(b8.data()) : static_cast<const void*>(b32.data())));
    a.fmt = fmt;
    a.n_grid = (int)N;
    a.lo_x = par[2]; a.lo_y = par[3]; a.lo_z = par[4]; a.h = par[5]; a.inv_h = inv_h; a.inv_hd = 1.0 / (double)par[5];
    a.inv_l = hyb::inv_step(L);
    a.two_e = (par[6] != 0.0f && fmt == 0) ? hyb::certified_slack(par[5], (int)N) : __builtin_inff();
    a.slope_x = slope[0];
    a.slope_y = slope[1];
    a.slope_z = slope[2];
    a.tmax = par[0];
    a.tau = par[1];
    a.n = n;
    if (what == 2) {
        const hyb::Grid g = {b32.data(), (int)N, par[2], par[3], par[4], par[5], inv_h, a.inv_l,
                             __builtin_inff(), a.slope_x, a.slope_y, a.slope_z, 1.0 / (double)par[5]};
        std::vector<long long> nodes(8 * n, -1);
        std::vector<float> dts(8 * n, 0.0f);
        for (long long i = 0; i < n; ++i) {
            const float t0 = (has_tmin & 1) ? tmin[i] : 0.0f;
            const float t1 = (has_tmin & 2) ? fminf(tmaxr[i], par[0]) : par[0];
            int64_t nd[8];
            float dt[8];
            if (hyb::df_hit_gradient(g, a.ox[i], a.oy[i], a.oz[i], a.dx[i], a.dy[i], a.dz[i], t0, t1, thit[i], nd, dt))
                for (int c = 0; c < 8; ++c) { nodes[8 * i + c] = nd[c]; dts[8 * i + c] = dt[c]; }
        }
        fwrite(nodes.data(), 8, 8 * n, o);
        fwrite(dts.data(), 4, 8 * n, o);
        fclose(o);
        return 0;
    }
    std::vector<int> stack(hyb::kLdsDepth);
    for (long long i = 0; i < n; ++i) {
        if (mode == 1) hyb::trace_ray<hyb::kBvhOnly, hyb::kF32, true>(a, i, stack.data(), 1);
        else if (mode == 3) hyb::trace_ray<hyb::kShadow, hyb::kF32, true>(a, i, stack.data(), 1);
        else if (fmt == 1) {
            if (mode == 0) hyb::trace_ray<hyb::kCombined, hyb::kF16, true>(a, i, stack.data(), 1);
            else hyb::trace_ray<hyb::kDfOnly, hyb::kF16, true>(a, i, stack.data(), 1);
        } else if (fmt == 3) {
            if (mode == 0) hyb::trace_ray<hyb::kCombined, hyb::kF16B2, true>(a, i, stack.data(), 1);
            else hyb::trace_ray<hyb::kDfOnly, hyb::kF16B2, true>(a, i, stack.data(), 1);
        } else if (fmt == 2) {
            if (mode == 0) hyb::trace_ray<hyb::kCombined, hyb::kI8, true>(a, i, stack.data(), 1);
            else hyb::trace_ray<hyb::kDfOnly, hyb::kI8, true>(a, i, stack.data(), 1);
        } else {
            if (mode == 0) hyb::trace_ray<hyb::kCombined, hyb::kF32, true>(a, i, stack.data(), 1);
            else hyb::trace_ray<hyb::kDfOnly, hyb::kF32, true>(a, i, stack.data(), 1);
        }
    }
    fwrite(t.data(), 4, n, o);
    fwrite(prim.data(), 4, n, o);
    fwrite(u.data(), 4, n, o);
    fwrite(v.data(), 4, n, o);
    fwrite(counts.data(), 4, 3 * n, o);
    fclose(o);
    return 0;
}
