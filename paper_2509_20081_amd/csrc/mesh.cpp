// Marching Cubes case table of the mesh export (host side).
//
// The paper exports the fused map as a mesh by Marching Cubes at iso = 0.0
// (the export block of its pipeline figure, Sec. III). The table below fixes
// the triangles of every corner case from these rules:
//   - a corner is inside when its signed distance is negative;
//   - edges are numbered 4 a + r (axis a, r the rank of the lower corner
//     among the four corners whose bit a is clear), corners c = x + 2 y + 4 z;
//   - on every face, taken counter-clockwise as seen from outside the cube,
//     each run of inside corners gives a segment from the crossed edge where
//     the run starts to the one where it ends (on a saddle face, with inside
//     corners on a diagonal, each inside corner is its own run, so two cubes
//     sharing the face draw the same segments and the surface is closed);
//   - segments chain into loops, each started at its smallest edge number;
//     a loop is fanned from that edge, unless it holds all four crossed edges
//     of a saddle face: then the fan's chords could lie in that face, and the
//     loop is fanned from its centre instead (the mean of its vertices).
// Triangles so wound have their normals towards positive distance.
#include <algorithm>
#include <mutex>

#include "internal.h"

namespace dbtsdf {

namespace {

int corner_bit(int c, int axis) { return (c >> axis) & 1; }

// number of the edge between corners c0 and c1 (which differ in one bit)
int edge_of(int c0, int c1) {
    const int lo = std::min(c0, c1), diff = c0 ^ c1;
    const int axis = diff == 1 ? 0 : diff == 2 ? 1 : 2;
    int rank = 0;
    for (int c = 0; c < lo; ++c)
        if (!corner_bit(c, axis)) ++rank;
    return 4 * axis + rank;
}

// the four corners of face (axis a, side v), counter-clockwise about its outward normal
void face_ring(int a, int v, int ring[4]) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;   // e_b x e_c = e_a
    static const int up[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
    static const int down[4][2] = {{0, 0}, {0, 1}, {1, 1}, {1, 0}};
    for (int i = 0; i < 4; ++i) {
        const int *p = v ? up[i] : down[i];
        ring[i] = (v << a) | (p[0] << b) | (p[1] << c);
    }
}

void build_case(int cs, uint8_t *out) {
    int next[12];
    std::fill(next, next + 12, -1);
    bool saddle_edges[6][12] = {};
    int n_saddle = 0;
    for (int a = 0; a < 3; ++a)
        for (int v = 0; v < 2; ++v) {
            int ring[4];
            face_ring(a, v, ring);
            int in[4];
            for (int i = 0; i < 4; ++i) in[i] = (cs >> ring[i]) & 1;
            if ((in[0] && in[2] && !in[1] && !in[3]) || (in[1] && in[3] && !in[0] && !in[2])) {
                for (int i = 0; i < 4; ++i) saddle_edges[n_saddle][edge_of(ring[i], ring[(i + 1) % 4])] = true;
                ++n_saddle;
            }
            for (int i = 0; i < 4; ++i) {
                if (!in[i] || in[(i + 3) % 4]) continue;   // not the start of an inside run
                int j = i;
                while (in[(j + 1) % 4] && (j + 1) % 4 != i) j = (j + 1) % 4;
                next[edge_of(ring[(i + 3) % 4], ring[i])] = edge_of(ring[j], ring[(j + 1) % 4]);
            }
        }
    int n_tris = 0, n_loops = 0, pos = 2;
    bool used[12] = {};
    for (int e0 = 0; e0 < 12; ++e0) {
        if (next[e0] < 0 || used[e0]) continue;
        // e0 is the smallest unused edge, so the smallest of its loop
        int loop[12], m = 0;
        for (int e = e0; !used[e]; e = next[e]) {
            used[e] = true;
            loop[m++] = e;
        }
        bool centred = false;
        for (int f = 0; f < n_saddle && !centred; ++f) {
            int hit = 0;
            for (int i = 0; i < m; ++i) hit += saddle_edges[f][loop[i]] ? 1 : 0;
            centred = hit == 4;
        }
        out[pos++] = (uint8_t)(m | (centred ? 16 : 0));
        for (int i = 0; i < m; ++i) out[pos++] = (uint8_t)loop[i];
        n_tris += centred ? m : m - 2;
        ++n_loops;
    }
    out[0] = (uint8_t)n_tris;
    out[1] = (uint8_t)n_loops;
}

// The case's triangles one by one: a loop fanned from its first edge gives
// (e_0, e_(w-1), e_w) for w = 2 .. m-1, one fanned from its centre C gives
// (C, e_w, e_(w+1 mod m)) for w = 0 .. m-1.
void list_triangles(const uint8_t *cs, uint8_t *tri) {
    int pos = 2, t = 0;
    for (int L = 0; L < cs[1]; ++L) {
        const int hdr = pos, m = cs[pos] & 15;
        const uint8_t *e = cs + pos + 1;
        if (cs[pos] & 16) {
            for (int w = 0; w < m; ++w, ++t) {
                tri[3 * t + 0] = (uint8_t)(kMeshCentre | hdr);
                tri[3 * t + 1] = e[w];
                tri[3 * t + 2] = e[(w + 1) % m];
            }
        } else {
            for (int w = 2; w < m; ++w, ++t) {
                tri[3 * t + 0] = e[0];
                tri[3 * t + 1] = e[w - 1];
                tri[3 * t + 2] = e[w];
            }
        }
        pos += 1 + m;
    }
}

}  // namespace

const MeshTable &mesh_table() {
    static MeshTable t;
    static std::once_flag once;
    std::call_once(once, [] {
        for (int cs = 0; cs < 256; ++cs) {
            std::fill(t.b[cs], t.b[cs] + kMeshCaseBytes, (uint8_t)0);
            std::fill(t.tri[cs], t.tri[cs] + kMeshTriBytes, (uint8_t)0);
            build_case(cs, t.b[cs]);
            list_triangles(t.b[cs], t.tri[cs]);
        }
    });
    return t;
}

}  // namespace dbtsdf
