// Compile-time geometry of the Freudenthal (Kuhn) triangulated grid, for the GPU kernels.
//
// Cells are {a, a+c1, ..., a+cd}: anchor a (componentwise minimum vertex) plus a strictly
// increasing chain of direction bit sets (bit 0 = +x, 1 = +y, 2 = +z).  Cell types of each
// dimension are the chains in lexicographic order of their bit values.
//
// Gradient codes are stored per cell type in planes (structure of arrays): plane p holds
// the code byte of the cell of type byte p anchored at every vertex.  Byte layout:
//   2D: 0 vertex | 1..3 edges | 4..5 triangles                    (6 planes)
//   3D: 0 vertex | 1..7 edges | 8..19 triangles | 20..25 tetrahedra (26 planes)
// Code byte: 0x00 critical; 0x40|c paired with the cofacet that adds vertex anchor+off(c);
// 0x80|c paired with the facet that drops vertex anchor+off(c); 0xFF not written.
// c = 13 + dx + 3*dy + 9*dz encodes an offset in {-1,0,1}^3 from the cell's anchor.
//
// The vertex star: a vertex v has NS = 2*(2^D - 1) neighbours, the offsets +-c for every
// nonzero c in {0,1}^D.  Slot s < NS/2 holds -c with c = NS/2 - s, slot s >= NS/2 holds +c
// with c = s - NS/2 + 1, so slot order is linear-id order (for nx, ny >= 2).
#pragma once
#include <stdint.h>

namespace dmt {

constexpr int popc3(int x) { return (x & 1) + ((x >> 1) & 1) + ((x >> 2) & 1); }
constexpr int c27_of(int dx, int dy, int dz) { return 13 + dx + 3 * dy + 9 * dz; }

template <int D>
struct Geom {
    static constexpr int FULL = (1 << D) - 1;
    static constexpr int NS = 2 * FULL;
    static constexpr int NB = D == 2 ? 6 : 26;       // planes (cell types incl. the vertex)
    static constexpr int NTRI = D == 2 ? 6 : 36;     // triangles in a vertex star
    static constexpr int NTET = D == 2 ? 0 : 24;     // tetrahedra in a vertex star

    int ntypes[4];
    int chain[4][12][3];
    int base[4];                 // first plane of each dimension
    // per plane
    int bdim[26];
    int bnv[26];                 // number of vertices
    int bvert[26][4][3];         // vertex offsets (chain order, [0] = anchor)
    int bmax[26][3];             // componentwise max offset (existence test)
    int facet_anchor[26][4][3];  // facet dropping vertex k: anchor offset ...
    int facet_plane[26][4];      // ... and plane
    int nbr_anchor[26][4][3];    // top cells: the other top cell through facet k
    int nbr_plane[26][4];
    int cof_n[26];               // (D-1)-cells: top-dimensional cofacets
    int cof_anchor[26][2][3];
    int cof_plane[26][2];
    int chain_plane[8][8][8];    // plane of the cell with chain (c1, c2, c3) (0 = unused), -1 none
    int ncofall[26];             // every cofacet of a cell: anchor offset, plane, and the apex it adds
    int cofall_anchor[26][14][3];
    int cofall_plane[26][14];
    int cofall_apex[26][14];     // apex as c27 relative to the cell's anchor
    // vertex star
    int slot_d[14][3];
    int edge_anchor_slot[14];    // -1: anchored at v itself
    int edge_plane[14];
    int tri_s[36], tri_t[36], tri_anchor_slot[36], tri_plane[36];
    int tet_s[24], tet_t[24], tet_u[24], tet_anchor_slot[24], tet_plane[24];
    int tri_index[14][14];
    uint32_t edge_trimask[14];   // apex slots of the star triangles on edge (v, s)
    uint32_t tri_tetmask[36];    // apex slots of the star tetrahedra on triangle (v, s, t)
    // anchors whose cells contain a vertex of the closed 1-ring of v (offsets from v)
    int naff;
    int aff_d[64][3];
};

template <int D>
constexpr void bits_to_d(int b, int out[3]) {
    out[0] = b & 1;
    out[1] = (b >> 1) & 1;
    out[2] = D == 3 ? ((b >> 2) & 1) : 0;
}

template <int D>
constexpr Geom<D> make_geom() {
    Geom<D> g{};
    constexpr int FULL = Geom<D>::FULL;
    constexpr int NS = Geom<D>::NS;
    // ---- cell types: chains 0 < c1 < ... < cd, lexicographic
    g.ntypes[0] = 1;
    for (int d = 1; d <= D; d++) {
        int nt = 0;
        for (int c1 = 1; c1 <= FULL; c1++) {
            if (d == 1) { g.chain[1][nt][0] = c1; nt++; continue; }
            for (int c2 = c1 + 1; c2 <= FULL; c2++) {
                if ((c1 & ~c2) != 0) continue;
                if (d == 2) { g.chain[2][nt][0] = c1; g.chain[2][nt][1] = c2; nt++; continue; }
                for (int c3 = c2 + 1; c3 <= FULL; c3++) {
                    if ((c2 & ~c3) != 0) continue;
                    g.chain[3][nt][0] = c1; g.chain[3][nt][1] = c2; g.chain[3][nt][2] = c3; nt++;
                }
            }
        }
        g.ntypes[d] = nt;
    }
    for (int d = D + 1; d < 4; d++) g.ntypes[d] = 0;
    int p = 0;
    for (int d = 0; d <= D; d++) {
        g.base[d] = p;
        for (int t = 0; t < g.ntypes[d]; t++, p++) {
            g.bdim[p] = d;
            g.bnv[p] = d + 1;
            int b[3] = {0, 0, 0};
            for (int k = 0; k < 3; k++) g.bvert[p][0][k] = 0;
            for (int i = 0; i < d; i++) {
                bits_to_d<D>(g.chain[d][t][i], b);
                for (int k = 0; k < 3; k++) g.bvert[p][i + 1][k] = b[k];
            }
            for (int k = 0; k < 3; k++) g.bmax[p][k] = g.bvert[p][d][k];
        }
    }
    for (int i = 0; i < 8; i++)
        for (int j = 0; j < 8; j++)
            for (int k = 0; k < 8; k++) g.chain_plane[i][j][k] = -1;
    g.chain_plane[0][0][0] = 0;
    for (int d = 1; d <= D; d++)
        for (int t = 0; t < g.ntypes[d]; t++) {
            int c1 = g.chain[d][t][0], c2 = d > 1 ? g.chain[d][t][1] : 0, c3 = d > 2 ? g.chain[d][t][2] : 0;
            g.chain_plane[c1][c2][c3] = g.base[d] + t;
        }
    // ---- facets: drop vertex k, re-anchor at the smallest remaining vertex
    for (int q = 0; q < Geom<D>::NB; q++) {
        int d = g.bdim[q];
        for (int k = 0; k <= d; k++) {
            if (d == 0) { g.facet_plane[q][k] = -1; continue; }
            int first = k == 0 ? 1 : 0;
            int cs[3] = {0, 0, 0};
            int m = 0;
            for (int i = 0; i <= d; i++) {
                if (i == k || i == first) continue;
                int bb = 0;
                for (int ax = 0; ax < 3; ax++) bb |= (g.bvert[q][i][ax] - g.bvert[q][first][ax]) << ax;
                cs[m++] = bb;
            }
            for (int ax = 0; ax < 3; ax++) g.facet_anchor[q][k][ax] = g.bvert[q][first][ax];
            g.facet_plane[q][k] = g.chain_plane[cs[0]][cs[1]][cs[2]];
        }
    }
    // ---- top cells: neighbour through facet k; (D-1)-cells: their top cofacets
    for (int q = 0; q < Geom<D>::NB; q++) {
        int d = g.bdim[q];
        g.cof_n[q] = 0;
        for (int k = 0; k <= d; k++) { g.nbr_plane[q][k] = -1; }
        if (d != D && d != D - 1) continue;
        // search top cells anchored at offsets in {-1,0,1}^D
        for (int az = (D == 3 ? -1 : 0); az <= (D == 3 ? 1 : 0); az++)
            for (int ay = -1; ay <= 1; ay++)
                for (int ax = -1; ax <= 1; ax++)
                    for (int t = 0; t < g.ntypes[D]; t++) {
                        int tp = g.base[D] + t;
                        int A[3] = {ax, ay, az};
                        // vertices of candidate top cell relative to q's anchor
                        int cv[4][3] = {};
                        for (int i = 0; i <= D; i++)
                            for (int c = 0; c < 3; c++) cv[i][c] = A[c] + g.bvert[tp][i][c];
                        if (d == D) {
                            if (ax == 0 && ay == 0 && az == 0 && tp == q) continue;
                            for (int k = 0; k <= D; k++) {
                                // does the candidate contain every vertex of q except k?
                                int all = 1;
                                for (int i = 0; i <= D; i++) {
                                    if (i == k) continue;
                                    int found = 0;
                                    for (int j = 0; j <= D; j++) {
                                        int eq = 1;
                                        for (int c = 0; c < 3; c++) eq &= cv[j][c] == g.bvert[q][i][c];
                                        found |= eq;
                                    }
                                    all &= found;
                                }
                                if (all) {
                                    g.nbr_plane[q][k] = tp;
                                    for (int c = 0; c < 3; c++) g.nbr_anchor[q][k][c] = A[c];
                                }
                            }
                        } else {
                            int all = 1;
                            for (int i = 0; i <= d; i++) {
                                int found = 0;
                                for (int j = 0; j <= D; j++) {
                                    int eq = 1;
                                    for (int c = 0; c < 3; c++) eq &= cv[j][c] == g.bvert[q][i][c];
                                    found |= eq;
                                }
                                all &= found;
                            }
                            if (all && g.cof_n[q] < 2) {
                                int n = g.cof_n[q]++;
                                g.cof_plane[q][n] = tp;
                                for (int c = 0; c < 3; c++) g.cof_anchor[q][n][c] = A[c];
                            }
                        }
                    }
    }
    // ---- every cofacet of every plane (cells anchored at offsets in {-1,0,1}^D)
    for (int q = 0; q < Geom<D>::NB; q++) {
        int d = g.bdim[q];
        g.ncofall[q] = 0;
        if (d == D) continue;
        for (int az = (D == 3 ? -1 : 0); az <= (D == 3 ? 1 : 0); az++)
            for (int ay = -1; ay <= 1; ay++)
                for (int ax = -1; ax <= 1; ax++)
                    for (int t = 0; t < g.ntypes[d + 1]; t++) {
                        int tp = g.base[d + 1] + t;
                        int A[3] = {ax, ay, az};
                        int cv[4][3] = {};
                        for (int i = 0; i <= d + 1; i++)
                            for (int c = 0; c < 3; c++) cv[i][c] = A[c] + g.bvert[tp][i][c];
                        int all = 1;
                        for (int i = 0; i <= d; i++) {
                            int found = 0;
                            for (int j = 0; j <= d + 1; j++) {
                                int eq = 1;
                                for (int c = 0; c < 3; c++) eq &= cv[j][c] == g.bvert[q][i][c];
                                found |= eq;
                            }
                            all &= found;
                        }
                        if (!all) continue;
                        int apex = -1;
                        for (int j = 0; j <= d + 1; j++) {
                            int inq = 0;
                            for (int i = 0; i <= d; i++) {
                                int eq = 1;
                                for (int c = 0; c < 3; c++) eq &= cv[j][c] == g.bvert[q][i][c];
                                inq |= eq;
                            }
                            if (!inq) apex = c27_of(cv[j][0], cv[j][1], cv[j][2]);
                        }
                        int n = g.ncofall[q]++;
                        for (int c = 0; c < 3; c++) g.cofall_anchor[q][n][c] = A[c];
                        g.cofall_plane[q][n] = tp;
                        g.cofall_apex[q][n] = apex;
                    }
    }
    // ---- vertex star
    for (int s = 0; s < NS; s++) {
        int c = s < FULL ? FULL - s : s - FULL + 1;
        int sg = s < FULL ? -1 : 1;
        int b[3] = {0, 0, 0};
        bits_to_d<D>(c, b);
        for (int k = 0; k < 3; k++) g.slot_d[s][k] = sg * b[k];
    }
    for (int i = 0; i < NS; i++)
        for (int j = 0; j < NS; j++) g.tri_index[i][j] = -1;
    int ntri = 0, ntet = 0;
    for (int ac = 0; ac <= FULL; ac++) {             // anchor = -bits(ac)
        int A[3] = {0, 0, 0};
        bits_to_d<D>(ac, A);
        for (int k = 0; k < 3; k++) A[k] = -A[k];
        int aslot = ac == 0 ? -1 : FULL - ac;
        for (int d = 1; d <= D; d++) {
            for (int t = 0; t < g.ntypes[d]; t++) {
                int pl = g.base[d] + t;
                int hasv = 0;
                int slots[4] = {0, 0, 0, 0};
                int ns = 0;
                for (int i = 0; i <= d; i++) {
                    int V[3] = {0, 0, 0};
                    for (int k = 0; k < 3; k++) V[k] = A[k] + g.bvert[pl][i][k];
                    if (V[0] == 0 && V[1] == 0 && V[2] == 0) { hasv = 1; continue; }
                    for (int s = 0; s < NS; s++)
                        if (g.slot_d[s][0] == V[0] && g.slot_d[s][1] == V[1] && g.slot_d[s][2] == V[2])
                            slots[ns] = s;
                    ns++;
                }
                if (!hasv) continue;
                // sort slots ascending
                for (int i = 0; i < ns; i++)
                    for (int j = i + 1; j < ns; j++)
                        if (slots[j] < slots[i]) { int tmp = slots[i]; slots[i] = slots[j]; slots[j] = tmp; }
                if (d == 1) {
                    g.edge_anchor_slot[slots[0]] = aslot;
                    g.edge_plane[slots[0]] = pl;
                } else if (d == 2) {
                    g.tri_s[ntri] = slots[0]; g.tri_t[ntri] = slots[1];
                    g.tri_anchor_slot[ntri] = aslot; g.tri_plane[ntri] = pl;
                    g.tri_index[slots[0]][slots[1]] = ntri;
                    g.tri_index[slots[1]][slots[0]] = ntri;
                    g.edge_trimask[slots[0]] |= 1u << slots[1];
                    g.edge_trimask[slots[1]] |= 1u << slots[0];
                    ntri++;
                } else {
                    g.tet_s[ntet] = slots[0]; g.tet_t[ntet] = slots[1]; g.tet_u[ntet] = slots[2];
                    g.tet_anchor_slot[ntet] = aslot; g.tet_plane[ntet] = pl;
                    ntet++;
                }
            }
        }
    }
    // affected anchors: d = o - c, o in the closed 1-ring offsets, c in {0,1}^D
    g.naff = 0;
    for (int dz = (D == 3 ? -2 : 0); dz <= (D == 3 ? 1 : 0); dz++)
        for (int dy = -2; dy <= 1; dy++)
            for (int dx = -2; dx <= 1; dx++) {
                int hit = 0;
                for (int s = -1; s < NS; s++) {
                    int o[3] = {0, 0, 0};
                    if (s >= 0) for (int k = 0; k < 3; k++) o[k] = g.slot_d[s][k];
                    for (int cb = 0; cb <= FULL; cb++) {
                        int c[3] = {0, 0, 0};
                        bits_to_d<D>(cb, c);
                        if (o[0] - c[0] == dx && o[1] - c[1] == dy && o[2] - c[2] == dz) hit = 1;
                    }
                }
                if (hit) {
                    g.aff_d[g.naff][0] = dx; g.aff_d[g.naff][1] = dy; g.aff_d[g.naff][2] = dz;
                    g.naff++;
                }
            }
    for (int i = 0; i < ntet; i++) {
        int s = g.tet_s[i], t = g.tet_t[i], u = g.tet_u[i];
        g.tri_tetmask[g.tri_index[s][t]] |= 1u << u;
        g.tri_tetmask[g.tri_index[s][u]] |= 1u << t;
        g.tri_tetmask[g.tri_index[t][u]] |= 1u << s;
    }
    return g;
}

template <int D>
struct G {
    static constexpr Geom<D> g = make_geom<D>();
};

}  // namespace dmt
