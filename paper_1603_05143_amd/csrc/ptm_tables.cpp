// ptm_tables.cpp -- host construction of the template tables.
//
// Templates (Table 1; coordinates and vertex numbering fixed by the output
// convention): ideal SC, FCC, HCP (c/a = sqrt(8/3)), ICO and BCC shells.
// For each template:
//   * proper rotation group by closure of known generators (orders 24, 24,
//     6, 60, 24; Sec. 4);
//   * hull faces (triangles, squares, rhombi) of the ideal shell and every
//     triangulation, two diagonals per four-point face (Sec. 4: 2^6 for FCC
//     and HCP, both triangulations of each BCC rhombus);
//   * the canonical code of every triangulation and all labellings reaching
//     it (its orientation-preserving automorphisms);
//   * candidates: canonical label -> template vertex maps, one per orbit of
//     the rotation group (App. A: symmetrically inequivalent
//     correspondences only).
// Codes shared between templates (FCC/HCP/ICO, Sec. 4) share one table
// entry whose candidate list spans the templates.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <set>

#include "ptm_tables.hpp"

namespace ptm {
namespace {

struct V3 {
    double x, y, z;
};
V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
V3 operator*(double s, V3 a) { return {s * a.x, s * a.y, s * a.z}; }
double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
V3 cross(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
double norm(V3 a) { return std::sqrt(dot(a, a)); }

struct M3 {
    double m[3][3];
};
M3 mul(const M3 &a, const M3 &b) {
    M3 c;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            c.m[i][j] = 0;
            for (int k = 0; k < 3; k++) c.m[i][j] += a.m[i][k] * b.m[k][j];
        }
    return c;
}
V3 apply(const M3 &a, V3 v) {
    return {a.m[0][0] * v.x + a.m[0][1] * v.y + a.m[0][2] * v.z,
            a.m[1][0] * v.x + a.m[1][1] * v.y + a.m[1][2] * v.z,
            a.m[2][0] * v.x + a.m[2][1] * v.y + a.m[2][2] * v.z};
}
// rotation by angle about a unit axis (Rodrigues)
M3 axis_angle(V3 u, double ang) {
    double n = norm(u);
    u = (1.0 / n) * u;
    double c = std::cos(ang), s = std::sin(ang), t = 1 - c;
    M3 r = {{{t * u.x * u.x + c, t * u.x * u.y - s * u.z, t * u.x * u.z + s * u.y},
             {t * u.x * u.y + s * u.z, t * u.y * u.y + c, t * u.y * u.z - s * u.x},
             {t * u.x * u.z - s * u.y, t * u.y * u.z + s * u.x, t * u.z * u.z + c}}};
    return r;
}

std::vector<V3> template_points(int t) {
    std::vector<V3> w;
    const double PI = 3.14159265358979323846;
    if (t == 0) {
        w = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    } else if (t == 1) {
        w = {{1, 1, 0}, {1, -1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, 0, 1}, {1, 0, -1},
             {-1, 0, 1}, {-1, 0, -1}, {0, 1, 1}, {0, 1, -1}, {0, -1, 1}, {0, -1, -1}};
    } else if (t == 2) {
        for (int m = 0; m < 6; m++) w.push_back({std::cos(PI * m / 3), std::sin(PI * m / 3), 0.0});
        const double r = 1 / std::sqrt(3.0), h = std::sqrt(2.0 / 3.0);
        for (int s = 0; s < 2; s++)
            for (int j = 0; j < 3; j++) {
                double a = PI / 6 + 2 * PI * j / 3;
                w.push_back({r * std::cos(a), r * std::sin(a), s == 0 ? h : -h});
            }
    } else if (t == 3) {
        const double p = (1 + std::sqrt(5.0)) / 2;
        w = {{0, 1, p}, {0, 1, -p}, {0, -1, p}, {0, -1, -p}, {1, p, 0}, {1, -p, 0},
             {-1, p, 0}, {-1, -p, 0}, {p, 0, 1}, {p, 0, -1}, {-p, 0, 1}, {-p, 0, -1}};
    } else {
        w = {{1, 1, 1},   {1, 1, -1},  {1, -1, 1},  {1, -1, -1}, {-1, 1, 1},
             {-1, 1, -1}, {-1, -1, 1}, {-1, -1, -1}, {2, 0, 0},   {-2, 0, 0},
             {0, 2, 0},   {0, -2, 0},  {0, 0, 2},   {0, 0, -2}};
    }
    return w;
}

// generators of the proper rotation group of each template
std::vector<M3> generators(int t) {
    const double PI = 3.14159265358979323846;
    if (t == 2)  // HCP: 3-fold about c, 2-fold about the in-plane axis at 30 degrees
        return {axis_angle({0, 0, 1}, 2 * PI / 3), axis_angle({std::cos(PI / 6), std::sin(PI / 6), 0}, PI)};
    if (t == 3) {  // ICO: 5-fold through a vertex, 3-fold through (1,1,1), 2-fold about z
        const double p = (1 + std::sqrt(5.0)) / 2;
        return {axis_angle({0, 1, p}, 2 * PI / 5), axis_angle({1, 1, 1}, 2 * PI / 3),
                axis_angle({0, 0, 1}, PI)};
    }
    return {axis_angle({1, 0, 0}, PI / 2), axis_angle({0, 1, 0}, PI / 2)};  // cubic
}

bool same(const M3 &a, const M3 &b) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (std::fabs(a.m[i][j] - b.m[i][j]) > 1e-9) return false;
    return true;
}

std::vector<M3> close_group(const std::vector<M3> &gen) {
    M3 id = {{{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}};
    std::vector<M3> G = {id};
    for (size_t i = 0; i < G.size(); i++)
        for (const M3 &g : gen) {
            M3 h = mul(g, G[i]);
            bool found = false;
            for (const M3 &e : G)
                if (same(e, h)) { found = true; break; }
            if (!found) G.push_back(h);
            if (G.size() > 200) return G;
        }
    return G;
}

int find_vertex(const std::vector<V3> &w, V3 p) {
    for (size_t j = 0; j < w.size(); j++)
        if (norm(w[j] - p) < 1e-9) return (int)j;
    return -1;
}

void mat_to_quat(const M3 &R, double q[4]) {
    const double (*r)[3] = R.m;
    double tr = r[0][0] + r[1][1] + r[2][2];
    if (tr > 0) {
        double s = std::sqrt(tr + 1.0) * 2;
        q[0] = 0.25 * s; q[1] = (r[2][1] - r[1][2]) / s; q[2] = (r[0][2] - r[2][0]) / s; q[3] = (r[1][0] - r[0][1]) / s;
    } else if (r[0][0] > r[1][1] && r[0][0] > r[2][2]) {
        double s = std::sqrt(1.0 + r[0][0] - r[1][1] - r[2][2]) * 2;
        q[0] = (r[2][1] - r[1][2]) / s; q[1] = 0.25 * s; q[2] = (r[0][1] + r[1][0]) / s; q[3] = (r[0][2] + r[2][0]) / s;
    } else if (r[1][1] > r[2][2]) {
        double s = std::sqrt(1.0 + r[1][1] - r[0][0] - r[2][2]) * 2;
        q[0] = (r[0][2] - r[2][0]) / s; q[1] = (r[0][1] + r[1][0]) / s; q[2] = 0.25 * s; q[3] = (r[1][2] + r[2][1]) / s;
    } else {
        double s = std::sqrt(1.0 + r[2][2] - r[0][0] - r[1][1]) * 2;
        q[0] = (r[1][0] - r[0][1]) / s; q[1] = (r[0][2] + r[2][0]) / s; q[2] = (r[1][2] + r[2][1]) / s; q[3] = 0.25 * s;
    }
    double n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int i = 0; i < 4; i++) q[i] /= n;
}

// hull faces of an ideal shell: maximal coplanar vertex sets on supporting
// planes, each listed counter-clockwise seen from outside
std::vector<std::vector<int>> shell_faces(const std::vector<V3> &w) {
    int k = (int)w.size();
    std::set<std::vector<int>> seen;
    std::vector<std::vector<int>> faces;
    for (int i = 0; i < k; i++)
        for (int j = i + 1; j < k; j++)
            for (int l = j + 1; l < k; l++) {
                V3 n = cross(w[j] - w[i], w[l] - w[i]);
                double nn = norm(n);
                if (nn < 1e-9) continue;
                n = (1.0 / nn) * n;
                int pos = 0, neg = 0;
                std::vector<int> on;
                for (int m = 0; m < k; m++) {
                    double s = dot(n, w[m] - w[i]);
                    if (s > 1e-8) pos++;
                    else if (s < -1e-8) neg++;
                    else on.push_back(m);
                }
                if (pos && neg) continue;
                if (!seen.insert(on).second) continue;
                if (pos) n = -1.0 * n;  // make n point outward
                V3 c = {0, 0, 0};
                for (int m : on) c = c + w[m];
                c = (1.0 / on.size()) * c;
                V3 e1 = w[on[0]] - c;
                e1 = (1.0 / norm(e1)) * e1;
                V3 e2 = cross(n, e1);
                std::sort(on.begin(), on.end(), [&](int a, int b) {
                    return std::atan2(dot(w[a] - c, e2), dot(w[a] - c, e1)) <
                           std::atan2(dot(w[b] - c, e2), dot(w[b] - c, e1));
                });
                faces.push_back(on);
            }
    return faces;
}

}  // namespace

// Start-edge code of a triangulated sphere, from a directed edge u->v.
//   word 0 (signature): deg(u) in the top nibble, then deg(v), then the
//     degrees of u's other neighbours in counter-clockwise order after v;
//   words 1..k-1 (BFS rows): u gets label 0 and its neighbours labels
//     1..deg(u) counter-clockwise from v; vertices are then processed in
//     label order and vertex x (label i >= 1) emits one row: deg(x) in the
//     top nibble, then the labels of its neighbours counter-clockwise from
//     the vertex that labelled x, new vertices being labelled in that order.
// The words determine the labelled rotation system.  A graph's key set is
// the set of codes of its start edges from vertices of minimum degree;
// isomorphisms preserve degrees and so map such start edges onto each
// other, so the code of any one of them is found in the key set of every
// graph it is isomorphic to (and in no other), and pairing the labellings
// of the two start edges gives the isomorphism.  The tables hold the key
// sets of all template triangulations; a hull needs the code of a single
// start edge, which the kernel takes without a search.
uint64_t dart_signature(int k, const uint64_t *nxt, const int *deg, int u, int v) {
    (void)k;
    uint64_t sig = ((uint64_t)deg[u] << 60) | ((uint64_t)deg[v] << 56);
    int w = v;
    for (int j = 1; j < deg[u]; j++) {
        w = (int)((nxt[u] >> (4 * w)) & 0xF);
        sig |= (uint64_t)deg[w] << (56 - 4 * j);
    }
    return sig;
}

void dart_code(int k, const uint64_t *nxt, const int *deg, int u, int v, uint64_t *rows, uint64_t *ordp) {
    int lab[KMAX], ord[KMAX], par[KMAX];
    for (int i = 0; i < k; i++) lab[i] = -1;
    lab[u] = 0;
    ord[0] = u;
    int nl = 1, y = v;
    for (int j = 0; j < deg[u]; j++) {
        lab[y] = nl;
        ord[nl] = y;
        par[y] = u;
        nl++;
        y = (int)((nxt[u] >> (4 * y)) & 0xF);
    }
    rows[0] = dart_signature(k, nxt, deg, u, v);
    for (int i = 1; i < k; i++) {
        int x = ord[i];
        y = par[x];
        uint64_t row = (uint64_t)deg[x] << 60;
        for (int j = 0; j < deg[x]; j++) {
            if (lab[y] < 0) {
                lab[y] = nl;
                ord[nl] = y;
                par[y] = x;
                nl++;
            }
            row |= (uint64_t)lab[y] << (56 - 4 * j);
            y = (int)((nxt[x] >> (4 * y)) & 0xF);
        }
        rows[i] = row;
    }
    uint64_t o = 0;
    for (int i = 0; i < k; i++) o |= (uint64_t)ord[i] << (4 * i);
    *ordp = o;
}

// Start edges from the vertices of minimum degree: u ascending, then v
// counter-clockwise around u from its lowest-numbered neighbour.  The first
// one is the start edge the kernel uses.
std::vector<std::pair<int, int>> min_degree_darts(int k, const uint64_t *nxt, const int *deg) {
    int mindeg = KMAX;
    for (int u = 0; u < k; u++) mindeg = std::min(mindeg, deg[u]);
    std::vector<std::pair<int, int>> out;
    for (int u = 0; u < k; u++) {
        if (deg[u] != mindeg) continue;
        int v0 = 0;
        while (v0 < k && ((nxt[u] >> (4 * v0)) & 0xF) == 0xF) v0++;
        if (v0 >= k) continue;
        int v = v0;
        for (int r = 0; r < deg[u]; r++, v = (int)((nxt[u] >> (4 * v)) & 0xF)) out.push_back({u, v});
    }
    return out;
}

bool build_tables(HostTables &T, std::string &err) {
    // per hull group: code (as vector) -> list of (template, perm)
    std::map<std::vector<uint64_t>, std::vector<std::pair<int, uint64_t>>> bucket[NGRP];
    for (int t = 0; t < NT; t++) {
        std::vector<V3> w = template_points(t);
        int k = (int)w.size();
        TemplateDev &D = T.tpl[t];
        std::memset(&D, 0, sizeof D);
        D.k = k;
        // eq.(4) normalisation over the N = k+1 points (centre included)
        V3 c = {0, 0, 0};
        for (V3 p : w) c = c + p;
        c = (1.0 / (k + 1)) * c;
        double l = norm(c);
        for (V3 p : w) l += norm(p - c);
        l /= (k + 1);
        V3 b0 = (-1.0 / l) * c;
        D.b[0][0] = b0.x; D.b[0][1] = b0.y; D.b[0][2] = b0.z;
        for (int j = 0; j < k; j++) {
            V3 bj = (1.0 / l) * (w[j] - c);
            D.b[j + 1][0] = bj.x; D.b[j + 1][1] = bj.y; D.b[j + 1][2] = bj.z;
        }
        // pseudoinverse (B^T B)^-1 B^T
        double g[3][3] = {{0}};
        for (int i = 0; i <= k; i++)
            for (int r = 0; r < 3; r++)
                for (int s = 0; s < 3; s++) g[r][s] += D.b[i][r] * D.b[i][s];
        double det = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
                     g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
                     g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
        double gi[3][3];
        for (int r = 0; r < 3; r++)
            for (int s = 0; s < 3; s++) {
                int r1 = (s + 1) % 3, r2 = (s + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
                gi[r][s] = (g[r1][c1] * g[r2][c2] - g[r1][c2] * g[r2][c1]) / det;
            }
        for (int r = 0; r < 3; r++)
            for (int i = 0; i <= k; i++)
                D.vpinv[r][i] = gi[r][0] * D.b[i][0] + gi[r][1] * D.b[i][1] + gi[r][2] * D.b[i][2];

        // rotation group
        std::vector<M3> G = close_group(generators(t));
        D.ngroup = (int)G.size();
        if (D.ngroup > GMAX) { err = "rotation group too large"; return false; }
        std::vector<std::vector<int>> gperm;
        for (size_t gi2 = 0; gi2 < G.size(); gi2++) {
            std::vector<int> pm(k);
            uint64_t inv = 0;
            for (int j = 0; j < k; j++) {
                pm[j] = find_vertex(w, apply(G[gi2], w[j]));
                if (pm[j] < 0) { err = "generator does not preserve the template"; return false; }
                inv |= (uint64_t)j << (4 * pm[j]);
            }
            D.ginv[gi2] = inv;
            mat_to_quat(G[gi2], D.gq[gi2]);
            gperm.push_back(pm);
        }

        // faces and triangulations
        std::vector<std::vector<int>> faces = shell_faces(w);
        std::vector<int> quads;
        std::vector<std::array<int, 3>> fixed;
        for (size_t f = 0; f < faces.size(); f++) {
            if (faces[f].size() == 3) fixed.push_back({faces[f][0], faces[f][1], faces[f][2]});
            else if (faces[f].size() == 4) quads.push_back((int)f);
            else { err = "unexpected face size"; return false; }
        }
        int nq = (int)quads.size();
        T.ntri[t] = 1ll << nq;
        std::set<std::vector<uint64_t>> codes_t;
        int64_t full = 0;
        for (int64_t s = 0; s < (1ll << nq); s++) {
            std::vector<std::array<int, 3>> tris = fixed;
            for (int q = 0; q < nq; q++) {
                const std::vector<int> &v = faces[quads[q]];
                if ((s >> q) & 1) {
                    tris.push_back({v[1], v[2], v[3]});
                    tris.push_back({v[1], v[3], v[0]});
                } else {
                    tris.push_back({v[0], v[1], v[2]});
                    tris.push_back({v[0], v[2], v[3]});
                }
            }
            uint64_t nxt[KMAX];
            int deg[KMAX] = {0};
            for (int x = 0; x < k; x++) nxt[x] = ~0ull;
            for (auto &tr : tris)
                for (int e = 0; e < 3; e++) {
                    int a = tr[e], bb = tr[(e + 1) % 3], cc = tr[(e + 2) % 3];
                    nxt[a] &= ~(0xFull << (4 * bb));
                    nxt[a] |= (uint64_t)cc << (4 * bb);
                    deg[a]++;
                }
            for (auto &d : min_degree_darts(k, nxt, deg)) {
                uint64_t rows[KMAX], perm;
                dart_code(k, nxt, deg, d.first, d.second, rows, &perm);
                std::vector<uint64_t> key(rows, rows + k);
                codes_t.insert(key);
                full++;
                // canonical orbit representative: smallest g o perm
                uint64_t best = ~0ull;
                for (auto &pm : gperm) {
                    uint64_t img = 0;
                    for (int lb = 0; lb < k; lb++) img |= (uint64_t)pm[(perm >> (4 * lb)) & 0xF] << (4 * lb);
                    best = std::min(best, img);
                }
                bucket[group_of_template(t)][key].push_back({t, best});
            }
        }
        T.ncand_full[t] = full;
        T.ncodes_t[t] = (int64_t)codes_t.size();
    }
    for (int t = 0; t < NT; t++) T.ncand_kept[t] = 0;
    for (int g = 0; g < NGRP; g++) {
        int k = group_k(g);
        T.codes[g].clear();
        T.cand[g].clear();
        T.cstart[g].assign(1, 0);
        T.max_cand_per_code[g] = 0;
        for (auto &kv : bucket[g]) {
            std::vector<std::pair<int, uint64_t>> v = kv.second;
            std::sort(v.begin(), v.end());
            v.erase(std::unique(v.begin(), v.end()), v.end());
            for (auto &pr : v) {
                T.cand[g].push_back({pr.second, pr.first, 0});
                T.ncand_kept[pr.first]++;
            }
            T.max_cand_per_code[g] = std::max(T.max_cand_per_code[g], (int)v.size());
            T.cstart[g].push_back((int32_t)T.cand[g].size());
            T.codes[g].insert(T.codes[g].end(), kv.first.begin(), kv.first.end());
        }
        int nc = (int)bucket[g].size();
        if (nc == 0) {  // the hull kernel reads code row 0 of every group
            err = "template tables: no code for hull size " + std::to_string(k);
            return false;
        }
        if (g == 0 && nc != 1) {  // the hull kernel takes the octahedron's code as code 0
            err = "template tables: more than one code for six points";
            return false;
        }
        T.ncodes[g] = nc;
        int size = 16;
        while (size < 4 * nc) size <<= 1;
        T.hmask[g] = size - 1;
        T.slots[g].assign(size, -1);
        for (int c = 0; c < nc; c++) {
            uint64_t h = code_hash(&T.codes[g][(size_t)c * k], k);
            int s = (int)(h & (uint64_t)(size - 1));
            while (T.slots[g][s] >= 0) s = (s + 1) & (size - 1);
            T.slots[g][s] = c;
        }
    }
    // the full decision superposes all candidates of an atom's three codes
    // with one lane each of a 64-lane wavefront
    if (T.max_cand_per_code[0] + T.max_cand_per_code[1] + T.max_cand_per_code[2] > 64) {
        err = "more than 64 candidate correspondences per atom";
        return false;
    }
    return true;
}

}  // namespace ptm
