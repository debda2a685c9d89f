// ptm_tables.hpp -- template tables of the HIP library (host-built, device
// read-only).  Polyhedral Template Matching, arXiv:1603.05143: the ideal
// templates of Table 1, their hull triangulations (Sec. 4, App. A), the
// orientation-preserving start-edge codes of those triangulations (the
// graph-isomorphism keys of Sec. 4) and the candidate correspondences, one
// per orbit of the template's proper rotation group (App. A: symmetrically
// equivalent correspondences give the same RMSD).
#pragma once
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

namespace ptm {

constexpr int NT = 5;    // templates SC, FCC, HCP, ICO, BCC
constexpr int KMAX = 14; // largest neighbour shell (BCC, Table 1)
constexpr int NMAX = KMAX + 1;
constexpr int NGRP = 3;  // hull sizes k = 6, 12, 14
constexpr int GMAX = 60; // largest rotation group (ICO)

__host__ __device__ constexpr int template_k(int t) { return t == 0 ? 6 : (t == 4 ? 14 : 12); }
__host__ __device__ constexpr int group_k(int g) { return g == 0 ? 6 : (g == 1 ? 12 : 14); }
__host__ __device__ constexpr int group_of_template(int t) { return t == 0 ? 0 : (t == 4 ? 2 : 1); }

// Per-template constants used by the match kernel.
struct TemplateDev {
    int k;
    int ngroup;
    int pad0, pad1;
    double b[NMAX][3];      // eq.(4)-normalised points, row 0 = centre, row j+1 = vertex j
    double vpinv[3][NMAX];  // Moore-Penrose pseudoinverse of b (3 x N), eq.(6)
    uint64_t ginv[GMAX];    // nibble m = g^-1(m) for every group element g
    double gq[GMAX][4];     // unit quaternion (w,x,y,z) of R_g, R_g w_j = w_{g(j)}
};

struct Candidate {
    uint64_t perm; // nibble l = template vertex of canonical label l
    int32_t tmpl;  // template index 0..4
    int32_t pad;
};

// Device view of the tables: plain pointers, passed to kernels by value.
struct TablesView {
    const TemplateDev *tpl;               // [NT]
    const uint64_t *codes[NGRP];          // [ncodes][k] canonical code rows
    const int32_t *slots[NGRP];           // [hmask+1] code id or -1
    const int32_t *cstart[NGRP];          // [ncodes+1] candidate ranges
    const Candidate *cand[NGRP];          // candidates
    int32_t hmask[NGRP];
    int32_t ncodes[NGRP];
};

// Host-side tables.
struct HostTables {
    TemplateDev tpl[NT];
    std::vector<uint64_t> codes[NGRP];
    std::vector<int32_t> slots[NGRP];
    std::vector<int32_t> cstart[NGRP];
    std::vector<Candidate> cand[NGRP];
    int32_t hmask[NGRP];
    int32_t ncodes[NGRP];
    int64_t ntri[NT];        // triangulations per template
    int64_t ncand_full[NT];  // table correspondences before symmetry reduction
    int64_t ncand_kept[NT];  // after
    int64_t ncodes_t[NT];    // distinct table keys (start-edge codes) per template
    int max_cand_per_code[NGRP];
};

// Hash of a code (k row words); used identically by host and device.
__host__ __device__ inline uint64_t code_hash(const uint64_t *rows, int k) {
    uint64_t h = 0x243F6A8885A308D3ull;
    for (int i = 0; i < k; i++) {
        h ^= rows[i];
        h *= 0x9E3779B97F4A7C15ull;
        h ^= h >> 29;
    }
    return h;
}

// Build all tables; returns false and sets err on failure.
bool build_tables(HostTables &T, std::string &err);

// Start-edge codes (definition in ptm_tables.cpp) of a rotation system
// given by nxt[x] (nibble y = vertex after y counter-clockwise around x,
// 0xF = none) and deg.  Host versions used by the generator and by the
// self-check entry points.
uint64_t dart_signature(int k, const uint64_t *nxt, const int *deg, int u, int v);
void dart_code(int k, const uint64_t *nxt, const int *deg, int u, int v, uint64_t *rows, uint64_t *ordp);
std::vector<std::pair<int, int>> min_degree_darts(int k, const uint64_t *nxt, const int *deg);

} // namespace ptm
