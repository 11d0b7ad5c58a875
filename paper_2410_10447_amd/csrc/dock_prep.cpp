// Host-side ligand preparation (see dock_prep.h).
//
// Method context (Sec. 2.1): a pose is {position, orientation, one angle per
// rotatable bond}; the score adds pairwise intramolecular terms. The
// preparation fixes, once per ligand, which atoms each torsion turns, how
// torsions nest, and which atom pairs contribute. Readings used here: the
// moving side of a torsion is the side away from the root atom; pairs are
// kept when >= 4 bonds apart and in different rigid fragments; a pair is a
// hydrogen-bond pair when one atom is a donor class and the other an
// acceptor class.
#include "dock_prep.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace dockprep {
namespace {

constexpr double kElec = 332.06363;   // kcal A / (mol e^2)
constexpr double kQSolv = 0.01097;    // charge term of the solvation parameter

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

int role_index(const int32_t list[2], int c) {
    if (list[0] == c) return 0;
    if (list[1] == c) return 1;
    return -1;
}

// LDS bank spreading of one batch. On gfx950 a wave's 16-byte LDS read is
// served in 4 passes of 16 lanes (see read_pass) over 64 four-byte banks,
// and two lanes of a pass whose different addresses agree mod 16 bank quads
// (address / 16 mod 16) wait for each other; a 16-byte write is served 8
// consecutive lanes at a time, conflicting mod 8 (see place_half). The pair
// loop reads and writes the first and the second atom of each lane's pair
// (position and slot: with a stride that is a multiple of 16 both lie in the
// quad of the atom index, its residue mod 16). The batch's records are
// therefore placed on the lanes, and a pair's two atoms may swap roles, so
// that within each read pass the first atoms' residues differ and so do the
// second atoms'. Seen as a multigraph on the 16 residues with one edge per
// pair, this is an orientation followed by an edge colouring with 4 colours
// (one per read pass): the orientation follows Euler circuits, so each
// residue is first atom about as often as second (|out - in| <= 1), and the
// bipartite (first residue, second residue) multigraph, after setting aside
// the few pairs that push a residue past 4 uses per role, is coloured with 4
// colours by Kempe-chain recolouring (Konig's theorem: a bipartite multigraph
// of maximum degree 4 has a proper 4-edge colouring); the pairs set aside go
// to the passes with room, where they add the fewest repeats. The unused
// lanes then take, one by one, the free slots whose residues their pass uses
// least, each half's two passes are laid onto their lanes for the write
// groups (place_half), and a descent over both kinds of repeat finishes the
// half (refine_half). Neither step changes which slots a pair updates or the
// order of additions to any slot.
struct LaneCounts {
    int c16[2][4][16] = {};   // [role][read pass][atom index mod 16]
};

// Lanes of one read pass: a 16-byte LDS read is served in 4 passes of 16
// lanes, a pass holding the lanes that agree in lane bit 5 and in the parity
// of lane bits 2..4 (measured on gfx950: two active lanes conflict exactly
// when their addresses agree mod 16 bank quads and they share such a pass).
inline int read_pass(int lane) {
    const int b = (lane >> 2) & 7;
    return 2 * (lane >> 5) + (((b >> 2) ^ (b >> 1) ^ b) & 1);
}

// A 16-byte LDS write is served 8 consecutive lanes at a time, over 8 bank
// quads: lanes of one aligned 8-lane group whose atom indices agree mod 8
// wait for each other. Each 8-lane group holds 4 lanes of each of the two
// read passes of its 32-lane half.
// Descent on read and write repeats together over a 32-lane half: swaps of
// any two lanes (also across the two read passes) and swaps of a pair's two
// atoms, on the sums of squared residue counts per read pass (mod 16) and per
// write group (mod 8); first-improvement passes until none helps.
constexpr int kRefinePasses = 12;

void refine_half(uint32_t* lanes32, int half) {
    int rc[2][2][16] = {}, wc[4][2][8] = {};
    auto atom = [&](int l, int role) { return role ? (int)((lanes32[l] >> 7) & 127) : (int)(lanes32[l] & 127); };
    auto pass = [&](int l) { return read_pass(32 * half + l) & 1; };
    auto put = [&](int l, int sgn, long long& cost) {
        for (int role = 0; role < 2; ++role) {
            const int a = atom(l, role);
            int& r = rc[pass(l)][role][a & 15];
            int& w = wc[l >> 3][role][a & 7];
            if (sgn > 0) { cost += 2 * r + 1; ++r; cost += 2 * w + 1; ++w; }
            else { --r; cost -= 2 * r + 1; --w; cost -= 2 * w + 1; }
        }
    };
    auto flip = [&](int l) {
        const uint32_t r = lanes32[l];
        const uint32_t i = r & 127, j = (r >> 7) & 127, ci = (r >> 14) & 15, cj = (r >> 18) & 15;
        lanes32[l] = (r & ~0x3FFFFFu) | j | (i << 7) | (cj << 14) | (ci << 18);
    };
    long long cost = 0;
    for (int l = 0; l < 32; ++l) put(l, +1, cost);
    // first-improvement passes over every lane pair and every lane's atom
    // swap, until a pass finds nothing better
    auto try_move = [&](int a, int b) {
        const long long before = cost;
        put(a, -1, cost);
        if (b != a) put(b, -1, cost);
        if (b == a) flip(a); else std::swap(lanes32[a], lanes32[b]);
        put(a, +1, cost);
        if (b != a) put(b, +1, cost);
        if (cost < before) return true;
        put(a, -1, cost);
        if (b != a) put(b, -1, cost);
        if (b == a) flip(a); else std::swap(lanes32[a], lanes32[b]);
        put(a, +1, cost);
        if (b != a) put(b, +1, cost);
        return false;
    };
    for (int pass = 0; pass < kRefinePasses; ++pass) {
        bool improved = false;
        for (int a = 0; a < 32; ++a)
            for (int b = a; b < 32; ++b) improved |= try_move(a, b);
        if (!improved) break;
    }
}

// Splits 16 records whose first-atom and second-atom classes mod 8 each occur
// exactly twice (a 2-regular bipartite multigraph) into two sets of 8 that
// each hold every class once per role: alternate edges around each cycle.
bool two_matchings(const std::vector<uint32_t>& rec, std::vector<int>& side) {
    const int n = (int)rec.size();
    if (n != 16) return false;
    std::vector<int> t(n), h(n);
    int ct[8] = {}, ch[8] = {};
    for (int e = 0; e < n; ++e) {
        t[e] = rec[e] & 7;
        h[e] = (rec[e] >> 7) & 7;
        ++ct[t[e]];
        ++ch[h[e]];
    }
    for (int c = 0; c < 8; ++c) if (ct[c] != 2 || ch[c] != 2) return false;
    side.assign(n, -1);
    for (int start = 0; start < n; ++start) {
        if (side[start] >= 0) continue;
        int e = start, s = 0;
        bool at_head = true;            // walk from e's head to the other edge there
        while (side[e] < 0) {
            side[e] = s;
            s ^= 1;
            const int v = at_head ? h[e] : t[e];
            int f = -1;
            for (int g = 0; g < n && f < 0; ++g)
                if (g != e && side[g] < 0 && (at_head ? h[g] : t[g]) == v) f = g;
            if (f < 0) break;
            e = f;
            at_head = !at_head;
        }
    }
    return true;
}

// Given perfect matchings X and Y on the 8 + 8 classes (8 records each),
// chooses cycles of X u Y so that one perfect matching takes 4 records of X
// and 4 of Y; the rest form the complementary one. m[e] in {0, 1} for the
// 16 records (X first). False if no subset of cycles has half-length 4.
bool balanced_pair(const std::vector<uint32_t>& xy, std::vector<int>& m) {
    const int n = 16;
    std::vector<int> cyc(n, -1);
    std::vector<int> len;
    for (int start = 0; start < n; ++start) {
        if (cyc[start] >= 0) continue;
        const int id = (int)len.size();
        len.push_back(0);
        std::vector<int> stack{start};
        cyc[start] = id;
        while (!stack.empty()) {
            const int e = stack.back();
            stack.pop_back();
            ++len[id];
            for (int f = 0; f < n; ++f) {
                if (cyc[f] >= 0) continue;
                if (((xy[f] & 7) == (xy[e] & 7)) || (((xy[f] >> 7) & 7) == ((xy[e] >> 7) & 7))) {
                    cyc[f] = id;
                    stack.push_back(f);
                }
            }
        }
    }
    const int K = (int)len.size();
    // subset of cycles whose X-edge count (half the length) sums to 4
    std::vector<std::vector<uint8_t>> reach(K + 1, std::vector<uint8_t>(9, 0));
    reach[0][0] = 1;
    for (int k = 0; k < K; ++k)
        for (int s0 = 0; s0 <= 8; ++s0) {
            if (!reach[k][s0]) continue;
            reach[k + 1][s0] = 1;
            if (s0 + len[k] / 2 <= 8) reach[k + 1][s0 + len[k] / 2] = 1;
        }
    if (!reach[K][4]) return false;
    std::vector<int> take(K, 0);
    int want = 4;
    for (int k = K - 1; k >= 0; --k)
        if (!reach[k][want]) { take[k] = 1; want -= len[k] / 2; }
    m.assign(n, 0);
    for (int e = 0; e < n; ++e) {
        const bool is_x = e < 8;
        m[e] = (take[cyc[e]] ? (is_x ? 0 : 1) : (is_x ? 1 : 0));
    }
    return true;
}

void place_half(const std::vector<uint32_t>& p0, const std::vector<uint32_t>& p1, int half, uint32_t* out64) {
    uint32_t* lanes32 = out64 + 32 * half;
    // lanes of each (write group, read pass) within the half
    std::vector<int> slot[4][2];
    for (int l = 0; l < 32; ++l) slot[l >> 3][read_pass(32 * half + l) & 1].push_back(l);
    // exact: both passes 2-regular on the classes mod 8, and the write groups
    // formed as balanced perfect matchings of X u Y
    std::vector<int> sa, sb;
    if (two_matchings(p0, sa) && two_matchings(p1, sb)) {
        std::vector<uint32_t> A[2], Bm[2];
        for (int e = 0; e < 16; ++e) { A[sa[e]].push_back(p0[e]); Bm[sb[e]].push_back(p1[e]); }
        for (int pairing = 0; pairing < 2; ++pairing) {
            std::vector<uint32_t> groups[4][2];
            bool ok = true;
            for (int q = 0; q < 2 && ok; ++q) {
                std::vector<uint32_t> xy(A[q]);
                const std::vector<uint32_t>& y = Bm[q ^ pairing];
                xy.insert(xy.end(), y.begin(), y.end());
                std::vector<int> m;
                ok = balanced_pair(xy, m);
                if (!ok) break;
                for (int e = 0; e < 16; ++e) groups[2 * q + m[e]][e < 8 ? 0 : 1].push_back(xy[e]);
            }
            if (!ok) continue;
            for (int w = 0; w < 4; ++w)
                for (int p = 0; p < 2; ++p)
                    for (int k = 0; k < 4; ++k) lanes32[slot[w][p][k]] = groups[w][p][k];
            return;
        }
    }
    int k[2] = {0, 0};
    for (int l = 0; l < 32; ++l) {
        const int p = read_pass(32 * half + l) & 1;
        lanes32[l] = (p ? p1 : p0)[k[p]++];
    }
    refine_half(lanes32, half);
}

// Orients the edges (u[e], v[e]) of a multigraph on 16 vertices along Euler
// circuits (odd vertices paired by virtual edges): flip[e] = 1 reverses edge e.
void euler_orient(const std::vector<int>& u, const std::vector<int>& v, std::vector<uint8_t>& flip) {
    const int n = (int)u.size();
    std::vector<int> eu(u), ev(v);
    std::vector<int> deg(16, 0);
    for (int e = 0; e < n; ++e) { ++deg[eu[e]]; ++deg[ev[e]]; }
    int odd = -1;
    for (int r = 0; r < 16; ++r)
        if (deg[r] & 1) {
            if (odd < 0) { odd = r; continue; }
            eu.push_back(odd); ev.push_back(r); odd = -1;
        }
    const int m = (int)eu.size();
    std::vector<std::vector<int>> adj(16);
    for (int e = 0; e < m; ++e) { adj[eu[e]].push_back(e); if (ev[e] != eu[e]) adj[ev[e]].push_back(e); }
    std::vector<uint8_t> used(m, 0);
    std::vector<size_t> next(16, 0);
    flip.assign(n, 0);
    for (int start = 0; start < 16; ++start) {
        // walk unused edges from `start`, orienting each edge in the walking direction
        int cur = start;
        while (true) {
            while (next[cur] < adj[cur].size() && used[adj[cur][next[cur]]]) ++next[cur];
            if (next[cur] == adj[cur].size()) {
                // stuck (closed a circuit): continue from any vertex with unused edges
                int w = -1;
                for (int r = 0; r < 16 && w < 0; ++r) {
                    while (next[r] < adj[r].size() && used[adj[r][next[r]]]) ++next[r];
                    if (next[r] < adj[r].size()) w = r;
                }
                if (w < 0) break;
                cur = w;
                continue;
            }
            const int e = adj[cur][next[cur]];
            used[e] = 1;
            const int to = (eu[e] == cur) ? ev[e] : eu[e];
            if (e < n) flip[e] = (eu[e] == cur) ? 0 : 1;
            cur = to;
        }
    }
}

std::vector<uint32_t> arrange_batch(const std::vector<uint32_t>& real, const uint8_t* use, int N, int S,
                                    int C, std::string& err) {
    const int B = dockblob::kBatch;
    const int n = (int)real.size();
    std::vector<int> ea(n), eb(n);   // first and second atom of each pair
    for (int e = 0; e < n; ++e) { ea[e] = real[e] & 127; eb[e] = (real[e] >> 7) & 127; }
    std::vector<int> ru(n), rv(n);
    for (int e = 0; e < n; ++e) { ru[e] = ea[e] & 15; rv[e] = eb[e] & 15; }
    std::vector<uint8_t> flip;
    euler_orient(ru, rv, flip);
    std::vector<int> tail(n), head(n);
    for (int e = 0; e < n; ++e) {
        tail[e] = flip[e] ? rv[e] : ru[e];
        head[e] = flip[e] ? ru[e] : rv[e];
    }
    // Residues used more than 4 times as first (or second) atom cannot be
    // kept apart in 4 groups: set aside as few pairs as needed to bring every
    // residue to <= 4 uses per role, preferring pairs that relieve both ends.
    std::vector<int> n_first(16, 0), n_second(16, 0);
    for (int e = 0; e < n; ++e) { ++n_first[tail[e]]; ++n_second[head[e]]; }
    std::vector<uint8_t> aside(n, 0);
    for (int pass = 0; pass < 2; ++pass)
        for (int e = 0; e < n; ++e) {
            if (aside[e]) continue;
            const bool xt = n_first[tail[e]] > 4, xh = n_second[head[e]] > 4;
            if (pass == 0 ? (xt && xh) : (xt || xh)) {
                aside[e] = 1;
                --n_first[tail[e]];
                --n_second[head[e]];
            }
        }
    // Kempe-chain colouring of the rest, a bipartite multigraph (first-atom
    // residues, second-atom residues) of maximum degree <= 4, with 4 colours
    const int K = 4;
    std::vector<int> at_t(16 * K, -1), at_h(16 * K, -1), col(n, -1);
    for (int e = 0; e < n; ++e) {
        if (aside[e]) continue;
        const int t = tail[e], h = head[e];
        int a = -1, b = -1;
        for (int c = 0; c < K && a < 0; ++c) if (at_t[t * K + c] < 0) a = c;
        for (int c = 0; c < K && b < 0; ++c) if (at_h[h * K + c] < 0) b = c;
        if (at_h[h * K + a] >= 0) {
            // swap colours a and b along the path from h that starts with colour a
            std::vector<int> path;
            int x = h, want = a;
            bool on_head = true;
            while (true) {
                const int f = on_head ? at_h[x * K + want] : at_t[x * K + want];
                if (f < 0) break;
                path.push_back(f);
                x = on_head ? tail[f] : head[f];
                on_head = !on_head;
                want = (want == a) ? b : a;
            }
            for (int f : path) { at_t[tail[f] * K + col[f]] = -1; at_h[head[f] * K + col[f]] = -1; }
            for (int f : path) {
                col[f] = (col[f] == a) ? b : a;
                at_t[tail[f] * K + col[f]] = f;
                at_h[head[f] * K + col[f]] = f;
            }
        }
        col[e] = a;
        at_t[t * K + a] = e;
        at_h[h * K + a] = e;
    }
    // colour g = lane group g; the pairs set aside go where they add the
    // fewest repeats
    std::vector<std::vector<int>> groups(4);
    LaneCounts lc;
    for (int e = 0; e < n; ++e) {
        if (aside[e]) continue;
        groups[col[e]].push_back(e);
        ++lc.c16[0][col[e]][tail[e]];
        ++lc.c16[1][col[e]][head[e]];
    }
    for (int e = 0; e < n; ++e) {
        if (!aside[e]) continue;
        int best = -1, best_cost = 0;
        for (int g = 0; g < 4; ++g) {
            if ((int)groups[g].size() >= 16) continue;
            const int c = lc.c16[0][g][tail[e]] + lc.c16[1][g][head[e]];
            if (best < 0 || c < best_cost) { best = g; best_cost = c; }
        }
        groups[best].push_back(e);
        ++lc.c16[0][best][tail[e]];
        ++lc.c16[1][best][head[e]];
    }
    // free slots (copy, atom): unused copies of real atoms, then every slot of
    // the atoms N .. S-1 past the end
    std::vector<std::pair<int, int>> free_slots;
    for (int c = 0; c < C; ++c)
        for (int a = 0; a < S; ++a)
            if (a >= N || c >= use[a]) free_slots.push_back({c, a});
    std::vector<uint8_t> taken(free_slots.size(), 0);
    auto take_best = [&](int role, int g) -> int {
        int best = -1, best_cost = 0;
        for (size_t k = 0; k < free_slots.size(); ++k) {
            if (taken[k]) continue;
            const int c = lc.c16[role][g][free_slots[k].second & 15];
            if (best < 0 || c < best_cost) { best = (int)k; best_cost = c; }
        }
        if (best >= 0) {
            taken[best] = 1;
            ++lc.c16[role][g][free_slots[best].second & 15];
        }
        return best;
    };
    // colour g becomes read pass g: half g / 2, parity g % 2
    std::vector<std::vector<uint32_t>> pass_rec(4);
    for (int g = 0; g < 4; ++g) {
        std::vector<uint32_t>& rec = pass_rec[g];
        for (int e : groups[g]) {
            const uint32_t r = real[e];
            if (!flip[e]) { rec.push_back(r); continue; }
            const uint32_t i = r & 127, j = (r >> 7) & 127, ci = (r >> 14) & 15, cj = (r >> 18) & 15;
            rec.push_back((r & ~0x3FFFFFu) | j | (i << 7) | (cj << 14) | (ci << 18));
        }
        for (int l = (int)groups[g].size(); l < 16; ++l) {
            const int u = take_best(0, g), v = take_best(1, g);
            if (u < 0 || v < 0) { err = "internal: no free accumulator slots for batch padding"; return {}; }
            rec.push_back(dockblob::make_pad_record(free_slots[u].second, free_slots[v].second,
                                                    free_slots[u].first, free_slots[v].first));
        }
    }
    std::vector<uint32_t> out(B);
    for (int half = 0; half < 2; ++half) place_half(pass_rec[2 * half], pass_rec[2 * half + 1], half, out.data());
    return out;
}

}  // namespace

int32_t prepare(const dock_ligand_desc& d, Prepared& P, std::string& err) {
    const int N = d.n_atoms;
    const int T = d.n_torsions;
    if (N < 1) { err = "n_atoms must be >= 1"; return DOCK_EINVAL; }
    if (N > dockblob::kMaxAtoms) { err = "n_atoms exceeds DOCK_MAX_ATOMS"; return DOCK_EUNSUPPORTED; }
    if (T < 0) { err = "n_torsions must be >= 0"; return DOCK_EINVAL; }
    if (T > dockblob::kMaxTorsions) { err = "n_torsions exceeds DOCK_MAX_TORSIONS"; return DOCK_EUNSUPPORTED; }
    if (!d.xyz || !d.charge || !d.cls || (N > 1 && !d.bonds) || (T > 0 && !d.rot_bonds) || !d.ff) {
        err = "NULL array in ligand description"; return DOCK_EINVAL;
    }
    const dock_ff_params& ff = *d.ff;
    if (ff.n_classes < 1 || ff.n_classes > DOCK_MAX_CLASSES || !ff.radius || !ff.eps || !ff.solv || !ff.vol) {
        err = "bad force-field table"; return DOCK_EINVAL;
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (ff.donor[i] >= 0 && ff.donor[i] == ff.acceptor[j]) {
                err = "a class cannot be both donor and acceptor"; return DOCK_EINVAL;
            }
    if (d.root_atom < 0 || d.root_atom >= N) { err = "root_atom out of range"; return DOCK_EINVAL; }
    for (int i = 0; i < N; ++i) {
        if (d.cls[i] < 0 || d.cls[i] >= ff.n_classes) { err = "atom class out of range"; return DOCK_EINVAL; }
        if (!std::isfinite(d.xyz[3 * i]) || !std::isfinite(d.xyz[3 * i + 1]) ||
            !std::isfinite(d.xyz[3 * i + 2]) || !std::isfinite(d.charge[i])) {
            err = "non-finite coordinate or charge"; return DOCK_EINVAL;
        }
    }
    // adjacency of the bond graph (a tree, or a connected graph with rings)
    const int NB = d.n_bonds;
    if (N > 1 && (NB < N - 1 || NB > 4 * N)) {
        err = "n_bonds must be in [n_atoms - 1, 4 n_atoms]"; return DOCK_EINVAL;
    }
    std::vector<std::vector<int>> adj(N);
    for (int e = 0; e < NB; ++e) {
        int u = d.bonds[2 * e], v = d.bonds[2 * e + 1];
        if (u < 0 || v < 0 || u >= N || v >= N || u == v) { err = "bond endpoint out of range"; return DOCK_EINVAL; }
        adj[u].push_back(v);
        adj[v].push_back(u);
    }
    for (auto& a : adj) {
        std::sort(a.begin(), a.end());
        if (std::adjacent_find(a.begin(), a.end()) != a.end()) { err = "duplicate bond"; return DOCK_EINVAL; }
    }
    // depth-first preorder from the root, neighbours by increasing index; the
    // depth-first tree keeps every subtree contiguous in the order, and a
    // rotatable bond (a bridge of the graph, checked below) is a tree edge
    // whose subtree is exactly the side it moves
    std::vector<int> parent(N, -2), depth(N, 0), order;
    order.reserve(N);
    {
        std::vector<std::pair<int, size_t>> stack{{d.root_atom, 0}};
        parent[d.root_atom] = -1;
        order.push_back(d.root_atom);
        while (!stack.empty()) {
            auto& top = stack.back();
            const int u = top.first;
            if (top.second == adj[u].size()) { stack.pop_back(); continue; }
            const int v = adj[u][top.second++];
            if (parent[v] != -2) continue;
            parent[v] = u;
            depth[v] = depth[u] + 1;
            order.push_back(v);
            stack.push_back({v, 0});
        }
    }
    if ((int)order.size() != N) { err = "bonds do not connect every atom"; return DOCK_EINVAL; }
    std::vector<int> pos(N), size(N, 1);
    for (int p = 0; p < N; ++p) pos[order[p]] = p;
    for (int p = N - 1; p > 0; --p) size[parent[order[p]]] += size[order[p]];
    // bond-graph distances (breadth-first from every atom; rings make them
    // shorter than depth-first tree paths)
    std::vector<int> gdist(size_t(N) * N, -1);
    {
        std::vector<int> queue(N);
        for (int s0 = 0; s0 < N; ++s0) {
            int* dist = &gdist[size_t(s0) * N];
            int head = 0, tail = 0;
            dist[s0] = 0;
            queue[tail++] = s0;
            while (head < tail) {
                const int u = queue[head++];
                for (int v : adj[u])
                    if (dist[v] < 0) { dist[v] = dist[u] + 1; queue[tail++] = v; }
            }
        }
    }

    // torsions
    std::vector<int> tor_a(T), tor_b(T), tor_of_b(N, -1);
    for (int k = 0; k < T; ++k) {
        int e = d.rot_bonds[k];
        if (e < 0 || e >= NB) { err = "rotatable bond index out of range"; return DOCK_EINVAL; }
        int u = d.bonds[2 * e], v = d.bonds[2 * e + 1];
        if (parent[v] != u && parent[u] != v) { err = "rotatable bond lies in a ring"; return DOCK_EINVAL; }
        int a = (parent[v] == u) ? u : v;
        int b = (a == u) ? v : u;
        // a tree edge is a bridge iff no non-tree bond leaves b's subtree
        for (int p = pos[b]; p < pos[b] + size[b]; ++p)
            for (int w : adj[order[p]]) {
                const bool inside = pos[w] >= pos[b] && pos[w] < pos[b] + size[b];
                if (!inside && !(order[p] == b && w == a)) { err = "rotatable bond lies in a ring"; return DOCK_EINVAL; }
            }
        if (adj[a].size() < 2 || adj[b].size() < 2) { err = "rotatable bond is not internal"; return DOCK_EINVAL; }
        if (tor_of_b[b] >= 0) { err = "rotatable bond listed twice"; return DOCK_EINVAL; }
        tor_a[k] = a;
        tor_b[k] = b;
        tor_of_b[b] = k;
    }
    // fragment of each atom: the nearest torsion b at or above it (k+1), else 0
    std::vector<int> frag(N, 0);
    for (int p = 0; p < N; ++p) {
        int i = order[p];
        frag[i] = (tor_of_b[i] >= 0) ? tor_of_b[i] + 1 : (parent[i] >= 0 ? frag[parent[i]] : 0);
    }
    // fragment chains (root-first torsion lists); parents come first in preorder
    const int NF = T + 1;
    std::vector<std::vector<int>> chain(NF);
    int max_depth = 0;
    for (int p = 0; p < N; ++p) {
        int b = order[p];
        int k = tor_of_b[b];
        if (k < 0) continue;
        chain[k + 1] = chain[frag[tor_a[k]]];
        chain[k + 1].push_back(k);
        max_depth = std::max(max_depth, (int)chain[k + 1].size());
    }
    auto graph_dist = [&](int i, int j) { return gdist[size_t(i) * N + j]; };
    // kept pairs in depth-first positions (p < q), with their 12-10 table index
    struct KeptPair { int p, q, hb, table; };
    std::vector<KeptPair> plist;
    for (int p = 0; p < N; ++p)
        for (int q = p + 1; q < N; ++q) {
            const int i = order[p], j = order[q];
            if (frag[i] == frag[j] || graph_dist(i, j) < 4) continue;
            const int ci = d.cls[i], cj = d.cls[j];
            int table = 0, hb = 0;
            if (role_index(ff.donor, ci) >= 0 && role_index(ff.acceptor, cj) >= 0) {
                hb = 1; table = 2 * role_index(ff.donor, ci) + role_index(ff.acceptor, cj);
            } else if (role_index(ff.acceptor, ci) >= 0 && role_index(ff.donor, cj) >= 0) {
                hb = 1; table = 2 * role_index(ff.donor, cj) + role_index(ff.acceptor, ci);
            }
            plist.push_back({p, q, hb, table});
        }
    const int n_pairs = (int)plist.size();
    // batches of kBatch pairs, each atom at most C times per batch. C grows for
    // small ligands so that C * N can hold a full batch's 128 pair ends (up to
    // 15, the largest copy index a record holds). The
    // batch count starts at its lower bound, max(P / 64, max degree / C);
    // pairs are placed most-constrained first (largest endpoint degree), each
    // into the open batch where its atoms' residues mod 16 stay within 8 uses
    // (the share of a full batch's 128 pair ends, which lets arrange_batch
    // place the batch without LDS bank repeats), then where its two atoms are
    // used least, then the least filled batch, then the lowest index; if a
    // pair finds no batch, the count grows by one and the placement restarts.
    using dockblob::kBatch;
    const int C = std::max(2, std::min(15, (2 * kBatch + N - 1) / N + 1));
    using dockblob::kMaxSlots;
    using dockblob::kMaxSlotsSmall;
    using dockblob::kMaxSlotsTiny;
    const int S = dockblob::slot_stride(N);
    if (C * S > (N <= 32 ? kMaxSlotsTiny : (N <= 64 ? kMaxSlotsSmall : kMaxSlots))) {
        err = "internal: accumulator slots exceed the build limit"; return DOCK_EUNSUPPORTED;
    }
    std::vector<int> degp(N, 0);
    for (const KeptPair& pr : plist) { ++degp[pr.p]; ++degp[pr.q]; }
    std::vector<int> porder(plist.size());
    for (size_t k = 0; k < porder.size(); ++k) porder[k] = (int)k;
    std::stable_sort(porder.begin(), porder.end(), [&](int a, int b) {
        return std::max(degp[plist[a].p], degp[plist[a].q]) > std::max(degp[plist[b].p], degp[plist[b].q]);
    });
    int maxdeg = 0;
    for (int v = 0; v < N; ++v) maxdeg = std::max(maxdeg, degp[v]);
    int nb = std::max((n_pairs + kBatch - 1) / kBatch, (maxdeg + C - 1) / C);
    std::vector<std::vector<uint32_t>> batch;      // records
    while (true) {
        batch.assign(nb, {});
        std::vector<int> cnt(nb, 0);
        std::vector<uint8_t> use(size_t(nb) * N, 0);
        std::vector<int> rload(size_t(nb) * 16, 0);   // pair ends per residue mod 16
        bool placed_all = true;
        for (int k : porder) {
            const KeptPair& pr = plist[k];
            const int rp = pr.p & 15, rq = pr.q & 15;
            int best = -1;
            long long best_score = 0;
            for (int b = 0; b < nb; ++b) {
                const int up = use[size_t(b) * N + pr.p], uq = use[size_t(b) * N + pr.q];
                if (cnt[b] >= kBatch || up >= C || uq >= C) continue;
                const int* rl = &rload[size_t(b) * 16];
                const int over = rp == rq ? std::max(0, rl[rp] + 2 - 8)
                                          : std::max(0, rl[rp] + 1 - 8) + std::max(0, rl[rq] + 1 - 8);
                const long long score = -(long long)over * 1000000 - (up + uq) * 1000 - cnt[b];
                if (best < 0 || score > best_score) { best = b; best_score = score; }
            }
            if (best < 0) { placed_all = false; break; }
            const int ci = use[size_t(best) * N + pr.p]++;
            const int cj = use[size_t(best) * N + pr.q]++;
            ++rload[size_t(best) * 16 + rp];
            ++rload[size_t(best) * 16 + rq];
            ++cnt[best];
            batch[best].push_back(dockblob::make_record(pr.p, pr.q, ci, cj, pr.hb, pr.table));
        }
        if (placed_all) {
            // Lanes are arranged for LDS bank spreading (arrange_batch).
            // Unused lanes get records with the valid bit clear whose two
            // slots are distinct and unused in their batch: free copies of
            // real atoms or slots of the "atoms" N .. S-1 past the end
            // (C * S >= 128 + N > 128 always leaves enough). Their force is
            // zero, so every lane may update its slots without a branch.
            for (int b = 0; b < nb; ++b) {
                batch[b] = arrange_batch(batch[b], &use[size_t(b) * N], N, S, C, err);
                if (batch[b].empty()) return DOCK_EUNSUPPORTED;
            }
            break;
        }
        ++nb;
    }
    if (n_pairs == 0) batch.clear();
    const int n_batches = (int)batch.size();

    // ---- pack the blob ----
    using namespace dockblob;
    Header h;
    std::memset(&h, 0, sizeof(h));
    size_t off = sizeof(Header);
    auto take = [&](size_t bytes) { size_t o = off; off = align16(off + bytes); return (int32_t)o; };
    h.off_ref = take(16 * size_t(N));
    h.off_chg = take(16 * size_t(N));
    h.off_int = take(16 * size_t(N));
    h.off_tors = take(sizeof(Torsion) * size_t(T));
    h.off_chain = take(size_t(NF) * kChainStride);
    h.off_plist = take(sizeof(dockblob::PairRec) * size_t(kBatch) * size_t(n_batches));
    h.magic = kMagic;
    h.n_atoms = N;
    h.n_torsions = T;
    h.n_frag = NF;
    h.n_genes = 7 + T;
    h.n_pairs = n_pairs;
    h.max_depth = max_depth;
    h.n_batches = n_batches;
    h.n_copies = C;
    h.slot_stride = S;
    h.total_bytes = (int32_t)off;
    int max_class = 0;
    for (int i = 0; i < N; ++i) max_class = std::max(max_class, (int)d.cls[i]);
    h.max_class = max_class;

    std::vector<uint8_t> blob(off, 0);
    std::memcpy(blob.data(), &h, sizeof(h));
    double cen[3] = {0, 0, 0};
    for (int i = 0; i < N; ++i)
        for (int c = 0; c < 3; ++c) cen[c] += d.xyz[3 * i + c];
    for (int c = 0; c < 3; ++c) cen[c] /= N;
    auto y0 = [&](int i, int c) { return d.xyz[3 * i + c] - cen[c]; };
    float* ref = reinterpret_cast<float*>(blob.data() + h.off_ref);
    float* chg = reinterpret_cast<float*>(blob.data() + h.off_chg);
    int32_t* iv = reinterpret_cast<int32_t*>(blob.data() + h.off_int);
    for (int p = 0; p < N; ++p) {
        int i = order[p];
        int c = d.cls[i];
        double q = d.charge[i];
        for (int a = 0; a < 3; ++a) ref[4 * p + a] = (float)y0(i, a);
        chg[4 * p + 0] = (float)(kElec * q);
        chg[4 * p + 1] = (float)q;
        chg[4 * p + 2] = (float)std::fabs(q);
        iv[4 * p + 0] = c;
        iv[4 * p + 1] = frag[i];
        iv[4 * p + 2] = i;
    }
    Torsion* tr = reinterpret_cast<Torsion*>(blob.data() + h.off_tors);
    for (int k = 0; k < T; ++k) {
        int a = tor_a[k], b = tor_b[k];
        double u[3], nrm = 0;
        for (int c = 0; c < 3; ++c) { u[c] = y0(b, c) - y0(a, c); nrm += u[c] * u[c]; }
        nrm = std::sqrt(nrm);
        for (int c = 0; c < 3; ++c) {
            tr[k].p[c] = (float)y0(a, c);
            tr[k].u[c] = (float)(u[c] / nrm);
        }
        tr[k].a_pos = pos[a];
        tr[k].b_pos = pos[b];
        tr[k].first = pos[b];
        tr[k].end = pos[b] + size[b];
    }
    PairRec* pl = reinterpret_cast<PairRec*>(blob.data() + h.off_plist);
    auto solv = [&](int i) { return ff.solv[d.cls[i]] + kQSolv * std::fabs((double)d.charge[i]); };
    for (int b = 0; b < n_batches; ++b)
        for (size_t k = 0; k < batch[b].size(); ++k) {
            const uint32_t r = batch[b][k];
            PairRec& o = pl[b * kBatch + k];
            o.rec = dockblob::device_word(r, S);
            if (!(r & kRecValid)) {
                uint32_t neg_zero = kPadC12;
                std::memcpy(&o.c12, &neg_zero, sizeof(float));
                o.cm = o.ds = 0.f;
                continue;
            }
            const int i = order[r & 127], j = order[(r >> 7) & 127];
            const int ci = d.cls[i], cj = d.cls[j];
            // A / r^12 + B / r^m: 12-10 (5, -6) eps r0^(12, 10) from the
            // donor-acceptor table, else 12-6 (1, -2) eps r0^(12, 6)
            if ((r >> 22) & 1u) {
                const int t = (r >> 23) & 3;
                const double r0 = ff.hb_r0[t >> 1][t & 1], eps = ff.hb_eps[t >> 1][t & 1];
                o.c12 = (float)(5.0 * eps * std::pow(r0, 12));
                o.cm = (float)(-6.0 * eps * std::pow(r0, 10));
            } else {
                const double r0 = ff.radius[ci] + ff.radius[cj];
                const double eps = std::sqrt(ff.eps[ci] * ff.eps[cj]);
                o.c12 = (float)(eps * std::pow(r0, 12));
                o.cm = (float)(-2.0 * eps * std::pow(r0, 6));
            }
            o.ds = (float)(solv(i) * ff.vol[cj] + solv(j) * ff.vol[ci]);
        }
    // fragment f: the torsions that enclose it, innermost first (the order
    // they are applied in), padded with the identity transform
    uint8_t* ch = blob.data() + h.off_chain;
    for (int f = 0; f < NF; ++f)
        for (int j = 0; j < kChainStride; ++j) {
            const int n = (int)chain[f].size();
            ch[f * kChainStride + j] = (uint8_t)(j < n ? chain[f][n - 1 - j] : kIdentity);
        }

    P.n_atoms = N;
    P.n_torsions = T;
    P.n_frag = NF;
    P.max_depth = max_depth;
    P.n_pairs = n_pairs;
    P.max_class = max_class;
    P.order.assign(order.begin(), order.end());
    P.pos.assign(pos.begin(), pos.end());
    P.tors_a.assign(tor_a.begin(), tor_a.end());
    P.tors_b.assign(tor_b.begin(), tor_b.end());
    P.tors_first.resize(T);
    P.tors_end.resize(T);
    for (int k = 0; k < T; ++k) { P.tors_first[k] = tr[k].first; P.tors_end[k] = tr[k].end; }
    P.frag_of_atom.assign(frag.begin(), frag.end());
    P.blob.swap(blob);
    return DOCK_OK;
}

uint32_t record_of(const Prepared& P, int k) {
    using namespace dockblob;
    const Header* h = reinterpret_cast<const Header*>(P.blob.data());
    const PairRec& pr = reinterpret_cast<const PairRec*>(P.blob.data() + h->off_plist)[k];
    uint32_t c12_bits;
    std::memcpy(&c12_bits, &pr.c12, sizeof(float));
    return logical_record(pr.rec, c12_bits != kPadC12, h->slot_stride);
}

void decode_pairs(const Prepared& P, std::vector<uint32_t>& pairs, std::vector<uint8_t>& hb) {
    using namespace dockblob;
    const Header* h = reinterpret_cast<const Header*>(P.blob.data());
    std::vector<std::pair<uint32_t, uint8_t>> v;
    for (int k = 0; k < h->n_batches * kBatch; ++k) {
        const uint32_t r = record_of(P, k);
        if (!(r & kRecValid)) continue;
        const int i = P.order[r & 127], j = P.order[(r >> 7) & 127];
        const uint32_t lo = (uint32_t)std::min(i, j), hi = (uint32_t)std::max(i, j);
        v.push_back({(lo << 16) | hi, (uint8_t)((r >> 22) & 1)});
    }
    std::sort(v.begin(), v.end());
    pairs.resize(v.size());
    hb.resize(v.size());
    for (size_t k = 0; k < v.size(); ++k) { pairs[k] = v[k].first; hb[k] = v[k].second; }
}

}  // namespace dockprep
