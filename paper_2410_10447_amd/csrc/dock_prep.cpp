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
#include <array>
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

// LDS bank spreading of one batch. A wave's 16-byte LDS accesses are
// served 16 lanes at a time over 64 four-byte banks (16 bank quads), and two
// lanes of a group whose different addresses fall into the same quad
// (address / 16 modulo 16) wait for each other. The pair loop reads and
// writes the first and the second atom of each lane's pair (position and
// slot: with a stride that is a multiple of 16 both lie in the quad of the
// atom index, its residue mod 16). The batch's records are therefore placed
// on the lanes, and a pair's two atoms may swap roles, so that within each
// aligned group of 16 lanes the first atoms' residues differ and so do the
// second atoms'. Seen as a multigraph on the 16 residues with one edge per
// pair, this is an orientation followed by an edge colouring with 4 colours
// (one per lane group): the orientation follows Euler circuits, so each
// residue is first atom about as often as second (|out - in| <= 1), and the
// bipartite (first residue, second residue) multigraph, after setting aside
// the few pairs that push a residue past 4 uses per role, is coloured with 4
// colours by Kempe-chain recolouring (Konig's theorem: a bipartite multigraph
// of maximum degree 4 has a proper 4-edge colouring); the pairs set aside go
// to the groups with room, where they add the fewest repeats. The unused
// lanes then take, one by one, the free slots whose residues their group
// uses least, and each group's records are ordered for the 8-lane halves of
// 16-byte writes (split_halves). Neither step changes which slots a pair
// updates or the order of additions to any slot.
struct LaneCounts {
    int c16[2][4][16] = {};   // [role][group of 16 lanes][atom index mod 16]
    void add(int role, int lane, int atom) { ++c16[role][lane >> 4][atom & 15]; }
};

// 16-byte LDS writes are served 8 lanes at a time: two lanes of an aligned
// 8-lane half whose atom indices agree mod 8 wait for each other. Orders a
// 16-lane group's records so that the halves repeat as few first-atom and
// second-atom residues mod 8 as possible. When each residue mod 8 occurs at
// most twice per role, "the two lanes of a residue go to different halves"
// is a graph of paths and even cycles (each lane has at most one partner per
// role, and the roles alternate around a cycle): it is 2-coloured per
// component and the components' colourings are chosen (subset sum) to fill
// both halves with 8 lanes. Otherwise, or if no such choice exists, pairwise
// swaps across the halves improve the split until none helps.
int halves_cost(const std::vector<uint32_t>& rec) {
    int c = 0;
    for (int h = 0; h < 2; ++h)
        for (int role = 0; role < 2; ++role) {
            int cnt[8] = {};
            for (int l = 8 * h; l < 8 * h + 8; ++l) {
                const int a = role ? (rec[l] >> 7) & 127 : rec[l] & 127;
                c += cnt[a & 7]++;
            }
        }
    return c;
}

void split_halves(std::vector<uint32_t>& rec) {
    const int L = 16;
    std::vector<std::vector<int>> adj(L);
    bool ok = true;
    for (int role = 0; role < 2; ++role)
        for (int cls = 0; cls < 8; ++cls) {
            std::vector<int> lanes;
            for (int l = 0; l < L; ++l) {
                const int a = role ? (rec[l] >> 7) & 127 : rec[l] & 127;
                if ((a & 7) == cls) lanes.push_back(l);
            }
            if (lanes.size() > 2) ok = false;
            if (lanes.size() == 2) { adj[lanes[0]].push_back(lanes[1]); adj[lanes[1]].push_back(lanes[0]); }
        }
    std::vector<int> col(L, -1), comp(L, -1);
    std::vector<std::array<int, 2>> size;
    for (int v = 0; v < L && ok; ++v) {
        if (col[v] >= 0) continue;
        const int id = (int)size.size();
        size.push_back({0, 0});
        std::vector<int> queue{v};
        col[v] = 0;
        for (size_t q = 0; q < queue.size() && ok; ++q) {
            const int x = queue[q];
            comp[x] = id;
            ++size[id][col[x]];
            for (int y : adj[x]) {
                if (col[y] < 0) { col[y] = col[x] ^ 1; queue.push_back(y); }
                else if (col[y] == col[x]) ok = false;
            }
        }
    }
    if (ok) {
        // reach[k][s]: the first k components can put s lanes into half 0
        const int K = (int)size.size();
        std::vector<std::vector<uint8_t>> reach(K + 1, std::vector<uint8_t>(L + 1, 0));
        reach[0][0] = 1;
        for (int k = 0; k < K; ++k)
            for (int s0 = 0; s0 <= L; ++s0) {
                if (!reach[k][s0]) continue;
                if (s0 + size[k][0] <= L) reach[k + 1][s0 + size[k][0]] = 1;
                if (s0 + size[k][1] <= L) reach[k + 1][s0 + size[k][1]] = 1;
            }
        if (reach[K][L / 2]) {
            std::vector<int> flip(K, 0);
            int want = L / 2;
            for (int k = K - 1; k >= 0; --k) {
                if (want - size[k][0] >= 0 && reach[k][want - size[k][0]]) { want -= size[k][0]; }
                else { flip[k] = 1; want -= size[k][1]; }
            }
            std::vector<uint32_t> out;
            for (int half = 0; half < 2; ++half)
                for (int l = 0; l < L; ++l)
                    if ((col[l] ^ flip[comp[l]]) == half) out.push_back(rec[l]);
            rec.swap(out);
            return;
        }
    }
    int best = halves_cost(rec);
    for (int pass = 0; pass < 16 && best > 0; ++pass) {
        bool improved = false;
        for (int a = 0; a < 8; ++a)
            for (int b = 8; b < 16; ++b) {
                std::swap(rec[a], rec[b]);
                const int c = halves_cost(rec);
                if (c < best) { best = c; improved = true; }
                else std::swap(rec[a], rec[b]);
            }
        if (!improved) break;
    }
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
    std::vector<uint32_t> out;
    out.reserve(B);
    for (int g = 0; g < 4; ++g) {
        std::vector<uint32_t> rec;
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
        split_halves(rec);
        out.insert(out.end(), rec.begin(), rec.end());
    }
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
    // adjacency of the bond tree
    std::vector<std::vector<int>> adj(N);
    for (int e = 0; e < N - 1; ++e) {
        int u = d.bonds[2 * e], v = d.bonds[2 * e + 1];
        if (u < 0 || v < 0 || u >= N || v >= N || u == v) { err = "bond endpoint out of range"; return DOCK_EINVAL; }
        adj[u].push_back(v);
        adj[v].push_back(u);
    }
    for (auto& a : adj) {
        std::sort(a.begin(), a.end());
        if (std::adjacent_find(a.begin(), a.end()) != a.end()) { err = "duplicate bond"; return DOCK_EINVAL; }
    }
    // depth-first preorder from the root, children by increasing index
    std::vector<int> parent(N, -2), depth(N, 0), order;
    order.reserve(N);
    std::vector<int> stack{d.root_atom};
    parent[d.root_atom] = -1;
    while (!stack.empty()) {
        int u = stack.back();
        stack.pop_back();
        order.push_back(u);
        for (auto it = adj[u].rbegin(); it != adj[u].rend(); ++it) {
            int v = *it;
            if (v == parent[u]) continue;
            if (parent[v] != -2) { err = "bonds contain a cycle"; return DOCK_EINVAL; }
            parent[v] = u;
            depth[v] = depth[u] + 1;
            stack.push_back(v);
        }
    }
    if ((int)order.size() != N) { err = "bonds do not connect every atom"; return DOCK_EINVAL; }
    std::vector<int> pos(N), size(N, 1);
    for (int p = 0; p < N; ++p) pos[order[p]] = p;
    for (int p = N - 1; p > 0; --p) size[parent[order[p]]] += size[order[p]];

    // torsions
    std::vector<int> tor_a(T), tor_b(T), tor_of_b(N, -1);
    for (int k = 0; k < T; ++k) {
        int e = d.rot_bonds[k];
        if (e < 0 || e >= N - 1) { err = "rotatable bond index out of range"; return DOCK_EINVAL; }
        int u = d.bonds[2 * e], v = d.bonds[2 * e + 1];
        int a = (parent[v] == u) ? u : v;
        int b = (a == u) ? v : u;
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
    // kept pairs (original indices) and their hydrogen-bond flag
    auto graph_dist = [&](int i, int j) {
        int a = i, b = j, da = depth[i], db = depth[j];
        while (da > db) { a = parent[a]; --da; }
        while (db > da) { b = parent[b]; --db; }
        while (a != b) { a = parent[a]; b = parent[b]; --da; }
        return depth[i] + depth[j] - 2 * da;
    };
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
    const int S = dockblob::slot_stride(N);
    if (C * S > (N <= 64 ? kMaxSlotsSmall : kMaxSlots)) {
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
