// lattice.cpp -- honeycomb lattices (Sec. II of arXiv:2212.04352: hopping
// j_ij = t between nearest neighbours of a graphene lattice) and Fock starts
// (Sec. IV.A: every site holds one electron of either spin).  Host code.
#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <set>
#include <utility>

#include "ftwa_internal.h"
#include "philox.h"

namespace ftwa {

namespace {

thread_local std::string g_last_error;

using Site = std::pair<int, int>;  // (row, column) on the brick wall

// Brick-wall honeycomb: every site has a left and a right neighbour in its
// row and one vertical neighbour, above when row + column is even.
bool vertical_up(int r, int c) { return ((r + c) % 2 + 2) % 2 == 0; }

// Builds a lattice from a set of brick-wall sites, numbered in the set's
// (row, column) order, with every brick-wall bond between two members.
ftwa_lattice from_brick_sites(const std::set<Site>& sites, double t) {
    std::map<Site, int> index;
    for (const Site& s : sites) index.emplace(s, (int)index.size());
    const int N = (int)index.size();
    std::vector<std::vector<int>> adj(N);
    int bonds = 0;
    for (const auto& [s, i] : index) {
        const Site right{s.first, s.second + 1};
        auto it = index.find(right);
        if (it != index.end()) { adj[i].push_back(it->second); adj[it->second].push_back(i); ++bonds; }
        if (vertical_up(s.first, s.second)) {
            auto up = index.find(Site{s.first + 1, s.second});
            if (up != index.end()) { adj[i].push_back(up->second); adj[up->second].push_back(i); ++bonds; }
        }
    }
    auto* lat = new ftwa_lattice_s;
    lat->N = N;
    lat->n_bonds = bonds;
    lat->t = t;
    lat->nbr.assign((size_t)N * kMaxDeg, -1);
    lat->deg.assign(N, 0);
    lat->sub.assign(N, 0);
    for (const auto& [s, i] : index) {
        auto& a = adj[i];
        std::sort(a.begin(), a.end());
        if (a.size() > (size_t)kMaxDeg) { delete lat; return nullptr; }
        for (size_t k = 0; k < a.size(); ++k) lat->nbr[(size_t)i * kMaxDeg + k] = a[k];
        lat->deg[i] = (uint8_t)a.size();
        lat->sub[i] = (uint8_t)(((s.first + s.second) % 2 + 2) % 2);
    }
    return lat;
}

int brick_degree(const std::set<Site>& alive, const Site& s) {
    int d = 0;
    if (alive.count({s.first, s.second - 1})) ++d;
    if (alive.count({s.first, s.second + 1})) ++d;
    if (vertical_up(s.first, s.second) ? alive.count({s.first + 1, s.second})
                                       : alive.count({s.first - 1, s.second}))
        ++d;
    return d;
}

ftwa_lattice build_torus(int L1, int L2, double t) {
    auto* lat = new ftwa_lattice_s;
    const int N = 2 * L1 * L2;
    lat->N = N;
    lat->t = t;
    std::vector<std::set<int>> adj(N);
    auto site = [&](int x, int y, int b) { return 2 * (x * L2 + y) + b; };
    for (int x = 0; x < L1; ++x)
        for (int y = 0; y < L2; ++y) {
            const int A = site(x, y, 0);
            const int partners[3] = {site(x, y, 1), site((x + L1 - 1) % L1, y, 1),
                                     site(x, (y + L2 - 1) % L2, 1)};
            for (int B : partners) { adj[A].insert(B); adj[B].insert(A); }
        }
    lat->nbr.assign((size_t)N * kMaxDeg, -1);
    lat->deg.assign(N, 0);
    lat->sub.assign(N, 0);
    int twice_bonds = 0;
    for (int i = 0; i < N; ++i) {
        int k = 0;
        for (int j : adj[i]) lat->nbr[(size_t)i * kMaxDeg + k++] = j;  // std::set is ascending
        lat->deg[i] = (uint8_t)k;
        lat->sub[i] = (uint8_t)(i & 1);
        twice_bonds += k;
    }
    lat->n_bonds = twice_bonds / 2;
    return lat;
}

ftwa_lattice build_armchair(int R, int C, double t) {
    std::set<Site> alive;
    for (int r = 0; r < R; ++r)
        for (int c = 0; c < C; ++c) alive.insert({r, c});
    // remove dangling sites (degree < 2) until none is left
    std::deque<Site> queue(alive.begin(), alive.end());
    while (!queue.empty()) {
        Site s = queue.front();
        queue.pop_front();
        if (!alive.count(s) || brick_degree(alive, s) >= 2) continue;
        alive.erase(s);
        const Site around[4] = {{s.first, s.second - 1}, {s.first, s.second + 1},
                                {s.first + 1, s.second}, {s.first - 1, s.second}};
        for (const Site& n : around)
            if (alive.count(n)) queue.push_back(n);
    }
    return alive.empty() ? nullptr : from_brick_sites(alive, t);
}

ftwa_lattice build_hex_flake(int rings, double t) {
    // hexagon with axial coordinates (q, w) has lower-left brick-wall site
    // (row w, column 2q + w) and spans rows w..w+1, columns 2q+w..2q+w+2
    std::set<Site> sites;
    const int R = rings - 1;
    for (int q = -R; q <= R; ++q)
        for (int w = -R; w <= R; ++w) {
            const int s = -q - w;
            if (std::max({std::abs(q), std::abs(w), std::abs(s)}) > R) continue;
            for (int dr = 0; dr <= 1; ++dr)
                for (int dc = 0; dc <= 2; ++dc) sites.insert({w + dr, 2 * q + w + dc});
        }
    return from_brick_sites(sites, t);
}

}  // namespace

ftwa_status fail(ftwa_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

ftwa_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return FTWA_EHIP;
}

const char* last_error() { return g_last_error.c_str(); }

}  // namespace ftwa

using namespace ftwa;

extern "C" {

const char* ftwa_last_error(void) { return ftwa::last_error(); }

ftwa_status ftwa_build_lattice(ftwa_lattice_kind kind, int a, int b, double t_hop,
                               ftwa_lattice* out) {
    if (!out) return fail(FTWA_EINVAL, "ftwa_build_lattice: out is NULL");
    *out = nullptr;
    ftwa_lattice lat = nullptr;
    switch (kind) {
        case FTWA_TORUS:
            if (a < 2 || b < 2) return fail(FTWA_EINVAL, "torus needs a, b >= 2");
            if (2LL * a * b > kMaxSites) return fail(FTWA_EINVAL, "more than 255 sites");
            lat = build_torus(a, b, t_hop);
            break;
        case FTWA_ARMCHAIR_RECT:
            if (a < 2 || b < 2) return fail(FTWA_EINVAL, "rectangle needs a, b >= 2");
            if ((long long)a * b > 4 * kMaxSites) return fail(FTWA_EINVAL, "rectangle too large");
            lat = build_armchair(a, b, t_hop);
            break;
        case FTWA_HEX_ZIGZAG:
            if (a < 1 || 6LL * a * a > kMaxSites) return fail(FTWA_EINVAL, "hex flake rings out of range");
            lat = build_hex_flake(a, t_hop);
            break;
        default:
            return fail(FTWA_EINVAL, "unknown lattice kind");
    }
    if (!lat) return fail(FTWA_EINVAL, "lattice construction failed");
    if (lat->N > kMaxSites || lat->N < 1) {
        delete lat;
        return fail(FTWA_EINVAL, "lattice has more than 255 sites");
    }
    compute_host_tables(lat);
    *out = lat;
    return FTWA_OK;
}

ftwa_status ftwa_build_lattice_bonds(int n_sites, int n_bonds, const int32_t* bonds,
                                     const uint8_t* sublattice, double t_hop,
                                     ftwa_lattice* out) {
    if (!out) return fail(FTWA_EINVAL, "ftwa_build_lattice_bonds: out is NULL");
    *out = nullptr;
    if (n_sites < 1 || n_sites > kMaxSites) return fail(FTWA_EINVAL, "n_sites out of range");
    if (n_bonds < 0 || (n_bonds > 0 && !bonds)) return fail(FTWA_EINVAL, "bad bond list");
    std::vector<std::set<int>> adj(n_sites);
    for (int k = 0; k < n_bonds; ++k) {
        int u = bonds[2 * k], v = bonds[2 * k + 1];
        if (u < 0 || v < 0 || u >= n_sites || v >= n_sites || u == v)
            return fail(FTWA_EINVAL, "bond endpoint out of range or self bond");
        if (adj[u].count(v)) return fail(FTWA_EINVAL, "duplicate bond");
        adj[u].insert(v);
        adj[v].insert(u);
        if (adj[u].size() > (size_t)kMaxDeg || adj[v].size() > (size_t)kMaxDeg)
            return fail(FTWA_EINVAL, "site degree above 3");
    }
    auto* lat = new ftwa_lattice_s;
    lat->N = n_sites;
    lat->n_bonds = n_bonds;
    lat->t = t_hop;
    lat->nbr.assign((size_t)n_sites * kMaxDeg, -1);
    lat->deg.assign(n_sites, 0);
    lat->sub.assign(n_sites, 0);
    for (int i = 0; i < n_sites; ++i) {
        int k = 0;
        for (int j : adj[i]) lat->nbr[(size_t)i * kMaxDeg + k++] = j;
        lat->deg[i] = (uint8_t)k;
        lat->sub[i] = sublattice ? (uint8_t)(sublattice[i] & 1) : 0;
    }
    compute_host_tables(lat);
    *out = lat;
    return FTWA_OK;
}

ftwa_status ftwa_lattice_info(ftwa_lattice lat, int* n_sites, int* n_bonds, const int32_t** nbr,
                              const uint8_t** deg, const uint8_t** sublattice) {
    if (!lat) return fail(FTWA_EINVAL, "ftwa_lattice_info: NULL lattice");
    if (n_sites) *n_sites = lat->N;
    if (n_bonds) *n_bonds = lat->n_bonds;
    if (nbr) *nbr = lat->nbr.data();
    if (deg) *deg = lat->deg.data();
    if (sublattice) *sublattice = lat->sub.data();
    return FTWA_OK;
}

void ftwa_free_lattice(ftwa_lattice lat) {
    if (!lat) return;
    if (lat->dev.empty() && lat->padded.empty() && lat->split.empty()) {
        delete lat;  // never uploaded: no HIP call
        return;
    }
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto& [dev, tab] : lat->dev) {
        if (hipSetDevice(dev) != hipSuccess) continue;
        (void)hipFree(tab.nb);
        (void)hipFree(tab.off);
        (void)hipFree(tab.elem);
        if (tab.ord) (void)hipFree(tab.ord);
        if (tab.dpos) (void)hipFree(tab.dpos);
        if (tab.rdesc) (void)hipFree(tab.rdesc);
        if (tab.rdescf) (void)hipFree(tab.rdescf);
    }
    for (auto& [key, ptr] : lat->padded) {
        if (hipSetDevice(std::get<0>(key)) != hipSuccess) continue;
        (void)hipFree(ptr);
    }
    for (auto& [key, val] : lat->split) {
        if (hipSetDevice(std::get<0>(key)) != hipSuccess) continue;
        (void)hipFree(std::get<0>(val));
    }
    if (cur >= 0) (void)hipSetDevice(cur);
    delete lat;
}

ftwa_status ftwa_fock_start(ftwa_lattice lat, ftwa_start kind, uint64_t seed, uint32_t instance,
                            double* n0_host) {
    if (!lat || !n0_host) return fail(FTWA_EINVAL, "ftwa_fock_start: NULL argument");
    const int N = lat->N;
    if (kind == FTWA_START_NEEL) {
        for (int i = 0; i < N; ++i) {
            n0_host[i] = lat->sub[i] ? 0.0 : 1.0;
            n0_host[N + i] = lat->sub[i] ? 1.0 : 0.0;
        }
        return FTWA_OK;
    }
    if (kind != FTWA_START_RANDOM) return fail(FTWA_EINVAL, "unknown start kind");
    if (N % 2) return fail(FTWA_EINVAL, "random half filling needs an even number of sites");
    std::vector<int> order(N);
    for (int i = 0; i < N; ++i) order[i] = i;
    for (int i = N - 1; i > 0; --i) {
        const PhiloxBlock x = philox4x32_10({(uint32_t)i, instance, 0u, 1u}, seed);
        const uint64_t a = x.bits53_first();
        const int j = (int)(((unsigned __int128)a * (unsigned)(i + 1)) >> 53);
        std::swap(order[i], order[j]);
    }
    for (int k = 0; k < N; ++k) {
        const bool up = k < N / 2;
        n0_host[order[k]] = up ? 1.0 : 0.0;
        n0_host[N + order[k]] = up ? 0.0 : 1.0;
    }
    return FTWA_OK;
}

}  // extern "C"

namespace ftwa {

// Two-colours the lattice graph (breadth first).  On a bipartite graph every
// stencil read of an element (i, j) with i, j on the same sublattice ("even")
// touches only elements joining different sublattices ("odd") and vice versa,
// which lets the resident kernel update the two classes in separate phases.
//
// Of each pair {i, j} the resident kernel stores one orientation rho_ab, a
// ranking no later than b in a Cuthill-McKee order of the sites (breadth
// first from a site of least degree, neighbours by ascending degree).  That
// order keeps bonded sites close, so an element reads a neighbour stored as
// its transpose only when a and b are close in rank: a small set, placed at
// the front of its class, and every other element takes the kernel's
// conjugation-free path.
//
// Class order of the stored elements: the even class (the diagonal first,
// (i,i) at position i, then the elements that read a transpose, then the
// rest), then the odd class (those that read a transpose, then the rest),
// each group ordered by the ranks of (a, b).  An element's position in this
// order is its slot in the kernel's LDS block.  Returns false for a
// non-bipartite graph.
bool build_class_order(ftwa_lattice lat, std::vector<uint32_t>* order, int64_t* n_even,
                       std::vector<int32_t>* diag_pos, int64_t* n_gen_even,
                       int64_t* n_gen_odd, std::vector<int32_t>* rank_out) {
    const int N = lat->N;
    std::vector<int> colour(N, -1);
    for (int root = 0; root < N; ++root) {
        if (colour[root] >= 0) continue;
        colour[root] = 0;
        std::deque<int> q{root};
        while (!q.empty()) {
            const int u = q.front();
            q.pop_front();
            for (int k = 0; k < lat->deg[u]; ++k) {
                const int v = lat->nbr[(size_t)u * kMaxDeg + k];
                if (colour[v] < 0) { colour[v] = 1 - colour[u]; q.push_back(v); }
                else if (colour[v] == colour[u]) return false;
            }
        }
    }
    diag_pos->assign(N, 0);
    int next = 0;
    for (int c = 0; c < 2; ++c)
        for (int i = 0; i < N; ++i)
            if (colour[i] == c) (*diag_pos)[i] = next++;

    // Cuthill-McKee rank of every site (each connected component in turn)
    std::vector<int> rank(N, -1);
    int r = 0;
    while (r < N) {
        int root = -1;
        for (int i = 0; i < N; ++i)
            if (rank[i] < 0 && (root < 0 || lat->deg[i] < lat->deg[root])) root = i;
        rank[root] = r++;
        std::deque<int> q{root};
        while (!q.empty()) {
            const int u = q.front();
            q.pop_front();
            int nb[kMaxDeg], n = 0;
            for (int k = 0; k < lat->deg[u]; ++k) nb[n++] = lat->nbr[(size_t)u * kMaxDeg + k];
            std::stable_sort(nb, nb + n, [&](int x, int y) { return lat->deg[x] < lat->deg[y]; });
            for (int k = 0; k < n; ++k)
                if (rank[nb[k]] < 0) { rank[nb[k]] = r++; q.push_back(nb[k]); }
        }
    }
    // stored element (a, b) of rho_ab, rank[a] <= rank[b]; it reads a
    // transpose when a column neighbour rho_ak (k in nb(b)) has rank[k] <
    // rank[a] or a row neighbour rho_kb (k in nb(a)) has rank[k] > rank[b]
    auto reads_transpose = [&](int a, int b) {
        for (int k = 0; k < lat->deg[b]; ++k)
            if (rank[lat->nbr[(size_t)b * kMaxDeg + k]] < rank[a]) return true;
        for (int k = 0; k < lat->deg[a]; ++k)
            if (rank[lat->nbr[(size_t)a * kMaxDeg + k]] > rank[b]) return true;
        return false;
    };
    std::vector<int> by_rank(N);
    for (int i = 0; i < N; ++i) by_rank[rank[i]] = i;
    auto ab = [](int a, int b) { return (uint32_t)a | ((uint32_t)b << 16); };
    order->clear();
    order->reserve((size_t)packed_count(N));
    for (int i = 0; i < N; ++i) order->push_back(ab(i, i));
    for (int cls = 0; cls < 2; ++cls) {
        const size_t start = order->size();
        std::vector<uint32_t> rest;
        for (int ra = 0; ra < N; ++ra)
            for (int rb = ra + 1; rb < N; ++rb) {
                const int a = by_rank[ra], b = by_rank[rb];
                if ((colour[a] != colour[b]) != (cls == 1)) continue;
                if (reads_transpose(a, b)) order->push_back(ab(a, b));
                else rest.push_back(ab(a, b));
            }
        if (cls == 0) *n_gen_even = (int64_t)order->size();
        else *n_gen_odd = (int64_t)(order->size() - start);
        order->insert(order->end(), rest.begin(), rest.end());
        if (cls == 0) *n_even = (int64_t)order->size();
    }
    rank_out->assign(rank.begin(), rank.end());
    return true;
}

namespace {

// One part of the split layout of a spin block (see split_tables).
struct SplitPart {
    std::vector<int64_t> interior;   // even, read no other part's element (transpose readers first)
    std::vector<int64_t> boundary;   // even: the diagonal, then the exported (transpose readers first)
    std::vector<int64_t> odd;        // transpose readers (exported first), exported, rest
    std::vector<int64_t> halo;       // elements read from other parts, even class first,
                                     // then by producer part and producer slot
    int n_halo_even = 0;
    int n_diag = 0;
    int int_gen = 0, bnd_gen = 0, odd_gen = 0, odd_x = 0;
};

// Owned elements in LDS-slot order: interior, boundary, odd.
std::vector<int64_t> owned(const SplitPart& sp) {
    std::vector<int64_t> v(sp.interior);
    v.insert(v.end(), sp.boundary.begin(), sp.boundary.end());
    v.insert(v.end(), sp.odd.begin(), sp.odd.end());
    return v;
}

// The rows of the stored elements (sites in rank order; the stored element
// rho_ab has rank a <= rank b and belongs to row a) cut into G strips; part p
// owns the elements of strip p.  An inner strip exchanges with two
// neighbours, an end strip with one, so for G > 2 the end strips take a
// larger share of the elements (1 + a each, the inner ones the rest; a =
// kEndShare, small enough that the configurations still hold the parts).  An
// element is exported when a stencil of another part reads it (it then reads
// that part's elements itself: the stencil relation is symmetric), and every
// diagonal element is (the other spin's U term reads it).
std::vector<SplitPart> split_layout(const ftwa_lattice_s& L, int G, int64_t n_even,
                                    int64_t n_gen_even, int64_t n_gen_odd) {
    const int N = L.N;
    const std::vector<uint32_t>& order = L.class_order;
    const int64_t P = packed_count(N), n = (int64_t)order.size();
    const double kEndShare = G == 3 ? 0.05 : 0.02;
    std::vector<double> upto(G);  // elements up to the end of strip p
    double acc = 0.0;
    for (int p = 0; p < G; ++p) {
        const double w = G <= 2 ? 1.0
                                : (p == 0 || p == G - 1 ? 1.0 + kEndShare
                                                        : 1.0 - 2.0 * kEndShare / (G - 2));
        acc += w;
        upto[p] = acc / G * (double)P;
    }
    std::vector<int> strip(N);
    int64_t before = 0;
    for (int r = 0; r < N; ++r) {
        const double mid = (double)before + 0.5 * (N - r);  // the row's middle element
        int sp = 0;
        while (sp < G - 1 && mid >= upto[sp]) ++sp;
        strip[r] = sp;
        before += N - r;
    }
    std::vector<int64_t> q_of((size_t)P);
    for (int64_t q = 0; q < n; ++q) {
        const int a = (int)(order[q] & 0xffffu), b = (int)(order[q] >> 16);
        const int i = std::min(a, b), j = std::max(a, b);
        q_of[(size_t)(packed_row(N, i) + (j - i))] = q;
    }
    auto q_at = [&](int x, int y) {
        const int i = std::min(x, y), j = std::max(x, y);
        return q_of[(size_t)(packed_row(N, i) + (j - i))];
    };
    auto part_of = [&](int64_t q) { return strip[L.rank[order[q] & 0xffffu]]; };
    std::vector<uint8_t> exported((size_t)n, 0);
    std::vector<std::vector<uint8_t>> in_halo(G, std::vector<uint8_t>((size_t)n, 0));
    std::vector<SplitPart> parts(G);
    for (int64_t q = 0; q < n; ++q) {
        const int a = (int)(order[q] & 0xffffu), b = (int)(order[q] >> 16);
        const int pe = part_of(q);
        auto touch = [&](int64_t r) {
            if (part_of(r) == pe) return;
            exported[(size_t)r] = 1;
            if (!in_halo[pe][(size_t)r]) {
                in_halo[pe][(size_t)r] = 1;
                parts[pe].halo.push_back(r);
            }
        };
        for (int k = 0; k < L.deg[b]; ++k) touch(q_at(a, L.nbr[(size_t)b * kMaxDeg + k]));
        for (int k = 0; k < L.deg[a]; ++k) touch(q_at(L.nbr[(size_t)a * kMaxDeg + k], b));
    }
    for (int i = 0; i < N; ++i) exported[(size_t)i] = 1;  // (i,i) sits at class-order index i
    auto gen_e = [&](int64_t q) { return q < n_gen_even; };  // (includes the diagonal)
    auto gen_o = [&](int64_t q) { return q - n_even < n_gen_odd; };
    for (int p = 0; p < G; ++p) {
        SplitPart& sp = parts[p];
        std::vector<int64_t> ig, ir, bg, br, og_x, og, ox, orr;
        for (int64_t q = 0; q < n; ++q) {
            if (part_of(q) != p) continue;
            if (q < N) sp.boundary.push_back(q);
            else if (q < n_even) (exported[(size_t)q] ? (gen_e(q) ? bg : br) : (gen_e(q) ? ig : ir)).push_back(q);
            else if (gen_o(q)) (exported[(size_t)q] ? og_x : og).push_back(q);
            else (exported[(size_t)q] ? ox : orr).push_back(q);
        }
        sp.n_diag = (int)sp.boundary.size();
        sp.interior = ig;
        sp.interior.insert(sp.interior.end(), ir.begin(), ir.end());
        sp.int_gen = (int)ig.size();
        sp.boundary.insert(sp.boundary.end(), bg.begin(), bg.end());
        sp.bnd_gen = (int)sp.boundary.size();
        sp.boundary.insert(sp.boundary.end(), br.begin(), br.end());
        sp.odd = og_x;
        sp.odd.insert(sp.odd.end(), og.begin(), og.end());
        sp.odd_gen = (int)sp.odd.size();
        sp.odd.insert(sp.odd.end(), ox.begin(), ox.end());
        sp.odd_x = ox.empty() ? (int)og_x.size() : (int)sp.odd.size();
        sp.odd.insert(sp.odd.end(), orr.begin(), orr.end());
    }
    // producer slots, then the halo order
    std::vector<int> slot_q((size_t)n);
    for (int p = 0; p < G; ++p) {
        const std::vector<int64_t> own = owned(parts[p]);
        for (size_t e = 0; e < own.size(); ++e) slot_q[(size_t)own[e]] = (int)e;
    }
    for (int p = 0; p < G; ++p) {
        SplitPart& sp = parts[p];
        auto hk = [&](int64_t q) {
            return std::make_tuple(q >= n_even, part_of(q), slot_q[(size_t)q]);
        };
        std::sort(sp.halo.begin(), sp.halo.end(), [&](int64_t x, int64_t y) { return hk(x) < hk(y); });
        sp.n_halo_even = 0;
        for (int64_t q : sp.halo) sp.n_halo_even += q < n_even ? 1 : 0;
    }
    return parts;
}

SplitShape split_shape(const std::vector<SplitPart>& parts) {
    SplitShape s;
    for (const SplitPart& sp : parts) {
        const int ne = (int)(sp.interior.size() + sp.boundary.size());
        s.n_even = std::max(s.n_even, ne);
        s.n_odd = std::max(s.n_odd, (int)sp.odd.size());
        s.int_gen = std::max(s.int_gen, sp.int_gen);
        s.n_bnd = std::max(s.n_bnd, (int)sp.boundary.size());
        s.bnd_gen = std::max(s.bnd_gen, sp.bnd_gen);
        s.odd_gen = std::max(s.odd_gen, sp.odd_gen);
        s.odd_x = std::max(s.odd_x, sp.odd_x);
        s.max_halo = std::max(s.max_halo, (int)sp.halo.size());
        s.max_slots = std::max(s.max_slots, ne + (int)(sp.odd.size() + sp.halo.size()));
    }
    return s;
}

}  // namespace

std::string split_key(int dev, int G, int64_t even_slots, int64_t odd_slots, int64_t bnd_entry,
                      int elem_bytes) {
    return "s" + std::to_string(dev) + ":" + std::to_string(G) + ":" + std::to_string(even_slots) +
           ":" + std::to_string(odd_slots) + ":" + std::to_string(bnd_entry) + ":" +
           std::to_string(elem_bytes);
}

std::string padded_key(int dev, int64_t even_slots, int64_t odd_slots, int elem_bytes,
                       bool compact) {
    return "p" + std::to_string(dev) + ":" + std::to_string(even_slots) + ":" +
           std::to_string(odd_slots) + ":" + std::to_string(elem_bytes) + ":" +
           std::to_string(compact ? 1 : 0);
}

// A table that ftwa_lattice_upload could not build for this device: the
// error it met then, else "not uploaded".
ftwa_status missing_table(ftwa_lattice lat, const std::string& key) {
    auto it = lat->table_err.find(key);
    if (it != lat->table_err.end()) return fail(it->second.first, it->second.second);
    return fail(FTWA_EINVAL,
                "the lattice's kernel tables are not on this device: call ftwa_lattice_upload first");
}

ftwa_status split_tables(ftwa_lattice lat, int G, int64_t even_slots, int64_t odd_slots,
                         int64_t bnd_entry, int elem_bytes, const void** out, int* part_words,
                         int* hmax, bool create) {
    const DeviceTables& tab = host_tables(lat);
    if (!tab.bipartite) return fail(FTWA_ENOTSUP, "lattice is not bipartite");
    if (G < 2 || G > kMaxParts) return fail(FTWA_EINVAL, "split: part count out of range");
    const int N = lat->N;
    if (N > 256) return fail(FTWA_EINVAL, "split: more than 256 sites");
    if (even_slots % 64 || odd_slots % 64) return fail(FTWA_EINVAL, "split: slots not whole waves");
    int dev = 0;
    FTWA_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(lat->mu);
    const auto key = std::make_tuple(dev, G, even_slots, odd_slots, bnd_entry, elem_bytes);
    auto it = lat->split.find(key);
    if (it != lat->split.end()) {
        *out = std::get<0>(it->second);
        *part_words = std::get<1>(it->second);
        *hmax = std::get<2>(it->second);
        return FTWA_OK;
    }
    if (!create)
        return missing_table(lat, split_key(dev, G, even_slots, odd_slots, bnd_entry, elem_bytes));
    const std::vector<uint32_t>& order = lat->class_order;
    const int64_t n = (int64_t)order.size();
    const std::vector<SplitPart> parts =
        split_layout(*lat, G, tab.n_even, tab.n_gen_even, tab.n_gen_odd);
    const int64_t E = even_slots + odd_slots;
    int H = 1;
    for (const SplitPart& sp : parts) H = std::max(H, (int)sp.halo.size());
    const int64_t pw = (8 + 4 * E + E + H + 256 + 3) / 4 * 4;
    std::vector<uint32_t> blob((size_t)(pw * G + N), 0u);
    std::vector<int> part_q((size_t)n), slot_q((size_t)n);
    for (int p = 0; p < G; ++p) {
        const SplitPart& sp = parts[p];
        const int64_t ne = (int64_t)(sp.interior.size() + sp.boundary.size());
        if (ne > even_slots || (int64_t)sp.odd.size() > odd_slots ||
            (int64_t)sp.boundary.size() > even_slots - bnd_entry)
            return fail(FTWA_EINVAL, "split: padding too small");
        const std::vector<int64_t> own = owned(sp);
        if (own.size() + sp.halo.size() + 33 > 0x7fff)
            return fail(FTWA_EINVAL, "split: part too large for 15-bit slots");
        for (size_t e = 0; e < own.size(); ++e) {
            part_q[(size_t)own[e]] = p;
            slot_q[(size_t)own[e]] = (int)e;
        }
    }
    std::vector<int64_t> q_of((size_t)packed_count(N));
    for (int64_t q = 0; q < n; ++q) {
        const int a = (int)(order[q] & 0xffffu), b = (int)(order[q] >> 16);
        const int i = std::min(a, b), j = std::max(a, b);
        q_of[(size_t)(packed_row(N, i) + (j - i))] = q;
    }
    // lanes that share one LDS pass and the slot residues that spread them
    // over the banks: 64 banks of 4 bytes
    const int R = 64 / (elem_bytes / 4);
    std::vector<int> hslot((size_t)n, -1);
    for (int p = 0; p < G; ++p) {
        const SplitPart& sp = parts[p];
        uint32_t* pb = blob.data() + (size_t)p * pw;
        const int n_ev = (int)(sp.interior.size() + sp.boundary.size());
        const int n_own = n_ev + (int)sp.odd.size();
        const int Z0 = n_own + (int)sp.halo.size();
        pb[0] = (uint32_t)n_ev;
        pb[1] = (uint32_t)n_own;
        pb[2] = (uint32_t)sp.n_halo_even;
        pb[3] = (uint32_t)(sp.halo.size() - sp.n_halo_even);
        pb[4] = (uint32_t)sp.n_diag;
        std::fill(hslot.begin(), hslot.end(), -1);
        for (size_t h = 0; h < sp.halo.size(); ++h) hslot[(size_t)sp.halo[h]] = n_own + (int)h;
        struct Ref {
            int slot;  // -1: missing neighbour (a zero slot)
            bool conj;
        };
        auto ref = [&](int x, int y) -> Ref {
            const int i = std::min(x, y), j = std::max(x, y);
            const int64_t q = q_of[(size_t)(packed_row(N, i) + (j - i))];
            const int a = (int)(order[q] & 0xffffu);
            const bool conj = x != y && a != x;
            const int s = part_q[(size_t)q] == p ? slot_q[(size_t)q] : hslot[(size_t)q];
            return Ref{s, conj};
        };
        struct Ent {
            Ref n[6];
            int own;
            bool exported;
            int a, b;
        };
        std::vector<Ent> ent((size_t)E);
        for (Ent& e : ent) {
            for (int k = 0; k < 6; ++k) e.n[k] = Ref{-1, false};
            e.own = Z0 + 32;  // padding entries own the scratch slot
            e.exported = false;
            e.a = e.b = -1;
        }
        std::vector<uint8_t> is_export((size_t)n, 0);
        for (int pp = 0; pp < G; ++pp)
            if (pp != p)
                for (int64_t q : parts[pp].halo) is_export[(size_t)q] = 1;
        for (int i = 0; i < N; ++i) is_export[(size_t)i] = 1;
        auto fill = [&](int64_t q, int64_t at, bool gen) -> bool {
            const int a = (int)(order[q] & 0xffffu), b = (int)(order[q] >> 16);
            Ent& e = ent[(size_t)at];
            for (int k = 0; k < kMaxDeg; ++k) {
                if (k < lat->deg[b]) e.n[k] = ref(a, lat->nbr[(size_t)b * kMaxDeg + k]);
                if (k < lat->deg[a]) e.n[3 + k] = ref(lat->nbr[(size_t)a * kMaxDeg + k], b);
            }
            for (int k = 0; k < 6; ++k) {
                if (e.n[k].slot == -1 && ((k < 3 && k < lat->deg[b]) || (k >= 3 && k - 3 < lat->deg[a])))
                    return false;  // a neighbour neither owned nor in the halo
                if (e.n[k].conj && !gen) return false;
            }
            e.own = slot_q[(size_t)q];
            e.exported = is_export[(size_t)q] != 0;
            e.a = a;
            e.b = b;
            return true;
        };
        // even entries: interior up to bnd_entry, boundary from bnd_entry,
        // the interior overflow after it
        const int64_t n_int0 = std::min<int64_t>((int64_t)sp.interior.size(), bnd_entry);
        for (int64_t k = 0; k < n_int0; ++k)
            if (!fill(sp.interior[(size_t)k], k, k < sp.int_gen))
                return fail(FTWA_ENOTSUP, "split: inconsistent stencil (interior)");
        for (size_t k = 0; k < sp.boundary.size(); ++k)
            if (!fill(sp.boundary[k], bnd_entry + (int64_t)k, (int)k < sp.bnd_gen))
                return fail(FTWA_ENOTSUP, "split: inconsistent stencil (boundary)");
        for (int64_t k = n_int0; k < (int64_t)sp.interior.size(); ++k)
            if (!fill(sp.interior[(size_t)k], bnd_entry + (int64_t)sp.boundary.size() + (k - n_int0),
                      k < sp.int_gen))
                return fail(FTWA_ENOTSUP, "split: inconsistent stencil (interior)");
        for (size_t k = 0; k < sp.odd.size(); ++k)
            if (!fill(sp.odd[k], even_slots + (int64_t)k, (int)k < sp.odd_gen))
                return fail(FTWA_ENOTSUP, "split: inconsistent stencil (odd class)");
        // missing neighbours: the zero slot whose bank residue no other lane
        // of the pass reads for that field
        // (each class is a whole number of passes: even_slots is a multiple of 64)
        for (int64_t c0 = 0; c0 < E; c0 += R) {
            const int64_t c1 = std::min<int64_t>(c0 + R, E);
            for (int k = 0; k < 6; ++k) {
                uint32_t used = 0;
                for (int64_t x = c0; x < c1; ++x)
                    if (ent[(size_t)x].n[k].slot >= 0) used |= 1u << (ent[(size_t)x].n[k].slot % R);
                int z = Z0;
                for (int r = 0; r < 32; ++r)
                    if (!(used >> ((Z0 + r) % R) & 1u)) { z = Z0 + r; break; }
                for (int64_t x = c0; x < c1; ++x)
                    if (ent[(size_t)x].n[k].slot < 0) ent[(size_t)x].n[k].slot = z;
            }
        }
        uint32_t* dsc = pb + 8;
        uint32_t* pord = dsc + 4 * E;
        uint32_t* imp = pord + E;
        uint32_t* dsite = imp + H;
        auto f = [](const Ref& r) { return (uint32_t)r.slot | (r.conj ? 0x8000u : 0u); };
        for (int64_t x = 0; x < E; ++x) {
            const Ent& e = ent[(size_t)x];
            const uint32_t pi = e.a < 0 ? 0u : (uint32_t)lat->diag_pos[e.a];
            const uint32_t pj = e.b < 0 ? 0u : (uint32_t)lat->diag_pos[e.b];
            dsc[4 * x + 0] = f(e.n[0]) | f(e.n[1]) << 16;
            dsc[4 * x + 1] = f(e.n[2]) | f(e.n[3]) << 16;
            dsc[4 * x + 2] = f(e.n[4]) | f(e.n[5]) << 16;
            dsc[4 * x + 3] = (uint32_t)e.own | (e.exported ? 0x8000u : 0u) | pi << 16 | pj << 24;
            if (e.a >= 0) pord[e.own] = (uint32_t)e.a | (uint32_t)e.b << 16;
        }
        for (size_t h = 0; h < sp.halo.size(); ++h) {
            const int64_t q = sp.halo[h];
            imp[h] = (uint32_t)part_q[(size_t)q] << 16 | (uint32_t)slot_q[(size_t)q];
        }
        for (int t = 0; t < sp.n_diag; ++t) dsite[t] = order[(size_t)sp.boundary[(size_t)t]] & 0xffffu;
    }
    uint32_t* dsrc = blob.data() + (size_t)G * pw;
    for (int i = 0; i < N; ++i) dsrc[i] = (uint32_t)part_q[(size_t)i] << 16 | (uint32_t)slot_q[(size_t)i];
    void* d = nullptr;
    FTWA_HIP_TRY(hipMalloc(&d, blob.size() * sizeof(uint32_t)));
    FTWA_HIP_TRY(hipMemcpy(d, blob.data(), blob.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    lat->split[key] = std::make_tuple(d, (int)pw, H);
    *out = d;
    *part_words = (int)pw;
    *hmax = H;
    return FTWA_OK;
}

ftwa_status padded_descriptors(ftwa_lattice lat, int64_t even_slots, int64_t odd_slots,
                               int elem_bytes, bool compact, const void** out, bool create) {
    const DeviceTables& tab = host_tables(lat);
    if (!tab.bipartite) return fail(FTWA_ENOTSUP, "lattice is not bipartite");
    const int N = lat->N;
    const int64_t P = packed_count(N);
    const std::vector<uint32_t>& order = lat->class_order;
    const int64_t n_even = tab.n_even, n_odd = (int64_t)order.size() - n_even;
    if (even_slots < n_even || odd_slots < n_odd) return fail(FTWA_EINVAL, "padding too small");
    if ((P + 2) * (int64_t)elem_bytes >= ((int64_t)1 << 31))
        return fail(FTWA_EINVAL, "lattice too large for the resident layout");
    if (compact && (P + 33 > 0x8000 || N > 256))
        return fail(FTWA_EINVAL, "lattice too large for compact descriptors");
    int dev = 0;
    FTWA_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(lat->mu);
    const auto key =
        std::make_tuple(dev, even_slots, odd_slots, elem_bytes * 2 + (compact ? 1 : 0));
    auto it = lat->padded.find(key);
    if (it != lat->padded.end()) {
        *out = it->second;
        return FTWA_OK;
    }
    if (!create) return missing_table(lat, padded_key(dev, even_slots, odd_slots, elem_bytes, compact));
    // LDS slot of every pair {i, j} (packed index of i <= j) and whether the
    // slot holds rho_ij (a = min) or rho_ji
    std::vector<uint32_t> slot((size_t)P);
    std::vector<uint8_t> lower((size_t)P, 0);
    for (size_t q = 0; q < order.size(); ++q) {
        const int a = (int)(order[q] & 0xffffu), b = (int)(order[q] >> 16);
        const int i = std::min(a, b), j = std::max(a, b);
        slot[(size_t)(packed_row(N, i) + (j - i))] = (uint32_t)q;
        lower[(size_t)(packed_row(N, i) + (j - i))] = a > b;
    }
    // one element's stencil as slot numbers; conj: the slot holds the
    // transpose of the element read
    struct Ref {
        uint32_t slot;
        bool conj;
    };
    struct Sten {
        Ref n[6];  // c0 c1 c2 r0 r1 r2
        uint32_t own;
        int i, j;
    };
    auto ref = [&](int x, int y) -> Ref {
        const int i = std::min(x, y), j = std::max(x, y);
        const size_t p = (size_t)(packed_row(N, i) + (j - i));
        const bool stored_xy = (x <= y) != (lower[p] != 0) || x == y;
        return Ref{slot[p], !stored_xy};
    };
    auto stencil = [&](int i, int j) {
        Sten e;
        for (int n = 0; n < kMaxDeg; ++n) {
            const int kc = n < lat->deg[j] ? lat->nbr[(size_t)j * kMaxDeg + n] : -1;
            const int kr = n < lat->deg[i] ? lat->nbr[(size_t)i * kMaxDeg + n] : -1;
            e.n[n] = kc < 0 ? Ref{(uint32_t)P, false} : ref(i, kc);
            e.n[3 + n] = kr < 0 ? Ref{(uint32_t)P, false} : ref(kr, j);
        }
        e.own = ref(i, j).slot;
        e.i = i;
        e.j = j;
        return e;
    };
    std::vector<Sten> all((size_t)(even_slots + odd_slots));
    {
        Sten dummy;  // padding: reads the zero slot, owns the scratch slot
        for (int n = 0; n < 6; ++n) dummy.n[n] = Ref{(uint32_t)P, false};
        dummy.own = (uint32_t)(P + 1);
        dummy.i = dummy.j = -1;
        std::fill(all.begin(), all.end(), dummy);
    }
    for (int64_t q = 0; q < (int64_t)order.size(); ++q) {
        const int a = (int)(order[q] & 0xffffu), b = (int)(order[q] >> 16);
        const int64_t at = q < n_even ? q : even_slots + (q - n_even);
        const Sten e = stencil(a, b);
        // past the leading groups no neighbour is a transpose (the kernel
        // reads those elements without the conjugation flags)
        const bool general = q < n_even ? q < tab.n_gen_even : q - n_even < tab.n_gen_odd;
        bool any = false;
        for (int n = 0; n < 6; ++n) any = any || e.n[n].conj;
        if (!general && any)
            return fail(FTWA_ENOTSUP, "class order: transpose read outside the leading group");
        if (e.own != (uint32_t)q) return fail(FTWA_ENOTSUP, "class order: element not stored");
        all[(size_t)at] = e;
    }
    void* d = nullptr;
    if (compact) {
        // 32 zero slots P..P+31 (scratch P+32): the lanes of one 32-lane
        // group that read a missing neighbour read the zero slot whose LDS
        // bank no other lane of the group reads for that field, so the zero
        // reads cost no bank conflict
        for (int64_t c0 = 0; c0 < even_slots + odd_slots; c0 += 32) {
            const int64_t c1 = std::min<int64_t>(c0 + 32, c0 < even_slots ? even_slots
                                                                          : even_slots + odd_slots);
            for (int n = 0; n < 6; ++n) {
                uint32_t used = 0;
                for (int64_t k = c0; k < c1; ++k)
                    if (all[(size_t)k].n[n].slot != (uint32_t)P) used |= 1u << (all[(size_t)k].n[n].slot % 32);
                uint32_t z = (uint32_t)P;
                for (uint32_t r = 0; r < 32; ++r)
                    if (!(used >> ((P + r) % 32) & 1u)) { z = (uint32_t)P + r; break; }
                for (int64_t k = c0; k < c1; ++k)
                    if (all[(size_t)k].n[n].slot == (uint32_t)P) all[(size_t)k].n[n].slot = z;
            }
            for (int64_t k = c0; k < c1; ++k)
                if (all[(size_t)k].own == (uint32_t)(P + 1)) all[(size_t)k].own = (uint32_t)(P + 32);
        }
        std::vector<uint4> tabp(all.size());
        auto f = [](const Ref& r) { return r.slot | (r.conj ? 0x8000u : 0u); };
        for (size_t k = 0; k < all.size(); ++k) {
            const Sten& e = all[k];
            const uint32_t pi = e.i < 0 ? 0u : (uint32_t)lat->diag_pos[e.i];
            const uint32_t pj = e.j < 0 ? 0u : (uint32_t)lat->diag_pos[e.j];
            tabp[k].x = f(e.n[0]) | f(e.n[1]) << 16;
            tabp[k].y = f(e.n[2]) | f(e.n[3]) << 16;
            tabp[k].z = f(e.n[4]) | f(e.n[5]) << 16;
            tabp[k].w = e.own | pi << 16 | pj << 24;
        }
        FTWA_HIP_TRY(hipMalloc(&d, tabp.size() * sizeof(uint4)));
        FTWA_HIP_TRY(hipMemcpy(d, tabp.data(), tabp.size() * sizeof(uint4), hipMemcpyHostToDevice));
    } else {
        const uint32_t eb = (uint32_t)elem_bytes;
        std::vector<ResDesc> tabp(all.size());
        auto f = [&](const Ref& r) { return r.slot * eb | (r.conj ? 0x80000000u : 0u); };
        for (size_t k = 0; k < all.size(); ++k) {
            const Sten& e = all[k];
            tabp[k].a = make_uint4(f(e.n[0]), f(e.n[1]), f(e.n[2]), e.own * eb);
            tabp[k].b = make_uint4(f(e.n[3]), f(e.n[4]), f(e.n[5]), 0u);
            if (e.i >= 0) tabp[k].b.w = ((uint32_t)e.i * eb) | (((uint32_t)e.j * eb) << 16);
        }
        FTWA_HIP_TRY(hipMalloc(&d, tabp.size() * sizeof(ResDesc)));
        FTWA_HIP_TRY(hipMemcpy(d, tabp.data(), tabp.size() * sizeof(ResDesc), hipMemcpyHostToDevice));
    }
    lat->padded[key] = d;
    *out = d;
    return FTWA_OK;
}

void compute_host_tables(ftwa_lattice lat) {
    DeviceTables& tab = lat->host;
    std::vector<uint32_t> order;
    std::vector<int32_t> dpos;
    std::vector<int32_t> rank;
    tab.bipartite = build_class_order(lat, &order, &tab.n_even, &dpos, &tab.n_gen_even,
                                      &tab.n_gen_odd, &rank);
    if (tab.bipartite) {
        lat->class_order = order;
        lat->diag_pos = dpos;
        lat->rank = rank;
        for (int G = 2; G <= kMaxParts; ++G)
            tab.split[G] = split_shape(
                split_layout(*lat, G, tab.n_even, tab.n_gen_even, tab.n_gen_odd));
    }
}

const DeviceTables& host_tables(ftwa_lattice lat) { return lat->host; }

ftwa_status device_tables(ftwa_lattice lat, DeviceTables* out) {
    int dev = 0;
    FTWA_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(lat->mu);
    auto it = lat->dev.find(dev);
    if (it == lat->dev.end())
        return fail(FTWA_EINVAL,
                    "the lattice's tables are not on this device: call ftwa_lattice_upload first");
    *out = it->second;
    return FTWA_OK;
}

std::vector<uint4> reverse_descriptors(const ftwa_lattice_s& lat, bool full) {
    const int N = lat.N;
    const int64_t P = packed_count(N), E = 2 * P;
    const uint32_t zero = full ? (uint32_t)(2 * N * N) : (uint32_t)E;
    std::vector<uint4> out((size_t)(2 * E));
    auto x_entry = [&](int s, int a, int b) -> uint32_t {  // element (a, b) of spin s
        if (full) return (uint32_t)((s * N + a) * N + b);
        const int i = std::min(a, b), j = std::max(a, b);
        return (uint32_t)(s * P + packed_row(N, i) + (j - i)) | (a > b ? 0x8000u : 0u);
    };
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < N; ++i)
            for (int j = i; j < N; ++j) {
                const int64_t e = s * P + packed_row(N, i) + (j - i);
                uint32_t f[6];
                for (int n = 0; n < kMaxDeg; ++n) {
                    const int kc = n < lat.deg[j] ? lat.nbr[(size_t)j * kMaxDeg + n] : -1;
                    const int kr = n < lat.deg[i] ? lat.nbr[(size_t)i * kMaxDeg + n] : -1;
                    f[n] = kc < 0 ? zero : x_entry(s, i, kc);
                    f[3 + n] = kr < 0 ? zero : x_entry(s, kr, j);
                }
                const uint32_t so = (uint32_t)((1 - s) * N);
                uint4& q0 = out[(size_t)(2 * e)];
                q0.x = f[0] | f[1] << 16;
                q0.y = f[2] | f[3] << 16;
                q0.z = f[4] | f[5] << 16;
                q0.w = (so + i) | (so + j) << 16;
                uint4& q1 = out[(size_t)(2 * e + 1)];
                q1.x = full ? x_entry(s, i, j) | x_entry(s, j, i) << 16
                            : (uint32_t)e | (uint32_t)e << 16;
                q1.y = (uint32_t)((s * N + i) * N + j) | (uint32_t)((s * N + j) * N + i) << 16;
                q1.z = (uint32_t)(s * N + i) | (i == j ? 1u << 16 : 0u);
                q1.w = (uint32_t)e;
            }
    return out;
}

ftwa_status upload_tables(ftwa_lattice lat) {
    int dev = 0;
    FTWA_HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(lat->mu);
    if (lat->dev.count(dev)) return FTWA_OK;
    const int N = lat->N;
    const int64_t P = packed_count(N);
    std::vector<int32_t> nb((size_t)N * 4), off(N);
    std::vector<uint32_t> elem((size_t)P);
    for (int i = 0; i < N; ++i) {
        for (int k = 0; k < kMaxDeg; ++k) nb[(size_t)i * 4 + k] = lat->nbr[(size_t)i * kMaxDeg + k];
        nb[(size_t)i * 4 + 3] = lat->deg[i];
        off[i] = (int32_t)packed_row(N, i);
        for (int j = i; j < N; ++j) elem[(size_t)(packed_row(N, i) + (j - i))] = (uint32_t)i | ((uint32_t)j << 16);
    }
    DeviceTables tab = lat->host;
    if (tab.bipartite) {
        const std::vector<uint32_t>& order = lat->class_order;
        const std::vector<int32_t>& dpos = lat->diag_pos;
        FTWA_HIP_TRY(hipMalloc(&tab.ord, order.size() * sizeof(uint32_t)));
        FTWA_HIP_TRY(hipMemcpy(tab.ord, order.data(), order.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice));
        FTWA_HIP_TRY(hipMalloc(&tab.dpos, dpos.size() * sizeof(int32_t)));
        FTWA_HIP_TRY(hipMemcpy(tab.dpos, dpos.data(), dpos.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice));
    }
    for (int full = 0; full < 2; ++full) {
        if (N > (full ? kReverseFullMaxSites : kReverseMaxSites)) continue;
        const std::vector<uint4> rd = reverse_descriptors(*lat, full != 0);
        uint4*& dst = full ? tab.rdescf : tab.rdesc;
        FTWA_HIP_TRY(hipMalloc(&dst, rd.size() * sizeof(uint4)));
        FTWA_HIP_TRY(hipMemcpy(dst, rd.data(), rd.size() * sizeof(uint4), hipMemcpyHostToDevice));
    }
    FTWA_HIP_TRY(hipMalloc(&tab.nb, nb.size() * sizeof(int32_t)));
    FTWA_HIP_TRY(hipMalloc(&tab.off, off.size() * sizeof(int32_t)));
    FTWA_HIP_TRY(hipMalloc(&tab.elem, elem.size() * sizeof(uint32_t)));
    FTWA_HIP_TRY(hipMemcpy(tab.nb, nb.data(), nb.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    FTWA_HIP_TRY(hipMemcpy(tab.off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    FTWA_HIP_TRY(hipMemcpy(tab.elem, elem.data(), elem.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    lat->dev[dev] = tab;
    return FTWA_OK;
}

}  // namespace ftwa
