// The LP relaxation of the Potts model (Sec. 6) on the device.
//
// Subgradient (eq. grad_lp): for each label i, order the pixels by y_a(i),
// descending (eq. simple_S; equal values keep ascending pixel index), and let
//   U_c = sum over pixels a after c of Kbar_ac,  Lo_c = sum over a before c,
// then g_c(i) = phi_c(i) + U_c - Lo_c and S_LP(y) = <g, y>.
//
// The two triangular sums are computed by the divide and conquer of App. E,
// level by level. At level l the sorted positions are split into nodes with
// boundaries floor(n N / 2^l); node n splits at floor((2n+1) N / 2^(l+1)).
// For every node with two non-empty halves, the indicator of the left half
// (channel 0) and of the right half (channel 1) are filtered over the node's
// points only: the right channel read at left points adds to U, the left
// channel read at right points adds to Lo. "Over the node's points only"
// means a permutohedral lattice built on those points: its vertices are the
// (node, global vertex) pairs touched by the node's points, found with a
// device hash keyed by node * M + v (a sub-vertex takes the number of the
// (position, vertex) entry that claims its slot), and its blur follows the
// global neighbour table, keeping neighbours present in the same node. Each node probes only its own region
// of the table (twice its entries), so the probes of neighbouring positions
// stay in a few cache lines; blocks map to XCDs in contiguous ranges of
// positions (xcd_block), so from the third level on a node's region and its
// sub-vertex rows are used by one XCD's L2.
// All nodes of a level are filtered in one pass, the first lattice on the
// context's stream and the others on a second stream joined before the
// slice; labels are processed one at a time (their hash tables then stay
// cache-resident).
//
// With the exact filter mode the two sums are computed directly, O(N^2) per
// label (the definition that the divide and conquer reproduces).
//
// Projected subgradient descent (Alg. lp_subgrad): y <- Pi(y - beta_t g),
// beta_t = beta0 / (1 + t), Pi the Euclidean projection of each pixel's row
// onto the simplex by the sort-based rule (one thread per pixel, a bitonic
// network in registers).

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "dcrf_internal.h"
#include "hash_scan.h"
#include "kernels_common.h"

namespace dcrf {
namespace {

// ------------------------------------------------------------ radix sort

constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;

// key for an ascending sort that orders y descending; -0 counts as +0
__device__ __forceinline__ uint32_t desc_key(float v) {
    if (v == 0.0f) v = 0.0f;
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? u : (~u & 0x7fffffffu);
}
__device__ __forceinline__ uint64_t desc_key(double v) {
    if (v == 0.0) v = 0.0;
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u & 0x8000000000000000ull) ? u : (~u & 0x7fffffffffffffffull);
}

template <typename T, typename K>
__global__ void k_rs_init(int N, int L, int col, const T *__restrict__ y,
                          K *__restrict__ keys, int *__restrict__ vals) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    keys[a] = desc_key(y[(size_t)a * L + col]);
    vals[a] = a;
}

// digit histogram of each tile, digit-major: hist[d * ntiles + tile]
template <typename K>
__global__ void __launch_bounds__(kRsThreads)
k_rs_hist(const K *__restrict__ keys, int n, int shift, int ntiles,
          int *__restrict__ hist) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const long long base = (long long)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        const long long i = base + (long long)r * kRsThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[int((keys[i] >> shift) & 0xffu)], 1);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// stable scatter: elements keep their order within each digit. Each round of
// kRsThreads elements is ranked per wave with ballots (lanes with the same
// digit), then across the block's waves with LDS counts.
template <typename K>
__global__ void __launch_bounds__(kRsThreads)
k_rs_scatter(const K *__restrict__ keys, const int *__restrict__ vals, int n,
             int shift, int ntiles, const int *__restrict__ offs,
             K *__restrict__ keys_out, int *__restrict__ vals_out) {
    constexpr int kWaves = kRsThreads / 64;
    __shared__ int wcount[kWaves][256];
    __shared__ int running[256];
    const int t = threadIdx.x;
    const int wave = t >> 6;
    const int lane = t & 63;
    running[t] = offs[(size_t)t * ntiles + blockIdx.x];
    const long long base = (long long)blockIdx.x * kRsTile;
    for (int r = 0; r < kRsItems; ++r) {
        for (int w = 0; w < kWaves; ++w) wcount[w][t] = 0;
        __syncthreads();
        const long long i = base + (long long)r * kRsThreads + t;
        const bool valid = i < n;
        K key = valid ? keys[i] : K(0);
        const int dg = int((key >> shift) & 0xffu);
        unsigned long long m = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dg >> b) & 1;
            const unsigned long long bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const int rank = __popcll(m & ((1ull << lane) - 1ull));
        if (valid && lane == __ffsll((long long)m) - 1) wcount[wave][dg] = __popcll(m);
        __syncthreads();
        if (valid) {
            int pos = running[dg] + rank;
            for (int w = 0; w < wave; ++w) pos += wcount[w][dg];
            keys_out[pos] = key;
            vals_out[pos] = vals[i];
        }
        __syncthreads();
        int tot = 0;
        for (int w = 0; w < kWaves; ++w) tot += wcount[w][t];
        running[t] += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------- divide and conquer

// floor(a / b) for a >= 0, b > 0: below 2^52 the double quotient is within
// one of the answer and one integer step corrects it (no 64-bit divide loop)
__device__ __forceinline__ long long floor_div(long long a, long long b) {
    if (a < (1ll << 52)) {
        long long q = (long long)((double)a / (double)b);
        const long long r = a - q * b;
        if (r < 0)
            --q;
        else if (r >= b)
            ++q;
        return q;
    }
    return a / b;
}

// node of sorted position p at level l and whether both of its halves are
// non-empty; side 0 = left half, 1 = right half
__device__ __forceinline__ bool dnc_node(long long p, int l, long long N,
                                         long long &node, int &side) {
    node = floor_div(((p + 1) << l) - 1, N);
    const long long lo = (node * N) >> l;
    const long long hi = ((node + 1) * N) >> l;
    const long long mid = ((2 * node + 1) * N) >> (l + 1);
    side = p < mid ? 0 : 1;
    return lo < mid && mid < hi;
}

// Hash region of a node: slots [2 lo D1, 2 hi D1) of the level's table, twice
// the node's (position, vertex) entries, so linear probing inside it always
// ends. Consecutive positions share a node, so a wave's probes, lookups and
// claims stay inside one small region instead of spreading over the table.
__device__ __forceinline__ void node_region(long long node, int l, long long N,
                                            int D1, long long &base,
                                            long long &size) {
    const long long lo = (node * N) >> l;
    const long long hi = ((node + 1) * N) >> l;
    base = 2 * lo * D1;
    size = 2 * (hi - lo) * D1;
}

// Level tags of the sub-lattice hash: a stored key carries the level's tag
// ep (1..kMaxTag) in its top 16 bits, so a slot whose tag differs (an older
// level's key, or a zero of a fresh table) counts as empty and no level
// clears the table. ep = 0 marks the untagged form (node keys of 48 bits or
// more): keys are stored as they are and the table is cleared to kEmpty
// before each level.
constexpr int kTagShift = 48;
constexpr unsigned kMaxTag = 0xfffe;

__device__ __forceinline__ bool slot_taken(uint64_t slot, unsigned ep) {
    return ep ? unsigned(slot >> kTagShift) == ep : slot != kEmpty;
}

// first probe of global vertex v in a region of `size` (< 2^32) slots
__device__ __forceinline__ long long region_slot(int v, long long size) {
    return (long long)(((mix64((uint64_t)v) >> 32) * (uint64_t)size) >> 32);
}

// insert the (node, vertex) keys of every entry e = (position p, vertex k)
// into the node's region. A new sub-vertex takes the number of the entry that
// claims its slot: unique, below N D1, and found without a shared counter
// (a single counter taken by every wave serialises across the chip). Entry e
// writes sub_nv[e] = (node, vertex) if it claimed a slot, else (-1, -1), so
// the sub-vertex numbers of a level are the e with sub_nv[e].y >= 0.
__global__ void k_lp_insert(int N, int l, int D1, int M, unsigned ep,
                            const int *__restrict__ pos_vid,
                            uint64_t *__restrict__ hkeys,
                            int *__restrict__ ent_slot, int *__restrict__ flags,
                            int *__restrict__ slot_vid,
                            int2 *__restrict__ sub_nv, int *__restrict__ nbr_sub,
                            int ld_nb) {
    const int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;   // N D1 < 2^31
    const bool in = e < N * D1;
    int slot = -1;
    bool claimed = false;
    uint64_t key = 0;
    int2 nv = make_int2(-1, -1);
    if (in) {
        const int p = e / D1;
        long long node;
        int side;
        if (dnc_node(p, l, N, node, side)) {
            const int v = pos_vid[e];
            if (v >= 0) {
                key = (uint64_t)node * (uint64_t)M + (uint64_t)v;
                if (ep) key |= (uint64_t)ep << kTagShift;
                nv = make_int2(int(node), v);
                long long base, size;
                node_region(node, l, N, D1, base, size);
                long long h = region_slot(v, size);
                long long probe = 0;
                for (; probe < size; ++probe) {
                    // during a level a slot changes once, from free to a key
                    // of the level: a plain load that sees such a key is
                    // final, and only a free slot needs the compare-and-swap
                    // (which fails, returning the key, if another entry took
                    // it first)
                    unsigned long long prev = hkeys[base + h];
                    if (!slot_taken(prev, ep)) {
                        const unsigned long long got =
                            atomicCAS((unsigned long long *)&hkeys[base + h], prev,
                                      (unsigned long long)key);
                        if (got == prev) {
                            claimed = true;
                            break;
                        }
                        prev = got;
                    }
                    if (prev == key) break;
                    if (++h == size) h = 0;
                }
                if (probe == size)
                    atomicOr(flags, 2);
                else
                    slot = int(base + h);
            }
        }
    }
    if (claimed) slot_vid[slot] = e;
    if (in) {
        ent_slot[e] = slot;
        sub_nv[e] = claimed ? nv : make_int2(-1, -1);
        // minus links start absent; the neighbour pass sets those present
        for (int j = 0; j < D1; ++j) nbr_sub[(size_t)(2 * j + 1) * ld_nb + e] = -1;
    }
}

// splat the two half indicators: V0[id][side] += b; records the entry's
// sub-vertex id for the slice. Neighbouring positions share sub-vertices, so
// a block first sums its entries per (id, side) in an LDS table (twice the
// block's entries, so probing ends) and then adds each sum with one atomic.
constexpr int kLpSplatThreads = 256;
constexpr int kLpSplatSlots = 2 * kLpSplatThreads;

// Small nodes share few sub-vertices within a block, and there each entry
// adds directly (AGG = false).
constexpr int kLpAggPixels = 64;   // node size from which the LDS sums pay

template <typename T, bool AGG>
__global__ void __launch_bounds__(kLpSplatThreads)
k_lp_splat(int N, int l, int D1, const T *__restrict__ pos_w,
           const int *__restrict__ ent_slot,
           const int *__restrict__ slot_vid, int *__restrict__ ent_id,
           T *__restrict__ V0) {
    if (!AGG) {
        const int e = xcd_block(blockIdx.x, gridDim.x) * kLpSplatThreads + threadIdx.x;
        if (e >= N * D1) return;
        const int s = ent_slot[e];
        int id = -1;
        if (s >= 0) {
            const int p = e / D1;
            long long node;
            int side;
            dnc_node(p, l, N, node, side);
            id = slot_vid[s];
            atomic_add(&V0[(size_t)id * 2 + side], pos_w[e]);
        }
        ent_id[e] = id;
        return;
    }
    __shared__ int skey[kLpSplatSlots];
    __shared__ T sval[kLpSplatSlots];
    for (int i = threadIdx.x; i < kLpSplatSlots; i += kLpSplatThreads) {
        skey[i] = -1;
        sval[i] = T(0);
    }
    __syncthreads();
    const int e = xcd_block(blockIdx.x, gridDim.x) * kLpSplatThreads + threadIdx.x;   // N D1 < 2^31
    if (e < N * D1) {
        const int s = ent_slot[e];
        int id = -1;
        if (s >= 0) {
            const int p = e / D1;
            long long node;
            int side;
            dnc_node(p, l, N, node, side);
            id = slot_vid[s];
            const int key = id * 2 + side;   // < 2 N D1 < 2^31
            const T w = pos_w[e];
            int h = int(mix64((uint64_t)key) & (kLpSplatSlots - 1));
            for (int probe = 0; probe < kLpSplatSlots; ++probe) {
                const int prev = atomicCAS(&skey[h], -1, key);
                if (prev == -1 || prev == key) {
                    atomicAdd(&sval[h], w);
                    break;
                }
                h = (h + 1) & (kLpSplatSlots - 1);
            }
        }
        ent_id[e] = id;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kLpSplatSlots; i += kLpSplatThreads) {
        const int key = skey[i];
        if (key >= 0) atomic_add(&V0[key], sval[i]);
    }
}

// neighbours of every sub-vertex: (node, v +- u_j) when present in the node,
// looked up in the node's region. Numbers that are no sub-vertex this level
// get no neighbours, so the blur keeps them at zero.
//
// Only the d + 1 "plus" neighbours are looked up: (node, v + u_j) present
// means its minus neighbour along j is (node, v), so a hit also writes that
// reverse link (the insert pass set every minus link absent beforehand). The
// lookups of a sub-vertex are independent: global neighbours, first probes
// and sub-vertex numbers are each loaded for all directions before any is
// used, so the loads overlap.
constexpr int kLpMaxNb = 6;   // d + 1 for d <= 5

__global__ void __launch_bounds__(256)
k_lp_neighbours(int S, int N, int l, int M, int D1, unsigned ep,
                const int2 *__restrict__ sub_nv, const int *__restrict__ nbr_global,
                const uint64_t *__restrict__ hkeys, const int *__restrict__ slot_vid,
                int *__restrict__ nbr_sub, int cap_sub) {
    const int id = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id >= S) return;
    const int2 nv = sub_nv[id];
    const int nq = D1;
    if (nv.y < 0) {
        for (int q = 0; q < nq; ++q) nbr_sub[(size_t)(2 * q) * cap_sub + id] = -1;
        return;
    }
    const long long node = nv.x;
    long long base, size;
    node_region(node, l, N, D1, base, size);
    int vn[kLpMaxNb];
#pragma unroll
    for (int q = 0; q < kLpMaxNb; ++q)
        vn[q] = q < nq ? nbr_global[((size_t)q * M + nv.y) * 2] : -1;
    long long h[kLpMaxNb];
    uint64_t kk[kLpMaxNb];
#pragma unroll
    for (int q = 0; q < kLpMaxNb; ++q) {
        h[q] = vn[q] >= 0 ? region_slot(vn[q], size) : 0;
        kk[q] = vn[q] >= 0 ? hkeys[base + h[q]] : kEmpty;
    }
    const uint64_t tag = ep ? (uint64_t)ep << kTagShift : 0;
#pragma unroll
    for (int q = 0; q < kLpMaxNb; ++q) {
        if (vn[q] < 0) continue;
        const uint64_t nk = ((uint64_t)node * (uint64_t)M + (uint64_t)vn[q]) | tag;
        // a present key is rarely displaced: continue the probe only then
        for (long long probe = 1; kk[q] != nk && slot_taken(kk[q], ep) && probe < size;
             ++probe) {
            if (++h[q] == size) h[q] = 0;
            kk[q] = hkeys[base + h[q]];
        }
    }
    int nid[kLpMaxNb];
#pragma unroll
    for (int q = 0; q < kLpMaxNb; ++q) {
        const bool hit = vn[q] >= 0 &&
                         kk[q] == (((uint64_t)node * (uint64_t)M + (uint64_t)vn[q]) | tag);
        nid[q] = hit ? slot_vid[base + h[q]] : -1;
    }
#pragma unroll
    for (int q = 0; q < kLpMaxNb; ++q) {
        if (q >= nq) continue;
        nbr_sub[(size_t)(2 * q) * cap_sub + id] = nid[q];
        if (nid[q] >= 0) nbr_sub[(size_t)(2 * q + 1) * cap_sub + nid[q]] = id;
    }
}

// Dense numbering for the first levels, where a level's nodes times the
// lattice's vertices fit the dense capacity (2^l M <= lp_dense_cap): the
// sub-vertex (node n, global vertex v) is number n M + v, so no hash is
// built. mark[n M + v] = the level's mark when some entry of node n has
// vertex v; the other numbers are no sub-vertex, hold zeros and have no
// neighbours. Neighbours come straight from the global table: (n, v +- u_j)
// is (n, nbr_j(v)) when that number is marked.
template <typename T, bool AGG>
__global__ void __launch_bounds__(kLpSplatThreads)
k_lp_dense_splat(int N, int l, int D1, int M, int mk, const int *__restrict__ pos_vid,
                 const T *__restrict__ pos_w, int *__restrict__ mark,
                 int *__restrict__ ent_id, T *__restrict__ V0) {
    __shared__ int skey[AGG ? kLpSplatSlots : 1];
    __shared__ T sval[AGG ? kLpSplatSlots : 1];
    if (AGG) {
        for (int i = threadIdx.x; i < kLpSplatSlots; i += kLpSplatThreads) {
            skey[i] = -1;
            sval[i] = T(0);
        }
        __syncthreads();
    }
    const int e = xcd_block(blockIdx.x, gridDim.x) * kLpSplatThreads + threadIdx.x;
    if (e < N * D1) {
        int id = -1;
        const int p = e / D1;
        long long node;
        int side;
        const int v = pos_vid[e];
        if (dnc_node(p, l, N, node, side) && v >= 0) {
            id = int(node) * M + v;   // < 2^l M <= N D1 < 2^31
            mark[id] = mk;
            const int key = id * 2 + side;
            const T w = pos_w[e];
            if (AGG) {
                int h = int(mix64((uint64_t)key) & (kLpSplatSlots - 1));
                for (int probe = 0; probe < kLpSplatSlots; ++probe) {
                    const int prev = atomicCAS(&skey[h], -1, key);
                    if (prev == -1 || prev == key) {
                        atomicAdd(&sval[h], w);
                        break;
                    }
                    h = (h + 1) & (kLpSplatSlots - 1);
                }
            } else {
                atomic_add(&V0[key], w);
            }
        }
        ent_id[e] = id;
    }
    if (AGG) {
        __syncthreads();
        for (int i = threadIdx.x; i < kLpSplatSlots; i += kLpSplatThreads) {
            const int key = skey[i];
            if (key >= 0) atomic_add(&V0[key], sval[i]);
        }
    }
}

// The same splat gathered by vertex (the lattice's inverse index): wave w of
// a block takes global vertex v, adds the weights of v's entries into LDS
// bins (node, side) of the level, and stores each non-zero bin at its dense
// number with a plain store (one wave owns every number n M + v), marking
// it. Levels with more than kLpVertexBins / 2 nodes use k_lp_dense_splat.
constexpr int kLpVertexBins = 512;

__device__ __forceinline__ int dnc_node_side(int p, int l, int N) {
    long long node;
    int side;
    return dnc_node(p, l, N, node, side) ? int(node) * 2 + side : -1;
}

template <typename T>
__global__ void __launch_bounds__(256)
k_lp_vertex_splat(int N, int l, int M, int mk, const int *__restrict__ csr_off,
                  const int *__restrict__ ent_pix, const T *__restrict__ ent_w,
                  const int *__restrict__ rank, int *__restrict__ mark,
                  T *__restrict__ V0) {
    __shared__ T bins[4][kLpVertexBins];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int v = xcd_block(blockIdx.x, gridDim.x) * 4 + wv;
    const int nb = 2 << l;   // bins of the level: 2^l nodes, two sides
    T *b = bins[wv];
    for (int i = lane; i < nb; i += 64) b[i] = T(0);
    __syncthreads();
    if (v < M) {
        const int e1 = csr_off[v + 1];
        for (int j = csr_off[v] + lane; j < e1; j += 64) {
            const int ns = dnc_node_side(rank[ent_pix[j]], l, N);
            if (ns >= 0) atomicAdd(&b[ns], ent_w[j]);
        }
    }
    __syncthreads();
    if (v < M)
        for (int i = lane; i < nb; i += 64) {
            const T x = b[i];
            if (x != T(0)) {
                const int id = (i >> 1) * M + v;
                V0[(size_t)id * 2 + (i & 1)] = x;
                mark[id] = mk;
            }
        }
}

// Node-local levels, where whole nodes fit a block: block b takes nodes
// [b k, b k + k), whose entries are one contiguous range of at most CAP
// (2048, or 4096 where a node needs more), and sorts their keys (node, vertex) in LDS (bitonic). Each run
// of equal keys is one sub-vertex, numbered by the entry number of its first
// element in sorted order; that element's thread sums the run's weights per
// side (a plain store: the block owns its numbers), and finds the plus and
// minus neighbours (node, nbr_j(v)) by binary search in the sorted keys.
// Every number of the block that is no sub-vertex gets no links. One launch
// replaces the hash insert, the splat and the neighbour lookups.
constexpr int kLpNodeCap = 4096;   // the larger block; 2048 where nodes fit it

__device__ __forceinline__ int lds_lower_bound(const unsigned long long *a, int n,
                                               unsigned long long x) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <typename T, int CAP>
__global__ void __launch_bounds__(CAP / 4)
k_lp_node_level(int N, int l, int D1, int M, int k, const int *__restrict__ pos_vid,
                const T *__restrict__ pos_w, const int *__restrict__ nbr_global,
                int *__restrict__ ent_id, T *__restrict__ V0, int *__restrict__ nbr_sub,
                int ld_nb) {
    constexpr int kLpNodeThreads = CAP / 4;
    __shared__ unsigned long long skey[CAP];
    __shared__ int sidx[CAP];
    // weight and side of the block's entry i (by entry, not by sorted
    // position): the run sums read them from LDS
    __shared__ T sw[CAP];
    __shared__ unsigned char sside[CAP];
    // keys: valid (node, vertex) pairs < 2^43; an entry that is no term
    // (a node with an empty half, a missing vertex) kNone; the padding up to
    // a power of two kPad, so that the block's ne entries fill the sorted
    // positions [0, ne) and every number written stays in the block's range
    constexpr unsigned long long kPad = ~0ull, kNone = kPad - 1;
    const long long n0 = (long long)blockIdx.x * k;
    const long long n1 = min(n0 + k, 1ll << l);
    const int lo = int((n0 * N) >> l), hi = int((n1 * N) >> l);
    const int ne = (hi - lo) * D1;   // <= CAP (k is chosen so)
    int P2 = 1;
    while (P2 < ne) P2 <<= 1;
    const long long e0 = (long long)lo * D1;
    for (int i = threadIdx.x; i < P2; i += kLpNodeThreads) {
        unsigned long long key = i < ne ? kNone : kPad;
        if (i < ne) {
            const int p = lo + i / D1;
            long long node;
            int side;
            const int v = pos_vid[e0 + i];
            const T w = pos_w[e0 + i];
            if (dnc_node(p, l, N, node, side) && v >= 0)
                key = ((unsigned long long)(node - n0) << 32) | (unsigned)v;
            sw[i] = w;
            sside[i] = (unsigned char)side;
        }
        skey[i] = key;
        sidx[i] = i;
    }
    __syncthreads();
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = threadIdx.x; t < (P2 >> 1); t += kLpNodeThreads) {
                const int i = ((t & ~(stride - 1)) << 1) | (t & (stride - 1));
                const int j = i + stride;
                const bool up = (i & size) == 0;
                const unsigned long long a = skey[i], b = skey[j];
                if ((a > b) == up && a != b) {
                    skey[i] = b;
                    skey[j] = a;
                    const int x = sidx[i];
                    sidx[i] = sidx[j];
                    sidx[j] = x;
                }
            }
            __syncthreads();
        }
    }
    const int nvalid = lds_lower_bound(skey, P2, kNone);
    for (int r = threadIdx.x; r < ne; r += kLpNodeThreads) {
        const unsigned long long key = skey[r];
        const long long e = e0 + sidx[r];
        const int r0 = r < nvalid ? lds_lower_bound(skey, nvalid, key) : -1;
        ent_id[e] = r0 >= 0 ? int(e0 + sidx[r0]) : -1;
        if (r0 != r) {   // no sub-vertex is numbered e
            for (int q = 0; q < 2 * D1; ++q) nbr_sub[(size_t)q * ld_nb + e] = -1;
            continue;
        }
        T s0 = T(0), s1 = T(0);
        for (int rr = r; rr < nvalid && skey[rr] == key; ++rr) {
            const int ii = sidx[rr];
            if (sside[ii])
                s1 += sw[ii];
            else
                s0 += sw[ii];
        }
        V0[e * 2] = s0;
        V0[e * 2 + 1] = s1;
        const int v = int(key & 0xffffffffull);
        const unsigned long long nb = key & ~0xffffffffull;
        for (int q = 0; q < 2 * D1; ++q) {
            const int vn = nbr_global[((size_t)(q >> 1) * M + v) * 2 + (q & 1)];
            int nid = -1;
            if (vn >= 0) {
                const unsigned long long kk = nb | (unsigned)vn;
                const int rn = lds_lower_bound(skey, nvalid, kk);
                if (rn < nvalid && skey[rn] == kk) nid = int(e0 + sidx[rn]);
            }
            nbr_sub[(size_t)q * ld_nb + e] = nid;
        }
    }
}

// rank[perm[p]] = p: the sorted position of every pixel
__global__ void k_lp_rank(int N, const int *__restrict__ perm, int *__restrict__ rank) {
    const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p < N) rank[perm[p]] = p;
}

__global__ void __launch_bounds__(256)
k_lp_dense_nbrs(int S, int M, int D1, int mk, const int *__restrict__ mark,
                const int *__restrict__ nbr_global, int *__restrict__ nbr_sub,
                int cap_sub) {
    const int id = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id >= S) return;
    const int n = id / M, v = id - n * M;
    const bool here = mark[id] == mk;
    int vn[2 * kLpMaxNb];
#pragma unroll
    for (int q = 0; q < 2 * kLpMaxNb; ++q)
        vn[q] = here && q < 2 * D1 ? nbr_global[((size_t)(q >> 1) * M + v) * 2 + (q & 1)] : -1;
    int ok[2 * kLpMaxNb];
#pragma unroll
    for (int q = 0; q < 2 * kLpMaxNb; ++q) ok[q] = vn[q] >= 0 ? mark[n * M + vn[q]] == mk : 0;
#pragma unroll
    for (int q = 0; q < 2 * kLpMaxNb; ++q)
        if (q < 2 * D1) nbr_sub[(size_t)q * cap_sub + id] = ok[q] ? n * M + vn[q] : -1;
}

// one blur pass over the sub-lattice (all S = N D1 numbers; those that are no
// sub-vertex hold zeros and have no neighbours): one thread per sub-vertex
// moves both channels as one 2-vector; the second pass clears V0
template <typename T>
struct alignas(2 * sizeof(T)) LpPair {
    T c0, c1;
};

// G = 1: pass j; G = 2: passes j then j + 1 in one launch. Per sub-vertex the
// second pass combines the first pass's values at the vertex and its two
// neighbours along j + 1, each computed as the single pass computes it, so
// the result is the same as two launches. `clr` (may be null) is set to zero.
template <typename T, int G>
__global__ void k_lp_blur(int S, int j, int cap_sub, const int *__restrict__ nbr_sub,
                          const LpPair<T> *__restrict__ src,
                          LpPair<T> *__restrict__ dst, LpPair<T> *__restrict__ clr) {
    const int id = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (id >= S) return;
    const LpPair<T> zero{T(0), T(0)};
    auto pass = [&](int y) {
        const int np = nbr_sub[(size_t)(2 * j) * cap_sub + y];
        const int nm = nbr_sub[(size_t)(2 * j + 1) * cap_sub + y];
        const LpPair<T> x = src[y];
        const LpPair<T> vp = np >= 0 ? src[np] : zero;
        const LpPair<T> vm = nm >= 0 ? src[nm] : zero;
        return LpPair<T>{T(0.5) * x.c0 + T(0.25) * (vp.c0 + vm.c0),
                         T(0.5) * x.c1 + T(0.25) * (vp.c1 + vm.c1)};
    };
    LpPair<T> out;
    if (G == 1) {
        out = pass(id);
    } else {
        const int np = nbr_sub[(size_t)(2 * j + 2) * cap_sub + id];
        const int nm = nbr_sub[(size_t)(2 * j + 3) * cap_sub + id];
        const LpPair<T> x = pass(id);
        const LpPair<T> vp = np >= 0 ? pass(np) : zero;
        const LpPair<T> vm = nm >= 0 ? pass(nm) : zero;
        out = LpPair<T>{T(0.5) * x.c0 + T(0.25) * (vp.c0 + vm.c0),
                        T(0.5) * x.c1 + T(0.25) * (vp.c1 + vm.c1)};
    }
    dst[id] = out;
    if (clr) clr[id] = zero;
}

// blur launches of a sub-lattice with D1 directions: two directions per
// launch; the first launch reads V0, later ones alternate V1 -> V2 -> V1, and
// the second clears V0 for the next level (D1 >= 3, so there is a second)
inline int lp_blur_launches(int D1) { return (D1 + 1) / 2; }

template <typename T>
struct LPLat {
    const T *pos_w;
    const int *ent_id;   // the entries' sub-vertex numbers (hashed levels)
    const T *Vf;
    int D1;
    T wg;
    const int *pos_vid;  // dense levels: entry (p, k) is number node M + pos_vid
    int M, dense;
};

template <typename T>
struct LPLats {
    LPLat<T> l[DCRF_MAXK];
    int nk;
};

// slice: the right channel at left points adds to U, the left channel at
// right points adds to Lo; acc[p] += U - Lo for sorted position p (added to
// g once the label's levels are done)
template <typename T>
__global__ void k_lp_slice(int N, int l, LPLats<T> lats, T *__restrict__ acc) {
    const int p = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (p >= N) return;
    long long node;
    int side;
    if (!dnc_node(p, l, N, node, side)) return;
    const int ch = 1 - side;
    T t = T(0);
    for (int m = 0; m < lats.nk; ++m) {
        const LPLat<T> &X = lats.l[m];
        T s = T(0);
        for (int k = 0; k < X.D1; ++k) {
            int id;
            if (X.dense) {
                const int v = X.pos_vid[(size_t)p * X.D1 + k];
                id = v >= 0 ? int(node) * X.M + v : -1;
            } else {
                id = X.ent_id[(size_t)p * X.D1 + k];
            }
            if (id >= 0)
                s += X.pos_w[(size_t)p * X.D1 + k] * X.Vf[(size_t)id * 2 + ch];
        }
        t += X.wg * s;
    }
    acc[p] += side == 0 ? t : -t;
}

// the label's vertex ids and weights in sorted-position order, gathered once
// for all its levels: pos_vid[p D1 + k] = vid[perm[p] D1 + k]
template <typename T>
__global__ void k_lp_gather(int N, int D1, const int *__restrict__ perm,
                            const int *__restrict__ pix_vid,
                            const T *__restrict__ pix_w, int *__restrict__ pos_vid,
                            T *__restrict__ pos_w) {
    const int e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;   // N D1 < 2^31
    if (e >= N * D1) return;
    const int p = e / D1;
    const size_t src = (size_t)perm[p] * D1 + (e - p * D1);
    pos_vid[e] = pix_vid[src];
    pos_w[e] = pix_w[src];
}

// g[perm[p]][col] += acc[p], and acc returns to zero for the next label
template <typename T>
__global__ void k_lp_add_col(int N, int L, int col, const int *__restrict__ perm,
                             T *__restrict__ acc, T *__restrict__ g) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    g[(size_t)perm[p] * L + col] += acc[p];
    acc[p] = T(0);
}

// leaf-exact divide and conquer: node n of level lcut holds the sorted
// positions [n N >> lcut, (n+1) N >> lcut), at most kLpLeafMax of them; the
// pixel at position p receives sum over the node's other positions q of
// Kbar(pi(q), pi(p)) (q > p ? 1 : -1), the exact Gaussian sum, with the
// node's features staged in LDS (one block per node, one lane per position)
constexpr int kLpLeafMax = 256;
constexpr int kLpLeafMaxF = 16;   // feature dimensions over all kernels

// The features of the node's positions sit in LDS (every lane of a wave
// reads the same position's row: a broadcast); each lane keeps its own in
// registers. FA, FB: the feature dimensions of the first two kernels, fixed
// at compile time for the usual layouts (0, 0: any layout, read at run time).
template <typename T, int FA, int FB>
__global__ void __launch_bounds__(kLpLeafMax)
k_lp_leaf(int N, int lcut, const int *__restrict__ perm, ExactSet<T> ex,
          T *__restrict__ acc) {
    constexpr bool fixed = FA > 0;
    constexpr int FS = fixed ? FA + FB : kLpLeafMaxF;   // LDS row stride
    __shared__ T sf[kLpLeafMax * FS];
    const long long n = blockIdx.x;
    const int lo = int((n * N) >> lcut), hi = int(((n + 1) * N) >> lcut);
    const int p = lo + (int)threadIdx.x;
    const int F = fixed ? FA + FB : ex.off[ex.nk];
    T fa[FS];
#pragma unroll
    for (int j = 0; j < FS; ++j) fa[j] = T(0);
    if (p < hi) {
        const int a = perm[p];
        for (int m = 0; m < ex.nk; ++m)
            for (int j = 0; j < ex.d[m]; ++j)
                sf[threadIdx.x * FS + ex.off[m] + j] = ex.f[m][(size_t)a * ex.d[m] + j];
    }
    __syncthreads();
    if (p >= hi) return;
    const int me = (int)threadIdx.x;
#pragma unroll
    for (int j = 0; j < FS; ++j)
        if (j < F) fa[j] = sf[me * FS + j];
    T s = T(0);
    for (int t = 0; t < hi - lo; ++t) {
        if (t == me) continue;
        const T *ft = sf + t * FS;
        T kab;
        if constexpr (fixed) {
            T ra = T(0), rb = T(0);
#pragma unroll
            for (int j = 0; j < FA; ++j) {
                const T df = fa[j] - ft[j];
                ra += df * df;
            }
#pragma unroll
            for (int j = FA; j < FA + FB; ++j) {
                const T df = fa[j] - ft[j];
                rb += df * df;
            }
            kab = ex.w[0] * exp(T(-0.5) * ra);
            if (FB > 0) kab += ex.w[1] * exp(T(-0.5) * rb);
        } else {
            kab = T(0);
            for (int m = 0; m < ex.nk; ++m) {
                T r2 = T(0);
#pragma unroll
                for (int j = 0; j < FS; ++j) {
                    if (j < ex.off[m] || j >= ex.off[m + 1]) continue;
                    const T df = fa[j] - ft[j];
                    r2 += df * df;
                }
                kab += ex.w[m] * exp(T(-0.5) * r2);
            }
        }
        s += t > me ? kab : -kab;
    }
    acc[p] += s;
}

// y_a(T) = sum of y_a(i) over the subtree's labels, in increasing label order
template <typename T>
__global__ void k_tree_col(int N, int L, const T *__restrict__ y,
                           const int *__restrict__ labs, int nlab, T *__restrict__ col) {
    const int a = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const T *row = y + (size_t)a * L;
    T s = T(0);
    for (int j = 0; j < nlab; ++j) s += row[labs[j]];
    col[a] = s;
}

// g[perm[p]][k] += c acc[p] for every label k of the subtree; acc returns
// to zero
template <typename T>
__global__ void k_lp_add_tree(int N, int L, const int *__restrict__ perm,
                              T *__restrict__ acc, T c, const int *__restrict__ labs,
                              int nlab, T *__restrict__ g) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const T v = c * acc[p];
    T *row = g + (size_t)perm[p] * L;
    for (int j = 0; j < nlab; ++j) row[labs[j]] += v;
    acc[p] = T(0);
}

// exact mode: for the point at sorted position p,
// acc[p] = sum_{q != p} Kbar(pi(q), pi(p)) (q > p ? 1 : -1), tiled through LDS
constexpr int kLpExTile = 128;

template <typename T>
__global__ void __launch_bounds__(kLpExTile)
k_lp_exact(int N, const int *__restrict__ perm, ExactSet<T> ex, T *__restrict__ acc_out) {
    __shared__ T sf[kLpExTile][16];
    const int p = blockIdx.x * kLpExTile + threadIdx.x;
    T fa[16];
    for (int j = 0; j < 16; ++j) fa[j] = T(0);
    int a = 0;
    if (p < N) {
        a = perm[p];
        for (int m = 0; m < ex.nk; ++m)
            for (int j = 0; j < ex.d[m]; ++j)
                fa[ex.off[m] + j] = ex.f[m][(size_t)a * ex.d[m] + j];
    }
    T acc = T(0);
    for (int q0 = 0; q0 < N; q0 += kLpExTile) {
        const int q = q0 + threadIdx.x;
        if (q < N) {
            const int b = perm[q];
            for (int m = 0; m < ex.nk; ++m)
                for (int j = 0; j < ex.d[m]; ++j)
                    sf[threadIdx.x][ex.off[m] + j] = ex.f[m][(size_t)b * ex.d[m] + j];
        }
        __syncthreads();
        const int nb = min(kLpExTile, N - q0);
        for (int t = 0; t < nb; ++t) {
            const int q2 = q0 + t;
            if (q2 == p) continue;
            T kab = T(0);
            for (int m = 0; m < ex.nk; ++m) {
                T r2 = T(0);
                for (int j = ex.off[m]; j < ex.off[m + 1]; ++j) {
                    const T df = fa[j] - sf[t][j];
                    r2 += df * df;
                }
                kab += ex.w[m] * exp(T(-0.5) * r2);
            }
            acc += q2 > p ? kab : -kab;
        }
        __syncthreads();
    }
    if (p < N) acc_out[p] = acc;
}

// ------------------------------------------------- projection and step


// y <- Pi(y - beta g) (beta = 0: plain projection of y), one thread per pixel
template <typename T, int LMAX>
__global__ void k_lp_step_rows(int N, int L, const T *src, const T *g, T beta,
                               T *dst) {
    constexpr int P = Pow2<LMAX>::v;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    T v[P];
#pragma unroll
    for (int j = 0; j < P; ++j)
        v[j] = (j < L) ? src[(size_t)a * L + j] - (g ? beta * g[(size_t)a * L + j] : T(0))
                       : T(0);
    const T tau = simplex_tau<T, P>(v, L);
#pragma unroll
    for (int j = 0; j < P; ++j)
        if (j < L) dst[(size_t)a * L + j] = fmax(v[j] - tau, T(0));
}

// the same for any L: the sort-free form tau = (S_i - 1) / n_i for the
// largest set {k : v_k >= v_i} whose smallest member stays positive
template <typename T>
__global__ void k_lp_step_flat(int N, int L, const T *src, const T *g, T beta,
                               T *dst) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= N) return;
    const T *s = src + (size_t)a * L;
    const T *gg = g ? g + (size_t)a * L : nullptr;
    int best_n = 0;
    T tau = T(0);
    for (int i = 0; i < L; ++i) {
        const T vi = s[i] - (gg ? beta * gg[i] : T(0));
        T S = T(0);
        int n = 0;
        for (int k = 0; k < L; ++k) {
            const T vk = s[k] - (gg ? beta * gg[k] : T(0));
            if (vk >= vi) {
                S += vk;
                ++n;
            }
        }
        const T t = (S - T(1)) / T(n);
        if (vi - t > T(0) && n > best_n) {
            best_n = n;
            tau = t;
        }
    }
    for (int j = 0; j < L; ++j) {
        const T vj = s[j] - (gg ? beta * gg[j] : T(0));
        dst[(size_t)a * L + j] = fmax(vj - tau, T(0));
    }
}

template <typename T>
__global__ void k_copy(size_t n, const T *__restrict__ s, T *__restrict__ d) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// per-block partial sums of <g, y>
template <typename T>
__global__ void __launch_bounds__(256)
k_dot(size_t n, const T *__restrict__ a, const T *__restrict__ b,
      double *__restrict__ part) {
    __shared__ double red[256];
    double acc[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n;
         i += (size_t)gridDim.x * 256)
        acc[0] += double(a[i]) * double(b[i]);
    block_sum<1, 256>(acc, red);
    if (threadIdx.x == 0) part[blockIdx.x] = acc[0];
}

// ------------------------------------------------------------------ host

struct LPWork {
    DevBuf keys, keys2, vals, vals2, hist;
    struct PerLat {
        DevBuf hkeys, slot_vid, ent_slot, ent_id, sub_nv, nbr_sub, V[3], mark;
        DevBuf pos_vid, pos_w;   // the label's vertex ids and weights by position
        size_t cap = 0;
        int cap_sub = 0;           // sub-vertex numbers of a hashed level: N (d + 1)
        int cap_dense = 0;         // numbers available to a dense level
        int ld_nb = 0;             // row stride of nbr_sub and of the V buffers' numbers
        unsigned tag = 0;          // the last level's tag in hkeys (0: none yet)
        int mk = 0;                // the last dense level's mark (0: none yet)
        const void *mk_buf = nullptr;    // the mark allocation mk refers to
        const void *tag_buf = nullptr;   // the hkeys allocation the tag refers to
    } lat[DCRF_MAXK];
    DevBuf g, part, acc;
    DevBuf rank;             // the sorted position of every pixel (dense levels)
    DevBuf col, tree_lab;    // a subtree's column y(T) and the subtrees' label lists
    // the second and later lattices of a level run on a stream of their own
    // (default priority), joined to the context's stream by two events
    hipStream_t side = nullptr;
    hipEvent_t ev_start = nullptr, ev_done = nullptr;
};

// level l of lattice m (M vertices) numbers its sub-vertices densely
inline bool lp_dense_level(const LPWork::PerLat &P, int M, int l) {
    return l < 31 && ((long long)M << l) <= (long long)P.cap_dense;
}

LPWork &lp_work(dcrf_ctx *ctx) {
    if (!ctx->lp) ctx->lp = new LPWork();
    return *static_cast<LPWork *>(ctx->lp);
}

template <typename T>
void sort_column(dcrf_ctx *ctx, LPWork &W, const T *y, int L, int col,
                 int **perm_out) {
    using K = typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type;
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    const int ntiles = ceil_div(N, kRsTile);
    W.keys.ensure((size_t)N * sizeof(K), s);
    W.keys2.ensure((size_t)N * sizeof(K), s);
    W.vals.ensure((size_t)N * 4, s);
    W.vals2.ensure((size_t)N * 4, s);
    W.hist.ensure((size_t)(256 * ntiles + 1) * 4 * 2, s);
    K *k0 = W.keys.as<K>(), *k1 = W.keys2.as<K>();
    int *v0 = W.vals.as<int>(), *v1 = W.vals2.as<int>();
    int *hist = W.hist.as<int>();
    int *offs = hist + 256 * ntiles + 1;
    hipLaunchKernelGGL((k_rs_init<T, K>), dim3(ceil_div(N, 256)), dim3(256), 0, s,
                       N, L, col, y, k0, v0);
    for (int shift = 0; shift < int(8 * sizeof(K)); shift += 8) {
        hipLaunchKernelGGL((k_rs_hist<K>), dim3(ntiles), dim3(kRsThreads), 0, s,
                           k0, N, shift, ntiles, hist);
        scan_ints(ctx, hist, 256 * ntiles, offs);
        hipLaunchKernelGGL((k_rs_scatter<K>), dim3(ntiles), dim3(kRsThreads), 0,
                           s, k0, v0, N, shift, ntiles, offs, k1, v1);
        std::swap(k0, k1);
        std::swap(v0, v1);
    }
    DCRF_CHECK_LAUNCH();
    *perm_out = v0;   // an even number of passes leaves the result in vals
}

// the blur launches of a level over sub-vertex numbers [0, S)
template <typename T>
void lp_blur(LPWork::PerLat &P, int D1, int S, hipStream_t s) {
    LpPair<T> *V0 = P.V[0].as<LpPair<T>>(), *V1 = P.V[1].as<LpPair<T>>(),
              *V2 = P.V[2].as<LpPair<T>>();
    const int nl = lp_blur_launches(D1);
    for (int t = 0; t < nl; ++t) {
        const LpPair<T> *src = t == 0 ? V0 : ((t & 1) ? V1 : V2);
        LpPair<T> *dst = (t & 1) ? V2 : V1;
        LpPair<T> *clr = t == 1 ? V0 : nullptr;
        if (2 * t + 1 < D1)
            hipLaunchKernelGGL((k_lp_blur<T, 2>), dim3(ceil_div(S, 256)), dim3(256), 0, s,
                               S, 2 * t, P.ld_nb, P.nbr_sub.as<int>(), src, dst, clr);
        else
            hipLaunchKernelGGL((k_lp_blur<T, 1>), dim3(ceil_div(S, 256)), dim3(256), 0, s,
                               S, 2 * t, P.ld_nb, P.nbr_sub.as<int>(), src, dst, clr);
    }
}

template <typename T>
void lp_level(dcrf_ctx *ctx, LPWork &W, int m, int l, hipStream_t s) {
    Lattice &Lt = ctx->lat[m];
    auto &P = W.lat[m];
    const int N = ctx->N, D1 = Lt.d + 1, M = Lt.M;
    const long long E = (long long)N * D1;
    if (lp_dense_level(P, M, l)) {
        // dense numbering: every level's numbers are [0, 2^l M), all of them
        // cleared by the previous level's blur (V0) or rewritten here
        const int S = int((long long)M << l);
        if (P.mk_buf != P.mark.p) {   // a new allocation: zeroed by ensure()
            P.mk = 0;
            P.mk_buf = P.mark.p;
        }
        if (P.mk == INT32_MAX) {
            DCRF_TRY_HIP(hipMemsetAsync(P.mark.p, 0, (size_t)P.cap_dense * 4, s));
            P.mk = 0;
        }
        const int mk = ++P.mk;
        if ((2 << l) <= kLpVertexBins)
            hipLaunchKernelGGL((k_lp_vertex_splat<T>), dim3(ceil_div(M, 4)), dim3(256), 0, s,
                               N, l, M, mk, Lt.csr_off.as<int>(), Lt.ent_pix.as<int>(),
                               Lt.ent_w.as<T>(), W.rank.as<int>(), P.mark.as<int>(),
                               P.V[0].as<T>());
        else if ((N >> l) >= kLpAggPixels)
            hipLaunchKernelGGL((k_lp_dense_splat<T, true>), dim3(ceil_div(E, kLpSplatThreads)),
                               dim3(kLpSplatThreads), 0, s, N, l, D1, M, mk,
                               P.pos_vid.as<int>(), P.pos_w.as<T>(), P.mark.as<int>(),
                               P.ent_id.as<int>(), P.V[0].as<T>());
        else
            hipLaunchKernelGGL((k_lp_dense_splat<T, false>), dim3(ceil_div(E, kLpSplatThreads)),
                               dim3(kLpSplatThreads), 0, s, N, l, D1, M, mk,
                               P.pos_vid.as<int>(), P.pos_w.as<T>(), P.mark.as<int>(),
                               P.ent_id.as<int>(), P.V[0].as<T>());
        hipLaunchKernelGGL(k_lp_dense_nbrs, dim3(ceil_div(S, 256)), dim3(256), 0, s, S, M,
                           D1, mk, P.mark.as<int>(), Lt.nbr.as<int>(), P.nbr_sub.as<int>(),
                           P.ld_nb);
        lp_blur<T>(P, D1, S, s);
        DCRF_CHECK_LAUNCH();
        return;
    }
    const long long smax = ((long long)N + (1ll << l) - 1) >> l;   // the largest node
    if (l < 31 && smax * D1 <= kLpNodeCap) {
        const int cap = smax * D1 <= 2048 ? 2048 : 4096;
        const int k = int(std::max(1ll, cap / (smax * D1)));
        const long long nodes = 1ll << l;
        const dim3 grid(unsigned((nodes + k - 1) / k)), block(cap / 4);
        if (cap == 2048)
            hipLaunchKernelGGL((k_lp_node_level<T, 2048>), grid, block, 0, s, N, l, D1, M, k,
                               P.pos_vid.as<int>(), P.pos_w.as<T>(), Lt.nbr.as<int>(),
                               P.ent_id.as<int>(), P.V[0].as<T>(), P.nbr_sub.as<int>(),
                               P.ld_nb);
        else
            hipLaunchKernelGGL((k_lp_node_level<T, 4096>), grid, block, 0, s, N, l, D1, M, k,
                               P.pos_vid.as<int>(), P.pos_w.as<T>(), Lt.nbr.as<int>(),
                               P.ent_id.as<int>(), P.V[0].as<T>(), P.nbr_sub.as<int>(),
                               P.ld_nb);
        lp_blur<T>(P, D1, P.cap_sub, s);
        DCRF_CHECK_LAUNCH();
        return;
    }
    int *flags = ctx->scratch.as<int>();
    // a fresh tag per level (the table starts zeroed: tag 0 is free); after
    // the last tag the table is cleared once and the tags start again. Node
    // keys of 48 bits or more go untagged, with a clear per level.
    unsigned ep = 0;
    if ((long double)N * (long double)M < (long double)(1ull << kTagShift)) {
        if (P.tag_buf != P.hkeys.p) {   // a new allocation: zeroed by ensure()
            P.tag = 0;
            P.tag_buf = P.hkeys.p;
        }
        if (P.tag >= kMaxTag) {
            DCRF_TRY_HIP(hipMemsetAsync(P.hkeys.p, 0, P.cap * 8, s));
            P.tag = 0;
        }
        ep = ++P.tag;
    } else {
        DCRF_TRY_HIP(hipMemsetAsync(P.hkeys.p, 0xff, P.cap * 8, s));
        P.tag_buf = nullptr;
    }
    hipLaunchKernelGGL(k_lp_insert, dim3(ceil_div(E, 256)), dim3(256), 0, s, N, l,
                       D1, M, ep, P.pos_vid.as<int>(), P.hkeys.as<uint64_t>(),
                       P.ent_slot.as<int>(), flags, P.slot_vid.as<int>(),
                       P.sub_nv.as<int2>(), P.nbr_sub.as<int>(), P.ld_nb);
    if ((N >> l) >= kLpAggPixels)
        hipLaunchKernelGGL((k_lp_splat<T, true>), dim3(ceil_div(E, kLpSplatThreads)),
                           dim3(kLpSplatThreads), 0, s, N, l, D1,
                           P.pos_w.as<T>(), P.ent_slot.as<int>(),
                           P.slot_vid.as<int>(), P.ent_id.as<int>(), P.V[0].as<T>());
    else
        hipLaunchKernelGGL((k_lp_splat<T, false>), dim3(ceil_div(E, kLpSplatThreads)),
                           dim3(kLpSplatThreads), 0, s, N, l, D1,
                           P.pos_w.as<T>(), P.ent_slot.as<int>(),
                           P.slot_vid.as<int>(), P.ent_id.as<int>(), P.V[0].as<T>());
    hipLaunchKernelGGL(k_lp_neighbours, dim3(ceil_div(P.cap_sub, 256)), dim3(256),
                       0, s, P.cap_sub, N, l, M, D1, ep, P.sub_nv.as<int2>(),
                       Lt.nbr.as<int>(), P.hkeys.as<uint64_t>(), P.slot_vid.as<int>(),
                       P.nbr_sub.as<int>(), P.ld_nb);
    lp_blur<T>(P, D1, P.cap_sub, s);
    DCRF_CHECK_LAUNCH();
}

template <typename T>
void lp_prepare(dcrf_ctx *ctx, LPWork &W, int L) {
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    W.g.ensure((size_t)N * L * sizeof(T), s);
    W.part.ensure(1024 * 8, s);
    W.acc.ensure((size_t)N * sizeof(T), s);   // zero between columns
    W.rank.ensure((size_t)N * 4, s);
    if (ctx->mode == DCRF_FILTER_EXACT) return;
    if (!W.side) {
        DCRF_TRY_HIP(hipStreamCreateWithFlags(&W.side, hipStreamNonBlocking));
        DCRF_TRY_HIP(hipEventCreateWithFlags(&W.ev_start, hipEventDisableTiming));
        DCRF_TRY_HIP(hipEventCreateWithFlags(&W.ev_done, hipEventDisableTiming));
    }
    for (int m = 0; m < ctx->nk; ++m) {
        auto &P = W.lat[m];
        const int D1 = ctx->lat[m].d + 1;
        if (D1 > kLpMaxNb || D1 < 3)
            fail(DCRF_EUNSUPPORTED, "the LP takes lattices of dimension 2 to 5");
        const size_t E = (size_t)N * D1;
        // one region of twice its entries per node; slots are int32
        if (2 * E > (size_t)INT32_MAX)
            fail(DCRF_ERANGE, "image too large for the LP's sub-lattice tables");
        const size_t cap = 2 * E;
        P.cap = cap;
        P.cap_sub = int(E);
        // the dense levels may number up to kLpDenseFactor N (d + 1) (node,
        // vertex) pairs, the hashed ones N (d + 1)
        const size_t dense = lp_dense_cap(E);
        P.cap_dense = int(dense);
        P.ld_nb = int(std::max(E, dense));
        const size_t ld = (size_t)P.ld_nb;
        P.hkeys.ensure(cap * 8, s);
        P.slot_vid.ensure(cap * 4, s);
        P.ent_slot.ensure(E * 4, s);
        P.ent_id.ensure(E * 4, s);
        P.sub_nv.ensure(E * sizeof(int2), s);
        P.nbr_sub.ensure(ld * D1 * 2 * 4, s);
        P.mark.ensure(dense * 4, s);
        for (int b = 0; b < 3; ++b) P.V[b].ensure(ld * 2 * sizeof(T), s);
        P.pos_vid.ensure(E * 4, s);
        P.pos_w.ensure(E * sizeof(T), s);
    }
}

// The two triangular sums of column `col` of y (leading dimension ld) in the
// order of its values: on return acc[p] = U - Lo of the pixel at sorted
// position p, and the order itself is returned.
template <typename T>
int *column_pair_sums(dcrf_ctx *ctx, LPWork &W, const T *y, int ld, int col, int levels) {
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    int *perm = nullptr;
    sort_column<T>(ctx, W, y, ld, col, &perm);
    if (ctx->mode == DCRF_FILTER_EXACT) {
        ExactSet<T> ex = make_exact_set<T>(ctx);
        hipLaunchKernelGGL((k_lp_exact<T>), dim3(ceil_div(N, kLpExTile)), dim3(kLpExTile),
                           0, s, N, perm, ex, W.acc.as<T>());
        DCRF_CHECK_LAUNCH();
        return perm;
    }
    hipLaunchKernelGGL(k_lp_rank, dim3(ceil_div(N, 256)), dim3(256), 0, s, N, perm,
                       W.rank.as<int>());
    for (int m = 0; m < ctx->nk; ++m) {
        Lattice &Lt = ctx->lat[m];
        const int D1 = Lt.d + 1;
        hipLaunchKernelGGL((k_lp_gather<T>), dim3(ceil_div((long long)N * D1, 256)),
                           dim3(256), 0, s, N, D1, perm, Lt.pix_vid.as<int>(),
                           Lt.pix_w.as<T>(), W.lat[m].pos_vid.as<int>(),
                           W.lat[m].pos_w.as<T>());
    }
    // leaf-exact: lattice levels down to the first whose nodes hold at most
    // ctx->lp_leaf positions, then the exact pairs inside those nodes
    int lcut = levels;
    if (ctx->lp_leaf > 1) {
        lcut = 0;
        while (((long long)N + (1ll << lcut) - 1) >> lcut > ctx->lp_leaf) ++lcut;
    }
    for (int l = 0; l < lcut; ++l) {
        // the lattices' chains are independent until the slice: the first
        // runs on the context's stream, the others on the side stream, which
        // starts after the previous level's slice
        if (ctx->nk > 1) {
            DCRF_TRY_HIP(hipEventRecord(W.ev_start, s));
            DCRF_TRY_HIP(hipStreamWaitEvent(W.side, W.ev_start, 0));
            for (int m = 1; m < ctx->nk; ++m) lp_level<T>(ctx, W, m, l, W.side);
            DCRF_TRY_HIP(hipEventRecord(W.ev_done, W.side));
        }
        lp_level<T>(ctx, W, 0, l, s);
        if (ctx->nk > 1) DCRF_TRY_HIP(hipStreamWaitEvent(s, W.ev_done, 0));
        LPLats<T> lats{};
        lats.nk = ctx->nk;
        for (int m = 0; m < ctx->nk; ++m) {
            Lattice &Lt = ctx->lat[m];
            lats.l[m] = LPLat<T>{W.lat[m].pos_w.as<T>(), W.lat[m].ent_id.as<int>(),
                                 W.lat[m].V[final_buffer_after(lp_blur_launches(Lt.d + 1))].as<T>(), Lt.d + 1,
                                 T(ctx->kern[m].weight * Lt.gamma), W.lat[m].pos_vid.as<int>(),
                                 Lt.M, lp_dense_level(W.lat[m], Lt.M, l) ? 1 : 0};
        }
        hipLaunchKernelGGL((k_lp_slice<T>), dim3(ceil_div(N, 256)), dim3(256), 0, s, N, l,
                           lats, W.acc.as<T>());
        DCRF_CHECK_LAUNCH();
    }
    if (lcut < levels) {
        ExactSet<T> ex = make_exact_set<T>(ctx);
        if (ex.off[ex.nk] > kLpLeafMaxF)
            fail(DCRF_EUNSUPPORTED, "leaf-exact sums take at most 16 feature dimensions");
        const dim3 grid(1u << lcut), block(kLpLeafMax);
        T *acc = W.acc.as<T>();
        const int d0 = ex.d[0], d1 = ex.nk > 1 ? ex.d[1] : 0;
        if (ex.nk == 2 && d0 == 5 && d1 == 2)
            hipLaunchKernelGGL((k_lp_leaf<T, 5, 2>), grid, block, 0, s, N, lcut, perm, ex, acc);
        else if (ex.nk == 2 && d0 == 2 && d1 == 5)
            hipLaunchKernelGGL((k_lp_leaf<T, 2, 5>), grid, block, 0, s, N, lcut, perm, ex, acc);
        else if (ex.nk == 1 && d0 == 5)
            hipLaunchKernelGGL((k_lp_leaf<T, 5, 0>), grid, block, 0, s, N, lcut, perm, ex, acc);
        else if (ex.nk == 1 && d0 == 2)
            hipLaunchKernelGGL((k_lp_leaf<T, 2, 0>), grid, block, 0, s, N, lcut, perm, ex, acc);
        else
            hipLaunchKernelGGL((k_lp_leaf<T, 0, 0>), grid, block, 0, s, N, lcut, perm, ex, acc);
        DCRF_CHECK_LAUNCH();
    }
    return perm;
}

int dnc_levels(int N) {
    int levels = 0;
    while ((1ll << levels) < N) ++levels;
    return levels;
}

// S = <g, y> (the objective, eq. simple_S), after checking the sub-lattice
// hash tables' overflow flag; waits for the stream
template <typename T>
double finish_subgradient(dcrf_ctx *ctx, LPWork &W, const T *g, const T *y, size_t NL) {
    const hipStream_t s = ctx->stream;
    int hflags = 0;
    DCRF_TRY_HIP(hipMemcpyAsync(&hflags, ctx->scratch.p, 4, hipMemcpyDeviceToHost, s));
    const int G = std::min(1024, ceil_div((long long)NL, 256));
    hipLaunchKernelGGL((k_dot<T>), dim3(G), dim3(256), 0, s, NL, g, y, W.part.as<double>());
    std::vector<double> h(G);
    DCRF_TRY_HIP(hipMemcpyAsync(h.data(), W.part.p, G * 8, hipMemcpyDeviceToHost, s));
    DCRF_TRY_HIP(hipStreamSynchronize(s));
    if (hflags & 2) fail(DCRF_ECAPACITY, "LP sub-lattice hash table full");
    double S = 0.0;
    for (double v : h) S += v;
    return S;
}

template <typename T>
double lp_subgradient_t(dcrf_ctx *ctx, const T *phi, int L, const T *y, T *g) {
    LPWork &W = lp_work(ctx);
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    lp_prepare<T>(ctx, W, L);
    const size_t NL = (size_t)N * L;
    hipLaunchKernelGGL((k_copy<T>), dim3(ceil_div((long long)NL, 256)), dim3(256),
                       0, s, NL, phi, g);
    const int levels = dnc_levels(N);
    DCRF_TRY_HIP(hipMemsetAsync(ctx->scratch.p, 0, 4, s));
    for (int col = 0; col < L; ++col) {
        int *perm = column_pair_sums<T>(ctx, W, y, L, col, levels);
        hipLaunchKernelGGL((k_lp_add_col<T>), dim3(ceil_div(N, 256)), dim3(256), 0, s,
                           N, L, col, perm, W.acc.as<T>(), g);
        DCRF_CHECK_LAUNCH();
    }
    return finish_subgradient<T>(ctx, W, g, y, NL);
}

// eq. rHST-LP's subgradient (Alg. rHST): g = phi, then for every subtree
// with c_T != 0 the column y(T), its order and pair sums, and
// g(., k) += c_T (U - Lo) for the subtree's labels k
template <typename T>
double lp_subgradient_tree_t(dcrf_ctx *ctx, const T *phi, int L, const T *y, T *g,
                             const TreeSpec &tr) {
    LPWork &W = lp_work(ctx);
    const hipStream_t s = ctx->stream;
    const int N = ctx->N;
    lp_prepare<T>(ctx, W, L);
    const size_t NL = (size_t)N * L;
    W.col.ensure((size_t)N * sizeof(T), s);
    W.tree_lab.ensure(tr.lab.size() * 4, s);
    DCRF_TRY_HIP(hipMemcpyAsync(W.tree_lab.p, tr.lab.data(), tr.lab.size() * 4,
                                hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL((k_copy<T>), dim3(ceil_div((long long)NL, 256)), dim3(256),
                       0, s, NL, phi, g);
    const int levels = dnc_levels(N);
    DCRF_TRY_HIP(hipMemsetAsync(ctx->scratch.p, 0, 4, s));
    const int *labs = W.tree_lab.as<int>();
    for (int t = 0; t < tr.n; ++t) {
        const int nlab = tr.off[t + 1] - tr.off[t];
        if (tr.c[t] == 0.0 || nlab == 0) continue;
        hipLaunchKernelGGL((k_tree_col<T>), dim3(ceil_div(N, 256)), dim3(256), 0, s, N, L, y,
                           labs + tr.off[t], nlab, W.col.as<T>());
        int *perm = column_pair_sums<T>(ctx, W, W.col.as<T>(), 1, 0, levels);
        hipLaunchKernelGGL((k_lp_add_tree<T>), dim3(ceil_div(N, 256)), dim3(256), 0, s, N,
                           L, perm, W.acc.as<T>(), T(tr.c[t]), labs + tr.off[t], nlab, g);
        DCRF_CHECK_LAUNCH();
    }
    return finish_subgradient<T>(ctx, W, g, y, NL);
}

template <typename T>
void project_t(dcrf_ctx *ctx, const T *src, const T *g, T beta, int L, T *dst) {
    const int N = ctx->N;
    if (L <= kRowMaxC) {
        DCRF_DISPATCH_ROWS(L, hipLaunchKernelGGL((k_lp_step_rows<T, LMAX>),
                                                 dim3(ceil_div(N, 128)), dim3(128),
                                                 0, ctx->stream, N, L, src, g, beta,
                                                 dst));
    } else {
        hipLaunchKernelGGL((k_lp_step_flat<T>), dim3(ceil_div(N, 128)), dim3(128),
                           0, ctx->stream, N, L, src, g, beta, dst);
    }
    DCRF_CHECK_LAUNCH();
}

// projected subgradient descent (Alg. lp_subgrad, Alg. rHST):
// y <- Pi(y - beta0 / (1 + t) g(y)), keeping the best objective seen
template <typename T, typename Subgradient>
void descent_t(dcrf_ctx *ctx, LPWork &W, int L, T *y, int steps, double beta0,
               double *best, T *best_y, double *hist, Subgradient subgradient) {
    const size_t NL = (size_t)ctx->N * L;
    double b = INFINITY;
    for (int t = 0; t < steps; ++t) {
        T *g = W.g.as<T>();
        const double S = subgradient(g);
        if (hist) hist[t] = S;
        if (S < b) {
            b = S;
            if (best_y)
                hipLaunchKernelGGL((k_copy<T>), dim3(ceil_div((long long)NL, 256)),
                                   dim3(256), 0, ctx->stream, NL, y, best_y);
        }
        project_t<T>(ctx, y, g, T(beta0 / (1.0 + t)), L, y);
    }
    if (best) *best = b;
}

template <typename T>
void lp_descent_t(dcrf_ctx *ctx, const T *phi, int L, T *y, int steps,
                  double beta0, double *best, T *best_y, double *hist) {
    LPWork &W = lp_work(ctx);
    lp_prepare<T>(ctx, W, L);
    descent_t<T>(ctx, W, L, y, steps, beta0, best, best_y, hist,
                 [&](T *g) { return lp_subgradient_t<T>(ctx, phi, L, y, g); });
}

template <typename T>
void lp_descent_tree_t(dcrf_ctx *ctx, const T *phi, int L, T *y, const TreeSpec &tr,
                       int steps, double beta0, double *best, T *best_y, double *hist) {
    LPWork &W = lp_work(ctx);
    lp_prepare<T>(ctx, W, L);
    descent_t<T>(ctx, W, L, y, steps, beta0, best, best_y, hist,
                 [&](T *g) { return lp_subgradient_tree_t<T>(ctx, phi, L, y, g, tr); });
}

}  // namespace

void lp_release(dcrf_ctx *ctx) {
    if (!ctx->lp) return;
    LPWork *W = static_cast<LPWork *>(ctx->lp);
    if (W->side) {
        (void)hipStreamSynchronize(W->side);
        (void)hipStreamDestroy(W->side);
        (void)hipEventDestroy(W->ev_start);
        (void)hipEventDestroy(W->ev_done);
    }
    for (DevBuf *b : {&W->keys, &W->keys2, &W->vals, &W->vals2, &W->hist, &W->g,
                      &W->part, &W->acc, &W->rank, &W->col, &W->tree_lab})
        b->release();
    for (auto &P : W->lat)
        for (DevBuf *b : {&P.hkeys, &P.slot_vid, &P.ent_slot, &P.ent_id,
                          &P.sub_nv, &P.nbr_sub, &P.V[0], &P.V[1], &P.V[2],
                          &P.mark, &P.pos_vid, &P.pos_w})
            b->release();
    delete W;
    ctx->lp = nullptr;
}

double lp_subgradient(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                      void *g) {
    if (ctx->dtype == DCRF_F64)
        return lp_subgradient_t<double>(ctx, static_cast<const double *>(unary), L,
                                        static_cast<const double *>(y),
                                        static_cast<double *>(g));
    return lp_subgradient_t<float>(ctx, static_cast<const float *>(unary), L,
                                   static_cast<const float *>(y),
                                   static_cast<float *>(g));
}

void lp_descent(dcrf_ctx *ctx, const void *unary, int L, void *y, int steps,
                double beta0, double *best, void *best_y, double *hist) {
    if (ctx->dtype == DCRF_F64)
        lp_descent_t<double>(ctx, static_cast<const double *>(unary), L,
                             static_cast<double *>(y), steps, beta0, best,
                             static_cast<double *>(best_y), hist);
    else
        lp_descent_t<float>(ctx, static_cast<const float *>(unary), L,
                            static_cast<float *>(y), steps, beta0, best,
                            static_cast<float *>(best_y), hist);
}

TreeSpec tree_spec(const int32_t *parent, const double *c, int n, int L) {
    if (n < L || n > kMaxTreeNodes)
        fail(DCRF_EINVAL, "n_nodes must be in [L, " + std::to_string(kMaxTreeNodes) + "]");
    int roots = 0;
    for (int t = 0; t < n; ++t) {
        if (parent[t] < -1 || parent[t] >= n || parent[t] == t)
            fail(DCRF_EINVAL, "parent[" + std::to_string(t) + "] is not a node index or -1");
        if (parent[t] >= 0 && parent[t] < L)
            fail(DCRF_EINVAL, "a label's node (0..L-1) cannot be a parent");
        if (parent[t] == -1) ++roots;
        if (!std::isfinite(c[t]) || c[t] < 0.0)
            fail(DCRF_EINVAL, "the subtree weights c must be finite and >= 0");
    }
    if (roots != 1) fail(DCRF_EINVAL, "the tree must have exactly one root (parent -1)");
    std::vector<std::vector<int>> labs(n);
    for (int k = 0; k < L; ++k) {
        int t = k, hops = 0;
        while (t >= 0) {
            if (++hops > n) fail(DCRF_EINVAL, "parent[] has a cycle");
            labs[t].push_back(k);
            t = parent[t];
        }
    }
    TreeSpec tr;
    tr.n = n;
    tr.c.assign(c, c + n);
    tr.off.push_back(0);
    for (int t = 0; t < n; ++t) {
        tr.lab.insert(tr.lab.end(), labs[t].begin(), labs[t].end());
        tr.off.push_back(int(tr.lab.size()));
    }
    return tr;
}

double lp_subgradient_tree(dcrf_ctx *ctx, const void *unary, int L, const void *y,
                           const TreeSpec &tr, void *g) {
    if (ctx->dtype == DCRF_F64)
        return lp_subgradient_tree_t<double>(ctx, static_cast<const double *>(unary), L,
                                             static_cast<const double *>(y),
                                             static_cast<double *>(g), tr);
    return lp_subgradient_tree_t<float>(ctx, static_cast<const float *>(unary), L,
                                        static_cast<const float *>(y),
                                        static_cast<float *>(g), tr);
}

void lp_descent_tree(dcrf_ctx *ctx, const void *unary, int L, void *y, const TreeSpec &tr,
                     int steps, double beta0, double *best, void *best_y, double *hist) {
    if (ctx->dtype == DCRF_F64)
        lp_descent_tree_t<double>(ctx, static_cast<const double *>(unary), L,
                                  static_cast<double *>(y), tr, steps, beta0, best,
                                  static_cast<double *>(best_y), hist);
    else
        lp_descent_tree_t<float>(ctx, static_cast<const float *>(unary), L,
                                 static_cast<float *>(y), tr, steps, beta0, best,
                                 static_cast<float *>(best_y), hist);
}

void project_simplex(dcrf_ctx *ctx, const void *v, int L, void *y) {
    if (ctx->dtype == DCRF_F64)
        project_t<double>(ctx, static_cast<const double *>(v), nullptr, 0.0, L,
                          static_cast<double *>(y));
    else
        project_t<float>(ctx, static_cast<const float *>(v), nullptr, 0.0f, L,
                         static_cast<float *>(y));
}

}  // namespace dcrf
