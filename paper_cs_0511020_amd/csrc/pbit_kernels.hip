// HIP kernels (gfx950) of the Pbit list sort.
//
// Path for one list of n nodes (the split/concatenate method of the paper's
// Sec. 3 and Sec. 5, reorganised for a wide machine):
//   pack       next[] and keys[] become one 8- or 16-byte record per node so a
//              walk step is one random access; the histograms of every K-bit
//              pattern are counted here (order-free).
//   walk0      sparse-ruler list ranking, level 0: every node whose index is a
//              multiple of 16 (and the head) starts a segment; each lane walks
//              its segment keeping up to 16 (key, node) entries in registers,
//              then writes them as one block.
//   walk_up    the same on the list of segments, recursively, until the list
//              fits one workgroup.
//   base       pointer jumping (Wyllie) in LDS over the last level.
//   down       offsets flow back down the levels.
//   unchain    segment contents are copied to list order.
//   schedule   per-pass digit bases; passes whose pattern is constant are
//              skipped (the identity), the paper's "empty groups are omitted".
//   digit pass stable K-bit split per pattern, least significant first:
//              wave ballot ranking, LDS tile staging, decoupled look-back.
//              Least-significant-first stable passes give the same order as
//              the paper's most-significant-first recursion (both are the
//              stable sort by the full key).
//   relink     next[order[j]] = order[j+1], the concatenation of Sec. 5.1.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pbit.h"
#include "pbit_internal.h"

namespace pbit {

// ---------------------------------------------------------------- records
template <typename KeyT> struct NodeRec { uint32_t next; uint32_t key; };
template <> struct __attribute__((aligned(16))) NodeRec<uint64_t> { uint32_t next; uint32_t pad; uint64_t key; };

template <typename KeyT> struct Entry { uint32_t key; uint32_t idx; };
template <> struct __attribute__((aligned(16))) Entry<uint64_t> { uint64_t key; uint32_t idx; uint32_t pad; };

// Digit-pass tile: kPassBlock threads x PassItems items.
constexpr int kPassBlock = 512;
template <typename KeyT> struct PassItems { static constexpr int value = sizeof(KeyT) == 8 ? 8 : 16; };
uint32_t pass_tile(uint32_t key_bytes) { return kPassBlock * (key_bytes == 8 ? 8 : 16); }

// Entries of a level-0 chain kept in registers by its walker.
template <typename KeyT> struct SegLen { static constexpr uint32_t value = sizeof(KeyT) == 8 ? 16 : 32; };
// Entries stored per level-0 chain slot; nodes past this are re-walked.
constexpr uint32_t kChainCap = 128;

template <typename KeyT> __device__ __forceinline__ KeyT entry_key(const Entry<KeyT>& e) { return (KeyT)e.key; }

__device__ __forceinline__ void set_error(int32_t* status, int32_t code)
{
    atomicCAS(status, 0, code);
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_agent(uint32_t* p, uint32_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- init
__global__ void k_zero(uint32_t* __restrict__ p, size_t words)
{
    size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride)
        p[i] = 0u;
}

__device__ __forceinline__ uint64_t mix64(uint64_t x, uint64_t k)
{
    x ^= x >> 31;
    x *= k;
    x ^= x >> 29;
    x *= 0xBF58476D1CE4E5B9ull;
    x ^= x >> 32;
    return x;
}
constexpr uint64_t kHashK1 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kHashK2 = 0xD6E8FEB86659FD93ull;

// Every walk kernel starts here: a list passes only if exactly one next[] is
// NIL and the non-NIL next[] values are all nodes but the head, once each.
__device__ __forceinline__ bool list_shape_ok(const Header* hdr, uint32_t head)
{
    return hdr->status == 0 && hdr->nil_count == 1 &&
           hdr->hsum[0] + mix64(head + 1ull, kHashK1) == 0 &&
           hdr->hsum[1] + mix64(head + 1ull, kHashK2) == 0;
}

// ---------------------------------------------------------------- pack
// Node records and the count of every pattern value of every pass.
template <typename KeyT, int RB>
__global__ __launch_bounds__(256) void k_pack(const uint32_t* __restrict__ next,
                                              const KeyT* __restrict__ keys, uint32_t n,
                                              KeyT xor_mask, uint32_t passes,
                                              NodeRec<KeyT>* __restrict__ nodes,
                                              uint32_t* __restrict__ hist, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    extern __shared__ uint32_t s_hist[];  // passes * RADIX
    const uint32_t nbins = passes * RADIX;
    for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x)
        s_hist[i] = 0;
    __syncthreads();
    bool bad = false;
    uint64_t h1 = 0, h2 = 0;
    uint32_t nils = 0;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t nx = next[i];
        const KeyT k = keys[i] ^ xor_mask;
        bad |= (nx != kNil) && (nx >= n);
        if (nx == kNil) {
            nils++;
        } else {
            h1 += mix64(nx + 1ull, kHashK1);
            h2 += mix64(nx + 1ull, kHashK2);
        }
        h1 -= mix64(i + 1ull, kHashK1);
        h2 -= mix64(i + 1ull, kHashK2);
        NodeRec<KeyT> r;
        r.next = nx;
        r.key = k;
        if constexpr (sizeof(KeyT) == 8) r.pad = 0;
        nodes[i] = r;
        for (uint32_t p = 0; p < passes; p++) {
            const uint32_t d = (uint32_t)(k >> (p * RB)) & (RADIX - 1u);
            atomicAdd(&s_hist[p * RADIX + d], 1u);
        }
    }
    if (bad)
        set_error(&hdr->status, PBIT_EMALFORMED);
    // block sums of the in-degree hashes and the NIL count
    for (int off = 32; off > 0; off >>= 1) {
        h1 += (uint64_t)__shfl_xor((unsigned long long)h1, off, 64);
        h2 += (uint64_t)__shfl_xor((unsigned long long)h2, off, 64);
        nils += __shfl_xor(nils, off, 64);
    }
    __shared__ uint64_t s_h[2][4];
    __shared__ uint32_t s_nil[4];
    const uint32_t wave = threadIdx.x / 64;
    if (__lane_id() == 0) {
        s_h[0][wave] = h1;
        s_h[1][wave] = h2;
        s_nil[wave] = nils;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t a = 0, b = 0;
        uint32_t z = 0;
        for (uint32_t w = 0; w < blockDim.x / 64; w++) {
            a += s_h[0][w];
            b += s_h[1][w];
            z += s_nil[w];
        }
        atomicAdd((unsigned long long*)&hdr->hsum[0], (unsigned long long)a);
        atomicAdd((unsigned long long*)&hdr->hsum[1], (unsigned long long)b);
        if (z)
            atomicAdd(&hdr->nil_count, z);
    }
    for (uint32_t i = threadIdx.x; i < nbins; i += blockDim.x) {
        const uint32_t v = s_hist[i];
        if (v)
            atomicAdd(&hist[i], v);
    }
}

// ---------------------------------------------------------------- list ranking
// Sparse-ruler ranking (Helman & JaJa style).  At level k the elements
// 0..m-1 form a list from `head` (element 0 for k >= 1).  Chain 0 starts at
// the head, chain 1 + j/L at element j for every multiple j of L = 2^log_l
// other than the head; a chain runs up to the next chain start or NIL.  One
// thread walks one chain to its end: no atomics, and the hardware refills a
// wave slot as soon as a wave's chains are done.  A chain's record is
// {successor chain or NIL, weight}; the chains form the list of level k + 1.
//
// Level 0 keeps the first SegLen (key, node) entries of its chain in
// registers, stores the following ones straight to the chain's slot of
// kChainCap entries, and records the node where a longer chain resumes; after
// ranking, walk2 re-walks only those (rare) rests.
// Levels >= 1 store nothing: their down pass walks the chain again.
//
// The walks assume every node has at most one predecessor; pack verifies it
// (hash sums over next[]), so every node is walked once in total and a bad
// list is rejected before any walk starts.

template <typename KeyT>
__global__ __launch_bounds__(256) void k_walk0(const NodeRec<KeyT>* __restrict__ nodes, uint32_t n,
                                               uint32_t head, uint32_t n_static,
                                               uint2* __restrict__ chain_rec,
                                               Entry<KeyT>* __restrict__ ent,
                                               uint32_t* __restrict__ resume, Header* hdr)
{
    constexpr uint32_t C = SegLen<KeyT>::value;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    if (!list_shape_ok(hdr, head)) {
        if (c == 0 && hdr->status == 0)
            set_error(&hdr->status, PBIT_EMALFORMED);
        return;
    }
    uint32_t start = head;
    if (c != 0) {
        const uint64_t s = (uint64_t)(c - 1) << kLog0;
        if (s >= n || (uint32_t)s == head) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = (uint32_t)s;
    }
    const uint32_t lmask = (1u << kLog0) - 1u;
    Entry<KeyT> e[C];
    uint32_t cur = start, len = 0, nx = kNil;
    bool stop = false;
#pragma unroll
    for (uint32_t t = 0; t < C; t++) {
        if (!stop) {
            const NodeRec<KeyT> r = nodes[cur];
            e[t].key = r.key;
            e[t].idx = cur;
            if constexpr (sizeof(KeyT) == 8) e[t].pad = 0;
            len = t + 1;
            nx = r.next;
            if (nx == kNil || nx >= n || (nx & lmask) == 0 || nx == head)
                stop = true;
            else
                cur = nx;
        }
    }
    Entry<KeyT>* b = ent + (size_t)c * kChainCap;
    uint32_t rest_from = kNil;
    while (!stop) {
        const NodeRec<KeyT> r = nodes[cur];
        if (len < kChainCap) {
            Entry<KeyT> x;
            x.key = r.key;
            x.idx = cur;
            if constexpr (sizeof(KeyT) == 8) x.pad = 0;
            b[len] = x;
        } else if (len == kChainCap) {
            rest_from = cur;
        }
        len++;
        nx = r.next;
        if (nx == kNil || nx >= n || (nx & lmask) == 0 || nx == head || len >= n)
            stop = true;
        else
            cur = nx;
    }
    if (nx != kNil && nx >= n) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        nx = kNil;
    }
#pragma unroll
    for (uint32_t t = 0; t < C; t++)
        if (t < len)
            b[t] = e[t];
    resume[c] = rest_from;
    const uint32_t succ = (nx == kNil) ? kNil : (nx == head ? 0u : 1u + (nx >> kLog0));
    chain_rec[c] = make_uint2(succ, len);
}

// Level >= 1: chains over the records {successor, weight} of level k.
__global__ __launch_bounds__(256) void k_walk_up(const uint2* __restrict__ recs, uint32_t m,
                                                 uint32_t log_l, uint32_t n_static,
                                                 uint2* __restrict__ chain_rec, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    uint32_t start = 0;
    if (c != 0) {
        const uint64_t s = (uint64_t)(c - 1) << log_l;
        if (s >= m || s == 0) {
            chain_rec[c] = make_uint2(kNil, 0);
            return;
        }
        start = (uint32_t)s;
    }
    const uint32_t lmask = (1u << log_l) - 1u;
    uint32_t cur = start, w = 0, steps = 0, nx;
    for (;;) {
        const uint2 r = recs[cur];
        if (r.y == 0) {  // empty chain of the level below: not part of a list
            set_error(&hdr->status, PBIT_EMALFORMED);
            nx = kNil;
            break;
        }
        w += r.y;
        nx = r.x;
        if (nx == kNil || nx >= m || (nx & lmask) == 0 || ++steps >= m)
            break;
        cur = nx;
    }
    if (nx != kNil && (nx >= m || steps >= m)) {
        set_error(&hdr->status, PBIT_EMALFORMED);
        nx = kNil;
    }
    chain_rec[c] = make_uint2(nx == kNil ? kNil : (nx == 0 ? 0u : 1u + (nx >> log_l)), w);
}

// ---------------------------------------------------------------- base
// Pointer jumping (Wyllie) in LDS: suffix weights from every element to the
// end of the list, then offset = total - suffix.  The list must end in NIL
// from element 0 and cover exactly n nodes.
constexpr int kBaseThreads = 1024;
constexpr int kBasePer = kBaseMax / kBaseThreads;

__global__ __launch_bounds__(kBaseThreads) void k_base(const uint2* __restrict__ rec, uint32_t m,
                                                       uint32_t n_total,
                                                       uint32_t* __restrict__ offn, Header* hdr)
{
    __shared__ uint32_t s_ptr[kBaseMax];
    __shared__ uint32_t s_val[kBaseMax];
    __shared__ int s_bad;
    if (hdr->status != 0)
        return;
    m = min(m, kBaseMax);
    const int tid = threadIdx.x;
    if (tid == 0)
        s_bad = 0;
    for (int j = 0; j < kBasePer; j++) {
        const uint32_t i = tid + j * kBaseThreads;
        uint32_t p = kNil, v = 0;
        if (i < m) {
            const uint2 r = rec[i];
            if (r.y != 0) {
                p = (r.x != kNil && r.x >= m) ? kNil : r.x;  // caught below: total != n
                v = r.y;
            }
        }
        s_ptr[i] = p;
        s_val[i] = v;
    }
    __syncthreads();
    int rounds = 1;
    while ((1u << (rounds - 1)) < m)
        rounds++;
    for (int r = 0; r < rounds; r++) {
        uint32_t np[kBasePer], nv[kBasePer];
#pragma unroll
        for (int j = 0; j < kBasePer; j++) {
            const uint32_t i = tid + j * kBaseThreads;
            uint32_t p = s_ptr[i];
            uint32_t v = s_val[i];
            if (p != kNil) {
                v += s_val[p];
                p = s_ptr[p];
            }
            np[j] = p;
            nv[j] = v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kBasePer; j++) {
            const uint32_t i = tid + j * kBaseThreads;
            s_ptr[i] = np[j];
            s_val[i] = nv[j];
        }
        __syncthreads();
    }
    const uint32_t total = s_val[0];
    if (tid == 0 && (m == 0 || s_ptr[0] != kNil || total != n_total)) {
        s_bad = 1;
        set_error(&hdr->status, PBIT_EMALFORMED);
    }
    __syncthreads();
    if (s_bad)
        return;
    for (int j = 0; j < kBasePer; j++) {
        const uint32_t i = tid + j * kBaseThreads;
        if (i < m)
            offn[i] = total - s_val[i];
    }
}

// ---------------------------------------------------------------- down
// Level k >= 1: walk each chain again, giving each element its offset
// (chain offset plus the weights before it).
__global__ __launch_bounds__(256) void k_down(const uint2* __restrict__ recs, uint32_t m,
                                              uint32_t log_l, uint32_t n_static,
                                              const uint2* __restrict__ chain_rec,
                                              const uint32_t* __restrict__ offn_chain,
                                              uint32_t* __restrict__ offn_elem, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    const uint2 cr = chain_rec[c];
    if (cr.y == 0)
        return;
    const uint32_t start = c == 0 ? 0u : (c - 1) << log_l;
    const uint32_t lmask = (1u << log_l) - 1u;
    uint32_t cur = start, off = offn_chain[c];
    for (uint32_t steps = 0; steps < m; steps++) {
        const uint2 r = recs[cur];
        offn_elem[cur] = off;
        off += r.y;
        const uint32_t nx = r.x;
        if (nx == kNil || nx >= m || (nx & lmask) == 0)
            break;
        cur = nx;
    }
}

// ---------------------------------------------------------------- unchain
// The stored head of every level-0 chain to list order.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_unchain(const uint2* __restrict__ chain_rec,
                                                 const Entry<KeyT>* __restrict__ ent,
                                                 uint32_t n_static,
                                                 const uint32_t* __restrict__ offn_chain, uint32_t n,
                                                 KeyT* __restrict__ keys_l,
                                                 uint32_t* __restrict__ idx_l, Header* hdr)
{
    constexpr uint32_t G = 16;  // threads per chain
    if (hdr->status != 0)
        return;
    const uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint32_t c = (uint32_t)(g / G);
    if (c >= n_static)
        return;
    const uint32_t len = min(chain_rec[c].y, kChainCap);
    const uint32_t base = offn_chain[c];
    const Entry<KeyT>* b = ent + (size_t)c * kChainCap;
    for (uint32_t t = (uint32_t)(g % G); t < len; t += G) {
        const uint32_t pos = base + t;
        if (pos >= n)
            break;
        const Entry<KeyT> e = b[t];
        keys_l[pos] = entry_key<KeyT>(e);
        idx_l[pos] = e.idx;
    }
}

// The rest of every level-0 chain longer than its slot, walked again from
// its resume node and written straight to list order.
template <typename KeyT>
__global__ __launch_bounds__(256) void k_walk2(const NodeRec<KeyT>* __restrict__ nodes,
                                               const uint2* __restrict__ chain_rec,
                                               const uint32_t* __restrict__ resume,
                                               uint32_t n_static,
                                               const uint32_t* __restrict__ offn_chain, uint32_t n,
                                               KeyT* __restrict__ keys_l,
                                               uint32_t* __restrict__ idx_l, Header* hdr)
{
    if (hdr->status != 0)
        return;
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_static)
        return;
    const uint32_t len = chain_rec[c].y;
    if (len <= kChainCap)
        return;
    uint32_t cur = resume[c];
    uint32_t pos = offn_chain[c] + kChainCap;
    const uint32_t end = min(offn_chain[c] + len, n);
    while (pos < end && cur < n) {
        const NodeRec<KeyT> r = nodes[cur];
        keys_l[pos] = (KeyT)r.key;
        idx_l[pos] = cur;
        pos++;
        cur = r.next;
    }
}

// ---------------------------------------------------------------- schedule
// Per pass: exclusive scan of the digit counts (global digit bases), whether
// the pass is the identity, and which ping-pong buffer it reads.
template <int RB>
__global__ __launch_bounds__(256) void k_schedule(const uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ dbase, uint32_t passes,
                                                  uint32_t n, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    __shared__ uint32_t s_v[RADIX];
    __shared__ uint32_t s_skip[kMaxPasses];
    const uint32_t tid = threadIdx.x;
    for (uint32_t p = 0; p < passes; p++) {
        uint32_t v = 0;
        if (tid < RADIX)
            v = hist[p * RADIX + tid];
        if (tid < RADIX)
            s_v[tid] = v;
        __syncthreads();
        int full = (tid < RADIX) && (v == n);
        int any_full = __syncthreads_or(full);
        if (tid == 0) {
            uint32_t sum = 0;
            for (uint32_t d = 0; d < RADIX; d++) {
                uint32_t x = s_v[d];
                s_v[d] = sum;
                sum += x;
            }
            s_skip[p] = any_full ? 1u : 0u;
        }
        __syncthreads();
        if (tid < RADIX)
            dbase[p * RADIX + tid] = s_v[tid];
        __syncthreads();
    }
    if (tid == 0) {
        uint32_t cur = 0;
        int last = -1;
        for (uint32_t p = 0; p < passes; p++) {
            PassSched ps;
            ps.skip = s_skip[p];
            ps.in_buf = cur;
            ps.last = 0;
            ps.pad = 0;
            if (!ps.skip) {
                cur ^= 1u;
                last = (int)p;
            }
            hdr->sched[p] = ps;
        }
        if (last >= 0)
            hdr->sched[last].last = 1;
        hdr->final_buf = cur;
    }
}

// ---------------------------------------------------------------- digit pass
// One stable split on the pattern at bit `shift`.  A tile of BLOCK * ITEMS
// consecutive list positions (tile = block index) is loaded wave-striped,
// ranked per wave (K ballots give each item the mask of lanes with the same
// digit; the first lane of each group adds the group size to a wave-private
// LDS counter with one in-order LDS atomic, and peers take the returned base
// from it), scanned across waves, chained across tiles by decoupled look-back
// (Merrill & Garland), staged in LDS grouped by digit and written out in
// runs.  The look-back spin is bounded: a tile that waits too long on a
// predecessor counts that predecessor's digit in its input itself, so no
// tile ever waits on a tile that has not been scheduled.
template <typename KeyT> struct KV { KeyT key; uint32_t idx; };

__device__ __forceinline__ uint64_t lanemask_lt()
{
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

constexpr uint32_t kSpinLimit = 4096;

template <typename KeyT, int RB, int BLOCK, int ITEMS>
__global__ __launch_bounds__(BLOCK, 4) void k_digit_pass(uint32_t pass, uint32_t shift, uint32_t n,
                                                      KeyT* __restrict__ keysA,
                                                      uint32_t* __restrict__ idxA,
                                                      KeyT* __restrict__ keysB,
                                                      uint32_t* __restrict__ idxB,
                                                      const uint32_t* __restrict__ dbase,
                                                      uint32_t* __restrict__ look, Header* hdr)
{
    constexpr uint32_t RADIX = 1u << RB;
    constexpr uint32_t WAVES = BLOCK / 64;
    constexpr uint32_t TILE = BLOCK * ITEMS;
    __shared__ uint32_t s_wave[WAVES][RADIX];
    __shared__ uint32_t s_count[RADIX];
    __shared__ uint32_t s_start[RADIX];
    __shared__ int32_t s_delta[RADIX];
    __shared__ KV<KeyT> s_kv[TILE];

    if (hdr->status != 0)
        return;
    const PassSched ps = hdr->sched[pass];
    if (ps.skip)
        return;
    const KeyT* kin = ps.in_buf ? keysB : keysA;
    const uint32_t* iin = ps.in_buf ? idxB : idxA;
    KeyT* kout = ps.in_buf ? keysA : keysB;
    uint32_t* iout = ps.in_buf ? idxA : idxB;

    const uint32_t tid = threadIdx.x;
    const uint32_t wave = tid / 64, lane = tid % 64;
    for (uint32_t i = tid; i < WAVES * RADIX; i += BLOCK)
        (&s_wave[0][0])[i] = 0;
    __syncthreads();
    const uint32_t tile = blockIdx.x;
    const uint64_t tbase = (uint64_t)tile * TILE;
    const uint64_t wbase = tbase + (uint64_t)wave * (64 * ITEMS);

    KeyT key[ITEMS];
    uint32_t idx[ITEMS], dig[ITEMS], rank[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint64_t e = wbase + (uint64_t)i * 64 + lane;
        if (e < n) {
            key[i] = kin[e];
            idx[i] = iin[e];
            dig[i] = (uint32_t)(key[i] >> shift) & (RADIX - 1u);
        } else {
            key[i] = 0;
            idx[i] = 0;
            dig[i] = RADIX;
        }
    }
    // dig[i] bits: 0..8 digit (RADIX = invalid), 16..21 rank in the wave's
    // group, 24..29 the group's first lane (which holds the LDS base)
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const bool valid = dig[i] < RADIX;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < RB; b++) {
            const bool bit = (dig[i] >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t first = valid ? (uint32_t)(__ffsll((unsigned long long)peers) - 1) : lane;
        uint32_t base = 0;
        if (valid && below == 0)
            base = atomicAdd(&s_wave[wave][dig[i]], (uint32_t)__popcll(peers));
        rank[i] = base;
        dig[i] |= (below << 16) | (first << 24);
    }
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        rank[i] = __shfl(rank[i], (int)(dig[i] >> 24), 64) + ((dig[i] >> 16) & 0xFFu);
        dig[i] &= 0xFFFFu;
    }
    __syncthreads();
    // per digit: exclusive offsets across waves and the tile count
    for (uint32_t d = tid; d < RADIX; d += BLOCK) {
        uint32_t sum = 0;
#pragma unroll
        for (uint32_t w = 0; w < WAVES; w++) {
            const uint32_t v = s_wave[w][d];
            s_wave[w][d] = sum;
            sum += v;
        }
        s_count[d] = sum;
        // publish this tile's count early so successors can proceed
        st_agent(&look[(size_t)tile * RADIX + d], (tile == 0 ? kFlagPrefix : kFlagAgg) | sum);
    }
    __syncthreads();
    // local digit starts (exclusive scan over digits) by wave 0
    if (wave == 0) {
        constexpr uint32_t PER = (RADIX + 63) / 64;
        uint32_t vals[PER];
        uint32_t local = 0;
#pragma unroll
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t d = lane * PER + j;
            vals[j] = d < RADIX ? s_count[d] : 0;
            local += vals[j];
        }
        uint32_t incl = local;
#pragma unroll
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint32_t up = __shfl_up(incl, off, 64);
            if (lane >= off)
                incl += up;
        }
        uint32_t run = incl - local;
#pragma unroll
        for (uint32_t j = 0; j < PER; j++) {
            const uint32_t d = lane * PER + j;
            if (d < RADIX)
                s_start[d] = run;
            run += vals[j];
        }
    }
    __syncthreads();
    // decoupled look-back per digit
    for (uint32_t d = tid; d < RADIX; d += BLOCK) {
        uint32_t excl = 0;
        if (tile != 0) {
            int64_t j = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (j >= 0) {
                const uint32_t v = ld_agent(&look[(size_t)j * RADIX + d]);
                const uint32_t f = v & ~kCountMask;
                if (f == 0) {
                    if (++spins <= kSpinLimit) {
                        __builtin_amdgcn_s_sleep(1);
                        continue;
                    }
                    // predecessor not running yet: count its digit d directly
                    const uint64_t b0 = (uint64_t)j * TILE;
                    const uint64_t b1 = min<uint64_t>(b0 + TILE, (uint64_t)n);
                    uint32_t c = 0;
                    for (uint64_t q = b0; q < b1; q++)
                        c += ((uint32_t)(kin[q] >> shift) & (RADIX - 1u)) == d;
                    excl += c;
                    j--;
                    spins = 0;
                    continue;
                }
                excl += v & kCountMask;
                if (f == kFlagPrefix)
                    break;
                j--;
                spins = 0;
            }
            st_agent(&look[(size_t)tile * RADIX + d], kFlagPrefix | (excl + s_count[d]));
        }
        s_delta[d] = (int32_t)(dbase[d] + excl) - (int32_t)s_start[d];
    }
    // stage the tile in LDS grouped by digit (stable)
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        if (dig[i] < RADIX) {
            const uint32_t pos = s_start[dig[i]] + s_wave[wave][dig[i]] + rank[i];
            KV<KeyT> kv;
            kv.key = key[i];
            kv.idx = idx[i];
            s_kv[pos] = kv;
        }
    }
    __syncthreads();
    const uint32_t valid_n = (uint32_t)min<uint64_t>((uint64_t)TILE, (uint64_t)n - tbase);
#pragma unroll
    for (int i = 0; i < ITEMS; i++) {
        const uint32_t j = tid + i * BLOCK;
        if (j < valid_n) {
            const KV<KeyT> kv = s_kv[j];
            const uint32_t d = (uint32_t)(kv.key >> shift) & (RADIX - 1u);
            const uint32_t g = (uint32_t)((int32_t)j + s_delta[d]);
            if (g < n) {
                if (!ps.last)
                    kout[g] = kv.key;
                iout[g] = kv.idx;
            }
        }
    }
}

// ---------------------------------------------------------------- relink
// next[order[j]] = order[j+1]; the last node gets NIL; result = {head, status}.
__global__ __launch_bounds__(256) void k_relink(const uint32_t* __restrict__ idxA,
                                                const uint32_t* __restrict__ idxB, uint32_t n,
                                                uint32_t* __restrict__ next_out,
                                                uint32_t* __restrict__ result, const Header* hdr)
{
    const int32_t st = hdr->status;
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (st != 0) {
        if (j == 0) {
            result[0] = kNil;
            result[1] = (uint32_t)st;
        }
        return;
    }
    const uint32_t* order = hdr->final_buf ? idxB : idxA;
    if (j < n) {
        const uint32_t node = order[j];
        const uint32_t succ = (j + 1 < n) ? order[j + 1] : kNil;
        if (node < n)
            next_out[node] = succ;
        if (j == 0) {
            result[0] = node;
            result[1] = 0;
        }
    }
}

__global__ void k_empty_result(uint32_t* result)
{
    result[0] = kNil;
    result[1] = 0;
}

// ---------------------------------------------------------------- launch helpers
template <typename KeyT>
struct Launcher {
    static hipError_t pack(const Plan& P, const uint32_t* next, const void* keys, char* ws,
                           hipStream_t s);
    static hipError_t walk0(const Plan& P, uint32_t head, char* ws, hipStream_t s);
    static hipError_t unchain(const Plan& P, char* ws, hipStream_t s, Prof* prof);
    static hipError_t passes(const Plan& P, char* ws, hipStream_t s, Prof* prof);
};

template <typename KeyT, int RB>
static hipError_t launch_pack_rb(const Plan& P, const uint32_t* next, const void* keys,
                                 char* ws, hipStream_t s)
{
    KeyT mask = 0;
    if (P.flags & PBIT_SIGNED)
        mask ^= (KeyT)((KeyT)1 << (sizeof(KeyT) * 8 - 1));
    if (P.flags & PBIT_DESCENDING)
        mask ^= (KeyT)~(KeyT)0;
    uint64_t want = (P.n + 255) / 256;
    uint32_t blocks = (uint32_t)(want < 1024 ? want : 1024);
    size_t shm = (size_t)P.passes * P.radix * sizeof(uint32_t);
    hipLaunchKernelGGL((k_pack<KeyT, RB>), dim3(blocks), dim3(256), shm, s, next,
                       (const KeyT*)keys, (uint32_t)P.n, mask, P.passes,
                       (NodeRec<KeyT>*)(ws + P.o_nodes), (uint32_t*)(ws + P.o_hist),
                       (Header*)(ws + P.o_header));
    return hipGetLastError();
}

static inline void mark(Prof* prof, hipStream_t s, int32_t stage);

template <typename KeyT, int RB>
static hipError_t launch_passes_rb(const Plan& P, char* ws, hipStream_t s, Prof* prof)
{
    constexpr int BLOCK = kPassBlock;
    constexpr int ITEMS = PassItems<KeyT>::value;
    constexpr uint32_t RADIX = 1u << RB;
    mark(prof, s, kStageSchedule);
    hipLaunchKernelGGL((k_schedule<RB>), dim3(1), dim3(256), 0, s,
                       (const uint32_t*)(ws + P.o_hist), (uint32_t*)(ws + P.o_dbase), P.passes,
                       (uint32_t)P.n, (Header*)(ws + P.o_header));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    for (uint32_t p = 0; p < P.passes; p++) {
        uint32_t* look = (uint32_t*)(ws + P.o_look) + (size_t)p * P.tiles * RADIX;
        mark(prof, s, kStagePass);
        hipLaunchKernelGGL((k_digit_pass<KeyT, RB, BLOCK, ITEMS>), dim3(P.tiles), dim3(BLOCK), 0,
                           s, p, p * RB, (uint32_t)P.n, (KeyT*)(ws + P.o_keysA),
                           (uint32_t*)(ws + P.o_idxA), (KeyT*)(ws + P.o_keysB),
                           (uint32_t*)(ws + P.o_idxB),
                           (const uint32_t*)(ws + P.o_dbase) + (size_t)p * RADIX, look,
                           (Header*)(ws + P.o_header));
        e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

template <typename KeyT>
hipError_t Launcher<KeyT>::pack(const Plan& P, const uint32_t* next, const void* keys, char* ws,
                                hipStream_t s)
{
    switch (P.RB) {
    case 1: return launch_pack_rb<KeyT, 1>(P, next, keys, ws, s);
    case 2: return launch_pack_rb<KeyT, 2>(P, next, keys, ws, s);
    case 4: return launch_pack_rb<KeyT, 4>(P, next, keys, ws, s);
    default: return launch_pack_rb<KeyT, 8>(P, next, keys, ws, s);
    }
}

template <typename KeyT>
hipError_t Launcher<KeyT>::passes(const Plan& P, char* ws, hipStream_t s, Prof* prof)
{
    switch (P.RB) {
    case 1: return launch_passes_rb<KeyT, 1>(P, ws, s, prof);
    case 2: return launch_passes_rb<KeyT, 2>(P, ws, s, prof);
    case 4: return launch_passes_rb<KeyT, 4>(P, ws, s, prof);
    default: return launch_passes_rb<KeyT, 8>(P, ws, s, prof);
    }
}

template <typename KeyT>
hipError_t Launcher<KeyT>::walk0(const Plan& P, uint32_t head, char* ws, hipStream_t s)
{
    const LevelPlan& L = P.lv[0];
    hipLaunchKernelGGL((k_walk0<KeyT>), dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0,
                       s, (const NodeRec<KeyT>*)(ws + P.o_nodes), (uint32_t)P.n, head,
                       (uint32_t)L.n_static, (uint2*)(ws + L.o_chain_rec),
                       (Entry<KeyT>*)(ws + L.o_ent), (uint32_t*)(ws + L.o_resume),
                       (Header*)(ws + P.o_header));
    return hipGetLastError();
}

template <typename KeyT>
hipError_t Launcher<KeyT>::unchain(const Plan& P, char* ws, hipStream_t s, Prof* prof)
{
    const LevelPlan& L = P.lv[0];
    const uint64_t threads = L.n_static * 16;
    mark(prof, s, kStageUnchain);
    hipLaunchKernelGGL((k_unchain<KeyT>), dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s,
                       (const uint2*)(ws + L.o_chain_rec), (const Entry<KeyT>*)(ws + L.o_ent),
                       (uint32_t)L.n_static, (const uint32_t*)(ws + L.o_offn), (uint32_t)P.n,
                       (KeyT*)(ws + P.o_keysA), (uint32_t*)(ws + P.o_idxA),
                       (Header*)(ws + P.o_header));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    mark(prof, s, kStageWalk2);
    hipLaunchKernelGGL((k_walk2<KeyT>), dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                       (const NodeRec<KeyT>*)(ws + P.o_nodes), (const uint2*)(ws + L.o_chain_rec),
                       (const uint32_t*)(ws + L.o_resume), (uint32_t)L.n_static,
                       (const uint32_t*)(ws + L.o_offn), (uint32_t)P.n, (KeyT*)(ws + P.o_keysA),
                       (uint32_t*)(ws + P.o_idxA), (Header*)(ws + P.o_header));
    return hipGetLastError();
}

size_t entry_bytes(uint32_t key_bytes) { return key_bytes == 8 ? 16 : 8; }
size_t node_bytes(uint32_t key_bytes) { return key_bytes == 8 ? 16 : 8; }
size_t chain_cap() { return kChainCap; }

static inline void mark(Prof* prof, hipStream_t s, int32_t stage)
{
    if (!prof || prof->count >= prof->n_events)
        return;
    hipEventRecord((hipEvent_t)prof->events[prof->count], s);
    if (prof->ids)
        prof->ids[prof->count] = stage;
    prof->count++;
}

// Everything after the plan: the whole path queued on one stream.
hipError_t enqueue_sort(const Plan& P, uint32_t head, const uint32_t* next_in, uint32_t* next_out,
                        const void* keys, uint32_t* d_result, char* ws, hipStream_t s, Prof* prof)
{
    hipError_t e;
    mark(prof, s, kStageZero);
    {
        size_t words = (P.zero_end - P.o_header) / 4;
        size_t want = (words + 255) / 256;
        uint32_t blocks = (uint32_t)(want < 2048 ? want : 2048);
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, (uint32_t*)(ws + P.o_header),
                           words);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    mark(prof, s, kStagePack);
    switch (P.key_bytes) {
    case 1: e = Launcher<uint8_t>::pack(P, next_in, keys, ws, s); break;
    case 2: e = Launcher<uint16_t>::pack(P, next_in, keys, ws, s); break;
    case 4: e = Launcher<uint32_t>::pack(P, next_in, keys, ws, s); break;
    default: e = Launcher<uint64_t>::pack(P, next_in, keys, ws, s); break;
    }
    if (e != hipSuccess)
        return e;
    mark(prof, s, kStageWalk0);
    switch (P.key_bytes) {
    case 1: e = Launcher<uint8_t>::walk0(P, head, ws, s); break;
    case 2: e = Launcher<uint16_t>::walk0(P, head, ws, s); break;
    case 4: e = Launcher<uint32_t>::walk0(P, head, ws, s); break;
    default: e = Launcher<uint64_t>::walk0(P, head, ws, s); break;
    }
    if (e != hipSuccess)
        return e;
    Header* hdr = (Header*)(ws + P.o_header);
    for (int k = 1; k < P.levels; k++) {
        const LevelPlan& L = P.lv[k];
        const LevelPlan& Lp = P.lv[k - 1];
        mark(prof, s, kStageWalkUp);
        hipLaunchKernelGGL(k_walk_up, dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                           (const uint2*)(ws + Lp.o_chain_rec), (uint32_t)L.m, L.log_l,
                           (uint32_t)L.n_static, (uint2*)(ws + L.o_chain_rec), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    {
        const LevelPlan& Lt = P.lv[P.levels - 1];
        mark(prof, s, kStageBase);
        hipLaunchKernelGGL(k_base, dim3(1), dim3(kBaseThreads), 0, s,
                           (const uint2*)(ws + Lt.o_chain_rec), (uint32_t)Lt.n_static,
                           (uint32_t)P.n, (uint32_t*)(ws + Lt.o_offn), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    for (int k = P.levels - 1; k >= 1; k--) {
        const LevelPlan& L = P.lv[k];
        const LevelPlan& Lp = P.lv[k - 1];
        mark(prof, s, kStageDown);
        hipLaunchKernelGGL(k_down, dim3((uint32_t)((L.n_static + 255) / 256)), dim3(256), 0, s,
                           (const uint2*)(ws + Lp.o_chain_rec), (uint32_t)L.m, L.log_l,
                           (uint32_t)L.n_static, (const uint2*)(ws + L.o_chain_rec),
                           (const uint32_t*)(ws + L.o_offn), (uint32_t*)(ws + Lp.o_offn), hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    switch (P.key_bytes) {
    case 1: e = Launcher<uint8_t>::unchain(P, ws, s, prof); break;
    case 2: e = Launcher<uint16_t>::unchain(P, ws, s, prof); break;
    case 4: e = Launcher<uint32_t>::unchain(P, ws, s, prof); break;
    default: e = Launcher<uint64_t>::unchain(P, ws, s, prof); break;
    }
    if (e != hipSuccess)
        return e;
    switch (P.key_bytes) {
    case 1: e = Launcher<uint8_t>::passes(P, ws, s, prof); break;
    case 2: e = Launcher<uint16_t>::passes(P, ws, s, prof); break;
    case 4: e = Launcher<uint32_t>::passes(P, ws, s, prof); break;
    default: e = Launcher<uint64_t>::passes(P, ws, s, prof); break;
    }
    if (e != hipSuccess)
        return e;
    {
        uint32_t blocks = (uint32_t)((P.n + 255) / 256);
        mark(prof, s, kStageRelink);
        hipLaunchKernelGGL(k_relink, dim3(blocks), dim3(256), 0, s,
                           (const uint32_t*)(ws + P.o_idxA), (const uint32_t*)(ws + P.o_idxB),
                           (uint32_t)P.n, next_out, d_result, (const Header*)hdr);
        if ((e = hipGetLastError()) != hipSuccess)
            return e;
    }
    mark(prof, s, kStageCount);
    return hipSuccess;
}

hipError_t enqueue_empty(uint32_t* d_result, hipStream_t s)
{
    hipLaunchKernelGGL(k_empty_result, dim3(1), dim3(1), 0, s, d_result);
    return hipGetLastError();
}

}  // namespace pbit
