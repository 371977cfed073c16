// Interaction lists and near-field lists (Sec. 4 notation table; Definition of
// HODLR3D admissibility; Algorithms 1 and 2).
//
// For a box t at level l >= 1 with parent p, the clan is the set of children
// of p and of p's face- and edge-sharing neighbours, minus t itself.  The
// interaction list keeps the clan members that share at most a vertex with t
// (relation V or W); each such pair becomes one low-rank block.  At the leaf
// level the near list of t is t itself plus its E and F neighbours.  Empty
// boxes create no blocks.  Lists are emitted in ascending Morton order of the
// partner box: the parent neighbours are sorted once and their children
// follow in order, so no per-block sort is needed.
#include "h3d_internal.hpp"

namespace h3d {

namespace {

enum { kRelSelf = 0, kRelF = 1, kRelE = 2, kRelV = 3, kRelW = 4 };

struct Levels {
    int64_t base[kMaxLevels + 1];  // first global box id of level l (levels 1..L)
    int L;
};

__device__ __forceinline__ uint64_t spread3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint64_t v) {
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10c30c30c30c30c3ull;
    v = (v ^ (v >> 4)) & 0x100f00f00f00f00full;
    v = (v ^ (v >> 8)) & 0x1f0000ff0000ffull;
    v = (v ^ (v >> 16)) & 0x1f00000000ffffull;
    v = (v ^ (v >> 32)) & 0x1fffffull;
    return uint32_t(v);
}

__device__ __forceinline__ uint64_t encode3(int x, int y, int z) {
    return (spread3(uint64_t(x)) << 2) | (spread3(uint64_t(y)) << 1) | spread3(uint64_t(z));
}

__device__ __forceinline__ void decode3(uint64_t code, int &x, int &y, int &z) {
    x = int(compact3(code >> 2));
    y = int(compact3(code >> 1));
    z = int(compact3(code));
}

__device__ __forceinline__ int relation(int ax, int ay, int az, int bx, int by, int bz) {
    int dx = abs(ax - bx), dy = abs(ay - by), dz = abs(az - bz);
    int m = max(dx, max(dy, dz));
    if (m == 0)
        return kRelSelf;
    if (m >= 2)
        return kRelW;
    int s = dx + dy + dz;
    return s == 3 ? kRelV : (s == 2 ? kRelE : kRelF);
}

struct BoxRange {
    int32_t start, count;
};

__device__ __forceinline__ BoxRange box_range(const int32_t *__restrict__ leaf_off, int L, int l,
                                             int64_t b) {
    const int sh = 3 * (L - l);
    int32_t a = leaf_off[b << sh];
    int32_t e = leaf_off[(b + 1) << sh];
    return {a, e - a};
}

__device__ __forceinline__ void level_of(const Levels &lv, int64_t g, int &l, int64_t &t) {
    l = 1;
    while (l < lv.L && g >= lv.base[l + 1])
        ++l;
    t = g - lv.base[l];
}

// Count (fill == 0) or write (fill == 1) the interaction list of every box.
__global__ void k_far_lists(Levels lv, const int32_t *__restrict__ leaf_off, int fill,
                            int64_t *__restrict__ cnt_or_begin, int32_t *__restrict__ blk_t,
                            int32_t *__restrict__ blk_s, int32_t *__restrict__ blk_toff,
                            int32_t *__restrict__ blk_m, int32_t *__restrict__ blk_soff,
                            int32_t *__restrict__ blk_n) {
    const int64_t g = lv.base[1] + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= lv.base[lv.L + 1])
        return;
    int l;
    int64_t t;
    level_of(lv, g, l, t);
    const BoxRange tr = box_range(leaf_off, lv.L, l, t);
    if (tr.count == 0) {
        if (!fill)
            cnt_or_begin[g] = 0;
        return;
    }
    int tx, ty, tz;
    decode3(uint64_t(t), tx, ty, tz);
    const int px = tx >> 1, py = ty >> 1, pz = tz >> 1;
    const int np = 1 << (l - 1);
    // parent and its E/F neighbours, ascending Morton code
    uint32_t q[19];
    int nq = 0;
    for (int ax = px - 1; ax <= px + 1; ++ax)
        for (int ay = py - 1; ay <= py + 1; ++ay)
            for (int az = pz - 1; az <= pz + 1; ++az) {
                if (ax < 0 || ay < 0 || az < 0 || ax >= np || ay >= np || az >= np)
                    continue;
                if (relation(px, py, pz, ax, ay, az) == kRelV)
                    continue;
                uint32_t code = uint32_t(encode3(ax, ay, az));
                int k = nq++;
                while (k > 0 && q[k - 1] > code) {
                    q[k] = q[k - 1];
                    --k;
                }
                q[k] = code;
            }
    int64_t out = fill ? cnt_or_begin[g] : 0;
    int64_t c = 0;
    for (int a = 0; a < nq; ++a)
        for (int ch = 0; ch < 8; ++ch) {
            const int64_t s = int64_t(q[a]) * 8 + ch;
            if (s == t)
                continue;
            const BoxRange sr = box_range(leaf_off, lv.L, l, s);
            if (sr.count == 0)
                continue;
            int sx, sy, sz;
            decode3(uint64_t(s), sx, sy, sz);
            const int rel = relation(tx, ty, tz, sx, sy, sz);
            if (rel != kRelV && rel != kRelW)
                continue;
            if (fill) {
                const int64_t b = out + c;
                blk_t[b] = int32_t(t);
                blk_s[b] = int32_t(s);
                blk_toff[b] = tr.start;
                blk_m[b] = tr.count;
                blk_soff[b] = sr.start;
                blk_n[b] = sr.count;
            }
            ++c;
        }
    if (!fill)
        cnt_or_begin[g] = c;
}

// Near list of each leaf: itself and its E and F neighbours, ascending code.
__global__ void k_near_lists(int L, const int32_t *__restrict__ leaf_off, int fill,
                             int32_t *__restrict__ cnt_or_ptr, int32_t *__restrict__ near_s,
                             int8_t *__restrict__ near_rel) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nleaf = int64_t(1) << (3 * L);
    if (t >= nleaf)
        return;
    if (leaf_off[t + 1] == leaf_off[t]) {
        if (!fill)
            cnt_or_ptr[t] = 0;
        return;
    }
    int tx, ty, tz;
    decode3(uint64_t(t), tx, ty, tz);
    const int nb = 1 << L;
    uint32_t q[19];
    int8_t r[19];
    int nq = 0;
    for (int ax = tx - 1; ax <= tx + 1; ++ax)
        for (int ay = ty - 1; ay <= ty + 1; ++ay)
            for (int az = tz - 1; az <= tz + 1; ++az) {
                if (ax < 0 || ay < 0 || az < 0 || ax >= nb || ay >= nb || az >= nb)
                    continue;
                const int rel = relation(tx, ty, tz, ax, ay, az);
                if (rel == kRelV)
                    continue;
                const uint32_t code = uint32_t(encode3(ax, ay, az));
                if (leaf_off[code + 1] == leaf_off[code])
                    continue;
                int k = nq++;
                while (k > 0 && q[k - 1] > code) {
                    q[k] = q[k - 1];
                    r[k] = r[k - 1];
                    --k;
                }
                q[k] = code;
                r[k] = int8_t(rel);
            }
    if (!fill) {
        cnt_or_ptr[t] = nq;
        return;
    }
    const int32_t out = cnt_or_ptr[t];
    for (int a = 0; a < nq; ++a) {
        near_s[out + a] = int32_t(q[a]);
        near_rel[out + a] = r[a];
    }
}

// Blocks grouped by source box.  The relation is symmetric, so the source
// group of box a has the same size and offsets as its target group, and its
// i-th entry is the block (t', a) with t' the i-th partner of a.
__global__ void k_src_groups(Levels lv, int64_t nfar, const int64_t *__restrict__ tgt_begin,
                             const int32_t *__restrict__ blk_t, const int32_t *__restrict__ blk_s,
                             const int64_t *__restrict__ lvl_blk, int64_t *__restrict__ src_blk,
                             unsigned int *__restrict__ missing) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= nfar)
        return;
    int l = 1;
    while (l < lv.L && e >= lvl_blk[l + 1])
        ++l;
    const int32_t a = blk_t[e];       // the source box of the wanted block
    const int32_t tp = blk_s[e];      // its target box
    const int64_t g = lv.base[l] + tp;
    int64_t lo = tgt_begin[g], hi = tgt_begin[g + 1];
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (blk_s[mid] < a)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < tgt_begin[g + 1] && blk_s[lo] == a) {
        src_blk[e] = lo;
    } else {
        src_blk[e] = e;  // never happens for symmetric lists; reported to the host
        atomicAdd(missing, 1u);
    }
}

__global__ void k_near_pairs(int64_t nleaf, const int32_t *__restrict__ leaf_off,
                             const int32_t *__restrict__ near_ptr, const int32_t *__restrict__ near_s,
                             unsigned long long *__restrict__ out) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= nleaf)
        return;
    const unsigned long long m = unsigned(leaf_off[t + 1] - leaf_off[t]);
    unsigned long long acc = 0;
    for (int32_t e = near_ptr[t]; e < near_ptr[t + 1]; ++e) {
        const int32_t sb = near_s[e];
        acc += m * unsigned(leaf_off[sb + 1] - leaf_off[sb]);
    }
    if (acc)
        atomicAdd(out, acc);
}

}  // namespace

// kernel evaluations of one near-field pass: sum over near leaf pairs of m n
void near_pair_count(Plan &P, hipStream_t s) {
    const int64_t nleaf = pow8(P.L);
    unsigned long long *d = P.mem.alloc_n<unsigned long long>(1);
    H3D_HIP(hipMemsetAsync(d, 0, sizeof(unsigned long long), s));
    k_near_pairs<<<grid_for(nleaf, 256), 256, 0, s>>>(nleaf, P.leaf_off, P.near_ptr, P.near_s, d);
    H3D_LAUNCH_CHECK();
    unsigned long long h = 0;
    to_host(&h, d, 1, s);
    P.mem.release(d);
    P.stats.near_pair_evals = int64_t(h);
}

void lists_build(Plan &P, hipStream_t s) {
    const int L = P.L;
    Levels lv{};
    lv.L = L;
    int64_t acc = 0;
    for (int l = 1; l <= L; ++l) {
        lv.base[l] = acc;
        P.box_base[l] = acc;
        acc += pow8(l);
    }
    lv.base[L + 1 <= kMaxLevels ? L + 1 : kMaxLevels] = acc;
    if (L + 1 <= kMaxLevels)
        P.box_base[L + 1] = acc;
    P.nbox_all = acc;

    // mean / max box size per level (host, from the leaf offsets)
    for (int l = 0; l <= L; ++l) {
        int64_t nb = pow8(l), nonempty = 0, mx = 0;
        int sh = 3 * (L - l);
        for (int64_t b = 0; b < nb; ++b) {
            int64_t c = int64_t(P.h_leaf_off[size_t((b + 1) << sh)]) - P.h_leaf_off[size_t(b << sh)];
            if (c > 0)
                ++nonempty;
            mx = std::max(mx, c);
        }
        P.mean_box[l] = nonempty ? int(P.n / nonempty) : 0;
        P.max_box[l] = int(mx);
    }

    // far blocks: count, scan, fill
    P.tgt_begin = P.mem.alloc_n<int64_t>(acc + 1);
    if (L >= 1) {
        H3D_HIP(hipMemsetAsync(P.tgt_begin + acc, 0, sizeof(int64_t), s));
        k_far_lists<<<grid_for(acc, 128), 128, 0, s>>>(lv, P.leaf_off, 0, P.tgt_begin, nullptr,
                                                       nullptr, nullptr, nullptr, nullptr,
                                                       nullptr);
        H3D_LAUNCH_CHECK();
        P.nfar = scan_exclusive_i64(P, P.tgt_begin, P.tgt_begin, acc + 1, s);
    } else {
        P.nfar = 0;
    }
    const int64_t nf = P.nfar;
    P.blk_t = P.mem.alloc_n<int32_t>(nf);
    P.blk_s = P.mem.alloc_n<int32_t>(nf);
    P.blk_toff = P.mem.alloc_n<int32_t>(nf);
    P.blk_m = P.mem.alloc_n<int32_t>(nf);
    P.blk_soff = P.mem.alloc_n<int32_t>(nf);
    P.blk_n = P.mem.alloc_n<int32_t>(nf);
    if (nf > 0) {
        k_far_lists<<<grid_for(acc, 128), 128, 0, s>>>(lv, P.leaf_off, 1, P.tgt_begin, P.blk_t,
                                                       P.blk_s, P.blk_toff, P.blk_m, P.blk_soff,
                                                       P.blk_n);
        H3D_LAUNCH_CHECK();
    }
    // level ranges of the block table
    for (int l = 1; l <= L; ++l) {
        int64_t v = 0;
        to_host(&v, P.tgt_begin + P.box_base[l], 1, s);
        P.lvl_blk[l] = v;
    }
    for (int l = L + 1; l <= kMaxLevels; ++l)
        P.lvl_blk[l] = nf;
    P.lvl_blk[0] = 0;

    // source grouping for the adjoint
    P.src_blk = P.mem.alloc_n<int64_t>(nf);
    if (nf > 0) {
        int64_t *d_lvl = P.mem.alloc_n<int64_t>(kMaxLevels + 1);
        unsigned int *missing = P.mem.alloc_n<unsigned int>(1);
        H3D_HIP(hipMemsetAsync(missing, 0, sizeof(unsigned int), s));
        H3D_HIP(hipMemcpyAsync(d_lvl, P.lvl_blk, sizeof(int64_t) * (kMaxLevels + 1),
                               hipMemcpyHostToDevice, s));
        k_src_groups<<<grid_for(nf, 256), 256, 0, s>>>(lv, nf, P.tgt_begin, P.blk_t, P.blk_s,
                                                       d_lvl, P.src_blk, missing);
        H3D_LAUNCH_CHECK();
        unsigned int h_missing = 0;
        to_host(&h_missing, missing, 1, s);
        P.mem.release(d_lvl);
        P.mem.release(missing);
        if (h_missing)
            fail(H3D_EDEVICE, "interaction lists are not symmetric (" + std::to_string(h_missing) +
                                  " blocks without a transposed partner)");
    }

    // near pairs
    const int64_t nleaf = pow8(L);
    P.near_ptr = P.mem.alloc_n<int32_t>(nleaf + 1);
    H3D_HIP(hipMemsetAsync(P.near_ptr + nleaf, 0, sizeof(int32_t), s));
    k_near_lists<<<grid_for(nleaf, 128), 128, 0, s>>>(L, P.leaf_off, 0, P.near_ptr, nullptr,
                                                      nullptr);
    H3D_LAUNCH_CHECK();
    scan_exclusive_i32_nototal(P, P.near_ptr, P.near_ptr, nleaf + 1, s);
    int32_t nn = 0;
    to_host(&nn, P.near_ptr + nleaf, 1, s);
    P.nnear = nn;
    P.near_s = P.mem.alloc_n<int32_t>(nn);
    P.near_rel = P.mem.alloc_n<int8_t>(nn);
    k_near_lists<<<grid_for(nleaf, 128), 128, 0, s>>>(L, P.leaf_off, 1, P.near_ptr, P.near_s,
                                                      P.near_rel);
    H3D_LAUNCH_CHECK();
    H3D_HIP(hipStreamSynchronize(s));
}

}  // namespace h3d
