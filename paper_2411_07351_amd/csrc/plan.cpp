// Host-side planner for the fused-pass HIP kernels.
//
// The order tree G(W) of Alg. 1 (proof of Theorem 1) is cut into a few
// "passes".  A pass takes the Hough images of the frontier of level lin (the
// maximal subtrees of height <= lin; level 0 is the input lanes) to those of
// the frontier of level lout, entirely in LDS, one work item per
// (pass root, slope tile, position tile).  For each work item the planner
// emits a straight-line program of row entries (k = 64-position chunks):
//   load   lds[d + c] = src[row][(s0 + off + c) mod H]             c < 64 k
//   merge  lds[d + c] = lds[a + c] + lds[b + c]                      c < 64 k
//   store  dst[row][s0 + c] = lds[d + c] (+ lds[b + c])  c < min(64 k, lim), s0 + c < H
// A merge is the vector operation of Alg. 1: row t of a node is row t0 of its
// left child plus row t1 of its right child rotated by r = t - t1, with
// t_P = [t (w_P - 1)/(w - 1)] rounded half to even.  Rotation is folded into
// the LDS address of the right operand: every node keeps a window of
// positions [lo, hi) relative to the tile start, and the right child's window
// is widened by the range of r over the rows the tile needs.
//
// The last merge of a pass root is done by its stores: each store entry adds
// the two child rows on the way out, so the root's rows never pass through
// LDS (one LDS write and one read less per output element).
//
// Rows are stored with a stride rounded up to whole chunks and every entry
// runs whole chunks: the positions past a window are computed but never
// read back.  A right child carries the few positions of slack that the
// shifted whole-chunk reads of its last row need, so they stay inside it.
//
// A node's subtree depends on its width alone, so the pass roots of equal
// widths (a handful per pass) run the same programs on different lanes: each
// width is planned once, and the other roots' headers point at its entries
// with a lane base that the kernels add to every row.
#include "plan.hpp"

#include <array>

#include <algorithm>
#include <map>

namespace fht {

int64_t round_half_even(int64_t num, int64_t den)
{
    int64_t q = num / den, r = num - q * den;
    if (2 * r > den) return q + 1;
    if (2 * r < den) return q;
    return q + (q & 1);
}

int split_left(int w, int split)
{
    if (split == 0) return w / 2;
    int p = 1;
    while (2 * p < w) p <<= 1;
    return p;
}

static int ceil_log2(int w)
{
    int h = 0;
    while ((1 << h) < w) ++h;
    return h;
}

int make_tree_height(int W) { return ceil_log2(W); }

Tree make_tree(int W, int split)
{
    Tree tr;
    tr.W = W;
    tr.split = split;
    tr.nodes.reserve(2 * static_cast<size_t>(W));
    Node root;
    root.a = 0;
    root.w = W;
    root.height = ceil_log2(W);
    tr.nodes.push_back(root);
    for (size_t i = 0; i < tr.nodes.size(); ++i) {
        const Node n = tr.nodes[i];
        if (n.w <= 1) continue;
        const int w0 = split_left(n.w, split);
        Node l, r;
        l.a = n.a;
        l.w = w0;
        l.height = ceil_log2(w0);
        r.a = n.a + w0;
        r.w = n.w - w0;
        r.height = ceil_log2(n.w - w0);
        const int li = static_cast<int>(tr.nodes.size());
        tr.nodes.push_back(l);
        tr.nodes.push_back(r);
        tr.nodes[i].w0 = w0;
        tr.nodes[i].left = li;
        tr.nodes[i].right = li + 1;
    }
    return tr;
}

namespace {

int chunks_of(int width) { return (width + kChunk - 1) / kChunk; }

struct Block {
    int node;
    int ulo, uhi;     // rows of the node this tile needs (inclusive)
    int lo, hi;       // position window relative to the tile start
    int step;         // 0 = loaded, k = computed in step k
    int last;         // last step that reads it
    int lb = -1, rb = -1;
    int off = -1;     // LDS element offset
    int overrun = 0;  // positions a merge reads past the end of the last row
    int row_stride = 0;
    bool virt = false;  // computed by the stores, never held in LDS
    int width() const { return hi - lo; }
    int rows() const { return uhi - ulo + 1; }
    int stride() const { return row_stride; }
    int size() const { return virt ? 0 : rows() * stride() + overrun; }
};

struct Live { int off, size, last; };

// State shared by the tile builds of one axis plan: the child rows t0, t1 of
// every row u of every non-leaf node, computed once per distinct (w, w0) of
// the tree (rows(n)[2 u], rows(n)[2 u + 1]), and buffers reused from one
// tile to the next.
struct PlanWork {
    const Tree &tr;
    std::map<std::pair<int, int>, std::vector<int32_t>> by_width;
    std::vector<const int32_t *> by_node;
    std::vector<Block> blocks;
    std::vector<int> order, step_at;
    std::vector<Live> live;

    explicit PlanWork(const Tree &t) : tr(t), by_node(t.nodes.size(), nullptr) {}

    const int32_t *rows(int ni)
    {
        if (by_node[ni]) return by_node[ni];
        const Node &n = tr.nodes[ni];
        const int w = n.w, w0 = n.w0, w1 = w - w0;
        std::vector<int32_t> &v = by_width[{w, w0}];
        if (v.empty()) {
            v.resize(2 * static_cast<size_t>(w));
            for (int u = 0; u < w; ++u) {
                v[2 * u] = static_cast<int32_t>(round_half_even(int64_t(u) * (w0 - 1), w - 1));
                v[2 * u + 1] = static_cast<int32_t>(round_half_even(int64_t(u) * (w1 - 1), w - 1));
            }
        }
        return by_node[ni] = v.data();
    }
};

struct TileBuilder {
    const Tree &tr;
    PlanWork &work;
    int lin;
    int K;                       // chunks every entry of the tile covers
    int stride;                  // LDS row stride: K chunks plus a bank-skew pad
    std::vector<Block> &blocks;  // cleared by the caller

    int need(int ni, int ulo, int uhi, int lo, int hi)
    {
        const Node &n = tr.nodes[ni];
        const int b = static_cast<int>(blocks.size());
        blocks.push_back(Block{ni, ulo, uhi, lo, hi, 0, -1});
        blocks[b].row_stride = stride;
        if (n.height <= lin) return b;
        blocks[b].step = n.height - lin;
        const int32_t *tt = work.rows(ni);
        const int t0lo = tt[2 * ulo], t0hi = tt[2 * uhi];
        const int t1lo = tt[2 * ulo + 1], t1hi = tt[2 * uhi + 1];
        const int lb = need(n.left, t0lo, t0hi, lo, hi);
        const int rb = need(n.right, t1lo, t1hi, lo + (ulo - t1lo), hi + (uhi - t1hi));
        blocks[lb].last = blocks[b].step;
        blocks[rb].last = blocks[b].step;
        blocks[b].lb = lb;
        blocks[b].rb = rb;
        // A merge reads K whole chunks of the right child, starting up to
        // (uhi - t1hi) - (ulo - t1lo) positions into a row.
        Block &R = blocks[rb];
        const int reach = (uhi - t1hi) - (ulo - t1lo) + K * kChunk;
        R.overrun = std::max(R.overrun, reach - R.stride());
        return b;
    }
};

// The widest window (hi - lo) of the blocks TileBuilder::need would make for
// rows [ulo, uhi] of node ni with window [lo, hi), without making them.
int widest_window(const Tree &tr, PlanWork &work, int lin, int ni, int ulo, int uhi, int lo, int hi)
{
    const Node &n = tr.nodes[ni];
    int w = hi - lo;
    if (n.height <= lin) return w;
    const int32_t *tt = work.rows(ni);
    const int t0lo = tt[2 * ulo], t0hi = tt[2 * uhi];
    const int t1lo = tt[2 * ulo + 1], t1hi = tt[2 * uhi + 1];
    w = std::max(w, widest_window(tr, work, lin, n.left, t0lo, t0hi, lo, hi));
    return std::max(w, widest_window(tr, work, lin, n.right, t1lo, t1hi, lo + (ulo - t1lo),
                                     hi + (uhi - t1hi)));
}

// First-fit placement of the blocks in LDS; a block may reuse the space of
// blocks whose last reader ran in an earlier step.  Returns the footprint.
int place(std::vector<Block> &blocks, PlanWork &work)
{
    // blocks in step order, in index order within a step (a counting sort)
    std::vector<int> &order = work.order;
    int max_step = 0;
    for (const Block &b : blocks) max_step = std::max(max_step, b.step);
    std::vector<int> &at = work.step_at;
    at.assign(static_cast<size_t>(max_step) + 2, 0);
    for (const Block &b : blocks) ++at[b.step + 1];
    for (int st = 0; st <= max_step; ++st) at[st + 1] += at[st];
    order.resize(blocks.size());
    for (size_t i = 0; i < blocks.size(); ++i) order[at[blocks[i].step]++] = static_cast<int>(i);
    std::vector<Live> &live = work.live;  // kept in offset order
    live.clear();
    int top = 0;
    for (int b : order) {
        Block &blk = blocks[b];
        live.erase(std::remove_if(live.begin(), live.end(),
                                  [&](const Live &l) { return l.last < blk.step; }),
                   live.end());
        const int size = blk.size();
        int pos = 0;
        for (const Live &l : live) {
            if (l.off - pos >= size) break;
            pos = std::max(pos, l.off + l.size);
        }
        blk.off = pos;
        const auto at = std::upper_bound(live.begin(), live.end(), pos,
                                         [](int off, const Live &l) { return off < l.off; });
        live.insert(at, Live{pos, size, blk.last});
        top = std::max(top, pos + size);
    }
    return top;
}

void collect_frontier(const Tree &tr, int ni, int level, std::vector<int> *out)
{
    const Node &n = tr.nodes[ni];
    if (n.height <= level) {
        out->push_back(ni);
        return;
    }
    collect_frontier(tr, n.left, level, out);
    collect_frontier(tr, n.right, level, out);
}

// Emits one tile program for rows [ta, tb) of pass root `root`.  Every entry
// covers the same K chunks (the pass's target width); rows are stored with a
// stride of K chunks plus `pad` elements, which skews consecutive rows across
// LDS banks.
//
// Entry formats (4 ints each):
//   load   {lds row start, source row, position offset, K}; in the first
//          pass there is one per lane, in lane order
//   load-merge {lds dst, source row a, source row b, offset | r << 16}:
//          lds[dst + c] = src[a][(s0 + offset + c) mod H]
//                       + src[b][(s0 + offset + r + c) mod H]
//          (step 1 of a later pass, read from the source rows)
//   merge  {lds dst, lds src0, lds src1, K}
//   store  {lds row start, destination row, position limit, lds src1 or -1}:
//          with src1 >= 0 (every store of a program with merges) the stored
//          value is lds[start + c] + lds[src1 + c], the root's last merge
void emit_tile(const Tree &tr, PlanWork &work, int root, int ta, int tb, int lin, int S, int K,
               int pad, bool load_merge, Pass *pass)
{
    work.blocks.clear();
    TileBuilder tb_{tr, work, lin, K, K * kChunk + pad, work.blocks};
    const int rb = tb_.need(root, ta, tb - 1, 0, S);
    std::vector<Block> &bl = tb_.blocks;
    const int nsteps = std::max(0, tr.nodes[root].height - lin);
    bl[rb].last = nsteps + 1;
    bl[rb].virt = nsteps > 0;  // the stores compute it
    // With load_merge, a later pass computes step 1 straight from the source
    // rows (load-merges), so the rows only step 1 reads are never held in LDS.
    // Offsets must fit the 16-bit fields of a load-merge entry.
    bool fuse_loads = load_merge && lin > 0 && nsteps >= 2;
    for (const Block &b : bl)
        if (fuse_loads && b.step == 1 && (b.lo >= 65536 || b.hi + tr.nodes[b.node].w >= 65536))
            fuse_loads = false;
    if (fuse_loads)
        for (Block &b : bl)
            if (b.step == 0 && b.last == 1) b.virt = true;
    const int lds = place(bl, work);

    int32_t hdr[kHdrInts] = {0};
    const int first = static_cast<int>(pass->ops.size() / 4);
    auto push = [&](int d, int a, int b, int n) {
        pass->ops.push_back(d);
        pass->ops.push_back(a);
        pass->ops.push_back(b);
        pass->ops.push_back(n);
    };
    int nload = 0, load_end = 0, widest = 0;
    for (const Block &b : bl) {
        widest = std::max(widest, b.width());
        if (b.step != 0 || b.virt) continue;
        const Node &n = tr.nodes[b.node];
        for (int u = b.ulo; u <= b.uhi; ++u, ++nload) {
            push(b.off + (u - b.ulo) * b.stride(), n.a + u, b.lo, K);
            load_end = std::max(load_end, b.lo + K * kChunk);
        }
    }
    // LDS offsets of the two operands of row u of computed block b
    auto operands = [&](const Block &b, int u) {
        const Block &L = bl[b.lb], &R = bl[b.rb];
        const int32_t *tt = work.rows(b.node);
        const int t0 = tt[2 * u], t1 = tt[2 * u + 1];
        const int r = u - t1;
        return std::make_pair(L.off + (t0 - L.ulo) * L.stride() + (b.lo - L.lo),
                              R.off + (t1 - R.ulo) * R.stride() + (b.lo + r - R.lo));
    };
    int nlm = 0;
    if (fuse_loads) {
        for (const Block &b : bl) {
            if (b.step != 1) continue;
            const Node &n = tr.nodes[b.node];
            const Node &nl = tr.nodes[n.left], &nr = tr.nodes[n.right];
            const int32_t *tt = work.rows(b.node);
            for (int u = b.ulo; u <= b.uhi; ++u, ++nlm) {
                const int t0 = tt[2 * u], t1 = tt[2 * u + 1];
                const uint32_t offs = static_cast<uint32_t>(b.lo) |
                                      (static_cast<uint32_t>(u - t1) << 16);
                push(b.off + (u - b.ulo) * b.stride(), nl.a + t0, nr.a + t1,
                     static_cast<int32_t>(offs));
            }
        }
    }
    // merge steps in LDS: all but the load-merged first and the stores' last
    const int step0 = fuse_loads ? 2 : 1;
    const int lds_steps = std::max(0, nsteps - step0);
    for (int k = step0; k < step0 + lds_steps; ++k) {
        int cnt = 0;
        for (const Block &b : bl) {
            if (b.step != k) continue;
            for (int u = b.ulo; u <= b.uhi; ++u, ++cnt) {
                const auto ab = operands(b, u);
                push(b.off + (u - b.ulo) * b.stride(), ab.first, ab.second, K);
            }
        }
        hdr[kHdrStepCounts + k - step0] = cnt;
    }
    int nstore = 0;
    {
        const Block &b = bl[rb];
        const Node &n = tr.nodes[b.node];
        for (int u = b.ulo; u <= b.uhi; ++u, ++nstore) {
            if (b.virt) {
                const auto ab = operands(b, u);
                push(ab.first, n.a + u, S, ab.second);
            } else {
                push(b.off + (u - b.ulo) * b.stride(), n.a + u, S, -1);
            }
        }
    }
    hdr[kHdrFirst] = first;
    hdr[kHdrLoads] = nload;
    hdr[kHdrStores] = nstore;
    hdr[kHdrSteps] = lds_steps;
    hdr[kHdrLds] = lds;
    hdr[kHdrEntries] = static_cast<int>(pass->ops.size() / 4) - first;
    hdr[kHdrLevelIn] = lin;
    hdr[kHdrHeight] = tr.nodes[root].height;
    hdr[kHdrLoadEnd] = load_end;
    hdr[kHdrSTile] = S;
    hdr[kHdrChunks] = K;
    hdr[kHdrStoreMerge] = bl[rb].virt ? 1 : 0;
    hdr[kHdrLoadMerges] = nlm;
    pass->hdrs.insert(pass->hdrs.end(), hdr, hdr + kHdrInts);
    pass->max_lds_elems = std::max(pass->max_lds_elems, lds);
    pass->widest = std::max(pass->widest, widest);
    if (widest > K * kChunk || K > kMaxChunks) pass->fits = false;
}

// Appends a header for program `src` of the pass moved by `delta` lanes: the
// program of a root with the same width as the root of `src`.  A node's
// subtree, and so every slope table, block and LDS offset of its tiles,
// depends on its width only; lanes enter the entries only as the source rows
// of loads and load-merges and the destination rows of stores, which the
// kernels offset by the header's lane base.  The two headers share entries.
void share_tile(Pass *pass, int src, int delta)
{
    const int32_t *sh = pass->hdrs.data() + static_cast<size_t>(src) * kHdrInts;
    int32_t hdr[kHdrInts];
    std::copy(sh, sh + kHdrInts, hdr);
    hdr[kHdrLaneBase] += delta;
    pass->hdrs.insert(pass->hdrs.end(), hdr, hdr + kHdrInts);
}

// Stops early (the pass then fails the caller's checks) once a program
// outgrows `max_lds` elements or the kernels' limits.
void build_pass(const Tree &tr, PlanWork &work, int lin, int lout, int T, int S, int K,
                int pad, int H, bool load_merge, int max_lds, Pass *pass)
{
    pass->lin = lin;
    pass->lout = lout;
    pass->t_tile = T;
    pass->S = S;
    std::vector<int> roots;
    collect_frontier(tr, 0, lout, &roots);
    // first root of each width: {width, its lane offset, its first program}
    std::vector<std::array<int, 3>> made;
    for (int r : roots) {
        const int w = tr.nodes[r].w;
        pass->max_root_w = std::max(pass->max_root_w, w);
        const int tt = (T <= 0) ? w : T;
        const std::array<int, 3> *same = nullptr;
        for (const auto &m : made)
            if (m[0] == w) same = &m;
        const int prog0 = static_cast<int>(pass->hdrs.size() / kHdrInts);
        const std::array<int, 3> here{w, tr.nodes[r].a, prog0};
        for (int ta = 0, j = 0; ta < w; ta += tt, ++j) {
            const int prog = static_cast<int>(pass->hdrs.size() / kHdrInts);
            if (same) {
                share_tile(pass, (*same)[2] + j, here[1] - (*same)[1]);
            } else {
                emit_tile(tr, work, r, ta, std::min(w, ta + tt), lin, S, K, pad, load_merge, pass);
                if (!pass->fits || pass->max_lds_elems > max_lds) return;
            }
            for (int s0 = 0; s0 < H; s0 += S) {
                pass->items.push_back(prog);
                pass->items.push_back(0);
                pass->items.push_back(s0);
                pass->items.push_back(0);
            }
        }
        if (!same) made.push_back(here);
    }
}

// Builds the pass with the largest position tile whose widest window still
// fits the target width (windows are the tile plus a spread that depends on
// the slope tile only).
void build_pass_fitted(const Tree &tr, PlanWork &work, int lin, int lout, int T, int target,
                       int pad, int H, bool load_merge, int max_lds, Pass *out)
{
    // Windows are S plus a spread that does not depend on S (nor on K): take
    // the widest window of every tile for S = 16, then pick the largest S.
    std::vector<int> roots;
    collect_frontier(tr, 0, lout, &roots);
    int widest = 0;
    std::vector<int> seen;  // root widths probed (equal widths, equal windows)
    for (int r : roots) {
        const int w = tr.nodes[r].w;
        if (std::find(seen.begin(), seen.end(), w) != seen.end()) continue;
        seen.push_back(w);
        const int tt = (T <= 0) ? w : T;
        for (int ta = 0; ta < w; ta += tt)
            widest = std::max(widest, widest_window(tr, work, lin, r, ta, std::min(w, ta + tt) - 1, 0, 16));
    }
    const int spread = widest - 16;
    const int S = std::min(H, std::max(16, target - spread));
    const int K = std::max(1, chunks_of(S + spread));
    build_pass(tr, work, lin, lout, T, S, K, pad, H, load_merge, max_lds, out);
}

}  // namespace

// Widest node of the frontier of `level`.
static int frontier_width(const Tree &tr, int level)
{
    std::vector<int> roots;
    collect_frontier(tr, 0, level, &roots);
    int w = 0;
    for (int r : roots) w = std::max(w, tr.nodes[r].w);
    return w;
}

bool plan_axis(int W, int H, int split, const ElemRule &rule, const Schedule &sched,
               AxisPlan *out, std::string *err)
{
    if (W < 1 || H < 1 || (split != 0 && split != 1) || rule.narrow_bytes <= 0 ||
        rule.wide_bytes <= 0) {
        if (err) *err = "bad axis arguments";
        return false;
    }
    const Tree tr = make_tree(W, split);
    PlanWork work(tr);
    const int L = tr.nodes[0].height;
    out->W = W;
    out->H = H;
    out->split = split;
    out->passes.clear();
    int lin = 0;
    do {
        int maxlv = (lin == 0) ? std::min(sched.first_levels, kMaxFirstLevels)
                               : std::min(sched.max_levels, kMaxSteps);
        // Later passes take one more level than the schedule asks for
        // wherever that saves a whole pass (an HBM round trip of every row):
        // the remaining r levels run in the fewest passes P of at most m + 1
        // levels, and the last r - P m of them take m + 1 (r = 4: 3 + 1
        // becomes 4; r = 7: 3 + 3 + 1 becomes 3 + 4).  The extra levels go to
        // the last passes so that earlier passes keep narrow rows (16-bit
        // pairs of uint8 images while nodes are at most 257 wide) as long as
        // they can.  A pass still takes fewer levels if the LDS budget
        // requires it.
        if (lin > 0 && maxlv + 1 <= kMaxSteps) {
            const int r = L - lin;
            const int P = (r + maxlv) / (maxlv + 1);
            if (r - P * maxlv >= P) ++maxlv;  // every remaining pass needs m + 1
        }
        const int target = (lin == 0) ? sched.s_tile_first : sched.s_tile;
        bool found = false;
        Pass best;
        const int hi = std::min(L, lin + maxlv);
        const int lo = (L > lin) ? lin + 1 : lin;
        for (int lout = hi; lout >= lo && !found; --lout) {
            const int eb = rule.bytes_for(frontier_width(tr, lin), frontier_width(tr, lout));
            const int budget_elems = sched.lds_budget / eb;
            const int pad = eb == 2 ? 2 : 1;  // skew rows by one 32-bit bank
            // The first pass takes whole roots (at most 64 lanes, loaded as one
            // lane x window rectangle).
            std::vector<int> tiles;
            if (lin == 0) tiles = {0};
            else if (sched.t_tile > 0) {
                // the requested slope tile, halved until the pass fits
                for (int T = sched.t_tile; T >= 4; T /= 2) tiles.push_back(T);
                if (tiles.empty()) tiles.push_back(sched.t_tile);
            } else {
                tiles = {32, 16, 8, 4};
            }
            // Load-merges pay off where rows reach LDS through registers anyway:
            // 4-byte LDS elements are loaded straight from memory into LDS
            // (cheaper than a second load per element), others are not.
            const bool load_merge = eb != 4;
            for (int T : tiles) {
                Pass p;
                build_pass_fitted(tr, work, lin, lout, T, target, pad, H, load_merge, budget_elems, &p);
                p.elem_bytes = eb;
                for (size_t h = 0; h < p.hdrs.size(); h += kHdrInts) p.hdrs[h + kHdrElemBytes] = eb;
                if (p.fits && p.max_lds_elems <= budget_elems) {
                    best = std::move(p);
                    found = true;
                    break;
                }
            }
        }
        if (!found) {
            if (err) *err = "no pass fits the LDS budget";
            return false;
        }
        lin = best.lout;
        out->passes.push_back(std::move(best));
    } while (lin < L);
    return true;
}

void retile_items(AxisPlan *ax, int H)
{
    ax->H = H;
    for (Pass &ps : ax->passes) {
        const int nprog = static_cast<int>(ps.hdrs.size() / kHdrInts);
        ps.items.clear();
        ps.items.reserve(static_cast<size_t>(nprog) * ((H + ps.S - 1) / ps.S) * 4);
        for (int prog = 0; prog < nprog; ++prog) {
            for (int s0 = 0; s0 < H; s0 += ps.S) {
                ps.items.push_back(prog);
                ps.items.push_back(0);
                ps.items.push_back(s0);
                ps.items.push_back(0);
            }
        }
    }
}

// Adjoint steps.  The forward merge of a node of width w into children of
// widths w0, w1 is J[t] = J0[t0(t)] + Rotate(J1[t1(t)], t - t1(t)); its adjoint
// gives left-child row u the sum of the parent rows t with t0(t) = u, and
// right-child row u the sum of the parent rows t with t1(t) = u, each rotated
// back by t - u.  Both preimages are contiguous ranges of t because t0 and t1
// are non-decreasing in t with steps of at most one, and neither is empty.
AdjointAxis plan_adjoint_axis(int W, int split)
{
    AdjointAxis ax;
    ax.W = W;
    const Tree tr = make_tree(W, split);
    ax.levels = tr.nodes[0].height;
    ax.tasks.assign(static_cast<size_t>(ax.levels) * W * 4, 0);
    for (int k = 0; k < ax.levels; ++k) {
        const int level = ax.levels - k;
        int32_t *task = ax.tasks.data() + static_cast<size_t>(k) * W * 4;
        std::vector<int> nodes;
        collect_frontier(tr, 0, level, &nodes);
        for (int ni : nodes) {
            const Node &n = tr.nodes[ni];
            if (n.height < level) {  // also in the next frontier: passed through
                for (int u = 0; u < n.w; ++u) {
                    int32_t *e = task + 4 * (n.a + u);
                    e[0] = n.a + u; e[1] = 1; e[2] = 0; e[3] = 0;
                }
                continue;
            }
            const int w = n.w, w0 = n.w0, w1 = w - w0;
            // preimages, walking t upwards
            int t = 0;
            for (int u = 0; u < w0; ++u) {
                const int lo = t;
                while (t < w && round_half_even(int64_t(t) * (w0 - 1), w - 1) == u) ++t;
                int32_t *e = task + 4 * (n.a + u);
                e[0] = n.a + lo; e[1] = t - lo; e[2] = 0; e[3] = 0;
            }
            t = 0;
            for (int u = 0; u < w1; ++u) {
                const int lo = t;
                while (t < w && round_half_even(int64_t(t) * (w1 - 1), w - 1) == u) ++t;
                int32_t *e = task + 4 * (n.a + w0 + u);
                e[0] = n.a + lo; e[1] = t - lo; e[2] = lo - u; e[3] = 1;
            }
        }
    }
    return ax;
}

std::vector<AdjointPass> fuse_adjoint(const AdjointAxis &ax, int H, int max_levels)
{
    std::vector<AdjointPass> passes;
    const int W = ax.W;
    max_levels = std::max(1, max_levels);
    for (int k0 = 0; k0 < ax.levels; k0 += max_levels) {
        const int k1 = std::min(ax.levels, k0 + max_levels);
        AdjointPass p;
        p.levels = k1 - k0;
        p.offs.reserve(static_cast<size_t>(W) + 1);
        std::vector<int64_t> cur, nxt;  // (row, shift) pairs, shifts mod H
        for (int x = 0; x < W; ++x) {
            p.offs.push_back(static_cast<int32_t>(p.terms.size() / 2));
            cur.assign({x, 0});
            // walk up from the last step of the pass to its first
            for (int k = k1 - 1; k >= k0; --k) {
                const int32_t *task = ax.tasks.data() + static_cast<size_t>(k) * W * 4;
                nxt.clear();
                for (size_t i = 0; i < cur.size(); i += 2) {
                    const int32_t *e = task + 4 * cur[i];
                    for (int j = 0; j < e[1]; ++j) {
                        nxt.push_back(e[0] + j);
                        nxt.push_back((cur[i + 1] + (e[3] ? e[2] + j : 0)) % H);
                    }
                }
                cur.swap(nxt);
            }
            for (int64_t v : cur) p.terms.push_back(static_cast<int32_t>(v));
        }
        p.offs.push_back(static_cast<int32_t>(p.terms.size() / 2));
        passes.push_back(std::move(p));
    }
    return passes;
}

}  // namespace fht
