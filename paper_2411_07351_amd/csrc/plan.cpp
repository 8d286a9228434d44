// Host-side planner for the fused-pass HIP kernels.
//
// The order tree G(W) of Alg. 1 (proof of Theorem 1) is cut into a few
// "passes".  A pass takes the Hough images of the frontier of level lin (the
// maximal subtrees of height <= lin; level 0 is the input lanes) to those of
// the frontier of level lout, entirely in LDS, one work item per
// (pass root, slope tile, position tile).  For each work item the planner
// emits a straight-line program of row operations:
//   load   lds[d + c]  = src[row][(s0 + off + c) mod H]          c < count
//   merge  lds[d + c]  = lds[a + c] + lds[b + c]                   c < count
//   store  dst[row][s0 + c] = lds[d + c]                           c < count, s0 + c < H
// A merge is the vector operation of Alg. 1: row t of a node is row t0 of its
// left child plus row t1 of its right child rotated by r = t - t1, with
// t_P = [t (w_P - 1)/(w - 1)] rounded half to even.  Rotation is folded into
// the LDS address of the right operand: every node stores a window of
// positions [lo, hi) relative to the tile start, and the right child's window
// is widened by the range of r over the rows the tile needs.
#include "plan.hpp"

#include <algorithm>
#include <numeric>

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

struct Block {
    int node;
    int ulo, uhi;     // rows of the node this tile needs (inclusive)
    int lo, hi;       // position window relative to the tile start
    int step;         // 0 = loaded, k = computed in step k
    int last;         // last step that reads it
    int lb = -1, rb = -1;
    int off = -1;     // LDS element offset
    int width() const { return hi - lo; }
    int rows() const { return uhi - ulo + 1; }
};

struct TileBuilder {
    const Tree &tr;
    int lin;
    std::vector<Block> blocks;

    int need(int ni, int ulo, int uhi, int lo, int hi)
    {
        const Node &n = tr.nodes[ni];
        const int b = static_cast<int>(blocks.size());
        blocks.push_back(Block{ni, ulo, uhi, lo, hi, 0, -1});
        if (n.height <= lin) return b;
        blocks[b].step = n.height - lin;
        const int w = n.w, w0 = n.w0, w1 = w - w0;
        const int t0lo = static_cast<int>(round_half_even(int64_t(ulo) * (w0 - 1), w - 1));
        const int t0hi = static_cast<int>(round_half_even(int64_t(uhi) * (w0 - 1), w - 1));
        const int t1lo = static_cast<int>(round_half_even(int64_t(ulo) * (w1 - 1), w - 1));
        const int t1hi = static_cast<int>(round_half_even(int64_t(uhi) * (w1 - 1), w - 1));
        const int lb = need(n.left, t0lo, t0hi, lo, hi);
        const int rb = need(n.right, t1lo, t1hi, lo + (ulo - t1lo), hi + (uhi - t1hi));
        blocks[lb].last = blocks[b].step;
        blocks[rb].last = blocks[b].step;
        blocks[b].lb = lb;
        blocks[b].rb = rb;
        return b;
    }
};

// First-fit placement of the blocks in LDS; a block may reuse the space of
// blocks whose last reader ran in an earlier step.  Returns the footprint.
int place(std::vector<Block> &blocks)
{
    std::vector<int> order(blocks.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return blocks[x].step < blocks[y].step; });
    struct Live { int off, size, last; };
    std::vector<Live> live;
    int top = 0;
    for (int b : order) {
        Block &blk = blocks[b];
        live.erase(std::remove_if(live.begin(), live.end(),
                                  [&](const Live &l) { return l.last < blk.step; }),
                   live.end());
        std::sort(live.begin(), live.end(), [](const Live &x, const Live &y) { return x.off < y.off; });
        const int size = blk.rows() * blk.width();
        int pos = 0;
        for (const Live &l : live) {
            if (l.off - pos >= size) break;
            pos = std::max(pos, l.off + l.size);
        }
        blk.off = pos;
        live.push_back(Live{pos, size, blk.last});
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

// Emits one tile program for rows [ta, tb) of pass root `root`.
void emit_tile(const Tree &tr, int root, int ta, int tb, int lin, int S, Pass *pass)
{
    TileBuilder tb_{tr, lin, {}};
    const int rb = tb_.need(root, ta, tb - 1, 0, S);
    std::vector<Block> &bl = tb_.blocks;
    const int nsteps = std::max(0, tr.nodes[root].height - lin);
    bl[rb].last = nsteps + 1;
    const int lds = place(bl);

    int32_t hdr[kHdrInts] = {0};
    const int first = static_cast<int>(pass->ops.size() / 4);
    auto push = [&](int d, int a, int b, int n) {
        pass->ops.push_back(d);
        pass->ops.push_back(a);
        pass->ops.push_back(b);
        pass->ops.push_back(n);
    };
    int nload = 0;
    for (const Block &b : bl) {
        if (b.step != 0) continue;
        const Node &n = tr.nodes[b.node];
        for (int u = b.ulo; u <= b.uhi; ++u, ++nload)
            push(b.off + (u - b.ulo) * b.width(), n.a + u, b.lo, b.width());
    }
    for (int k = 1; k <= nsteps; ++k) {
        int cnt = 0;
        for (const Block &b : bl) {
            if (b.step != k) continue;
            const Node &n = tr.nodes[b.node];
            const Block &L = bl[b.lb], &R = bl[b.rb];
            const int w = n.w, w0 = n.w0, w1 = w - w0;
            for (int u = b.ulo; u <= b.uhi; ++u, ++cnt) {
                const int t0 = static_cast<int>(round_half_even(int64_t(u) * (w0 - 1), w - 1));
                const int t1 = static_cast<int>(round_half_even(int64_t(u) * (w1 - 1), w - 1));
                const int r = u - t1;
                push(b.off + (u - b.ulo) * b.width(),
                     L.off + (t0 - L.ulo) * L.width() + (b.lo - L.lo),
                     R.off + (t1 - R.ulo) * R.width() + (b.lo + r - R.lo),
                     b.width());
            }
        }
        hdr[8 + k - 1] = cnt;
    }
    int nstore = 0;
    {
        const Block &b = bl[rb];
        const Node &n = tr.nodes[b.node];
        for (int u = b.ulo; u <= b.uhi; ++u, ++nstore)
            push(b.off + (u - b.ulo) * b.width(), n.a + u, 0, b.width());
    }
    hdr[0] = first;
    hdr[1] = nload;
    hdr[2] = nstore;
    hdr[3] = nsteps;
    hdr[4] = lds;
    hdr[5] = static_cast<int>(pass->ops.size() / 4) - first;
    hdr[6] = lin;
    hdr[7] = tr.nodes[root].height;
    pass->hdrs.insert(pass->hdrs.end(), hdr, hdr + kHdrInts);
    pass->max_lds_elems = std::max(pass->max_lds_elems, lds);
}

bool build_pass(const Tree &tr, int lin, int lout, int T, int S, int H, Pass *pass)
{
    pass->lin = lin;
    pass->lout = lout;
    pass->t_tile = T;
    std::vector<int> roots;
    collect_frontier(tr, 0, lout, &roots);
    for (int r : roots) {
        const int w = tr.nodes[r].w;
        const int tt = (T <= 0) ? w : T;
        for (int ta = 0; ta < w; ta += tt) {
            const int prog = static_cast<int>(pass->hdrs.size() / kHdrInts);
            emit_tile(tr, r, ta, std::min(w, ta + tt), lin, S, pass);
            for (int s0 = 0; s0 < H; s0 += S) {
                pass->items.push_back(prog);
                pass->items.push_back(0);
                pass->items.push_back(s0);
                pass->items.push_back(0);
            }
        }
    }
    return true;
}

}  // namespace

bool plan_axis(int W, int H, int split, int elem_bytes, const Schedule &sched,
               AxisPlan *out, std::string *err)
{
    if (W < 1 || H < 1 || (split != 0 && split != 1) || elem_bytes <= 0) {
        if (err) *err = "bad axis arguments";
        return false;
    }
    const Tree tr = make_tree(W, split);
    const int L = tr.nodes[0].height;
    out->W = W;
    out->H = H;
    out->split = split;
    out->S = std::min(sched.s_tile, (H + 15) / 16 * 16);
    out->passes.clear();
    const int budget_elems = sched.lds_budget / elem_bytes;
    int lin = 0;
    do {
        const int maxlv = (lin == 0) ? sched.first_levels : sched.max_levels;
        bool found = false;
        Pass best;
        const int hi = std::min(L, lin + maxlv);
        const int lo = (L > lin) ? lin + 1 : lin;
        for (int lout = hi; lout >= lo && !found; --lout) {
            std::vector<int> tiles;
            if (sched.t_tile > 0) tiles = {sched.t_tile};
            else tiles = {0, 64, 32, 16, 8, 4};
            for (int T : tiles) {
                Pass p;
                build_pass(tr, lin, lout, T, out->S, H, &p);
                if (p.max_lds_elems <= budget_elems) {
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

}  // namespace fht
