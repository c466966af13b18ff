// hsga_tree.cpp -- host formatting of a reconstructed tree (the output of
// hstrat_phylo_tree_ex / ga_phylo_tree) as canonical Newick text.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "hsga_host.hpp"

using namespace hsga_host;

namespace {
constexpr uint32_t kRoot = 0xffffffffu, kNotNode = 0xfffffffeu;
}

extern "C" {

int hstrat_phylo_newick(uint32_t n, uint32_t T, const uint32_t* leaf_parent,
                        const uint32_t* node_parent, const uint32_t* node_time, char* text,
                        size_t cap, size_t* length) {
    if (n == 0 || !leaf_parent || !length || (n > 1 && (!node_parent || !node_time)))
        return fail(GA_EINVAL, "NULL argument or n = 0");
    std::string out;
    if (n == 1) {
        out = "0;";
    } else {
        const uint32_t m = n - 1;              // boundaries; node ids are boundary indices
        // children lists: entries >= 0 are nodes (boundary b), < 0 leaves (-1 - a)
        std::vector<std::vector<int64_t>> kids(m);
        uint32_t root = kRoot;
        for (uint32_t b = 0; b < m; ++b) {
            const uint32_t p = node_parent[b];
            if (p == kNotNode) continue;
            if (p == kRoot) {
                if (root != kRoot) return fail(GA_EINVAL, "two roots");
                root = b;
            } else if (p < m) {
                kids[p].push_back((int64_t)b);
            } else {
                return fail(GA_EINVAL, "node parent out of range");
            }
        }
        if (root == kRoot) return fail(GA_EINVAL, "no root");
        for (uint32_t a = 0; a < n; ++a) {
            if (leaf_parent[a] >= m) return fail(GA_EINVAL, "leaf parent out of range");
            kids[leaf_parent[a]].push_back(-1 - (int64_t)a);
        }
        // smallest leaf below each node, children before parents (post-order)
        std::vector<uint32_t> least(m, kRoot);
        std::vector<uint32_t> order;
        order.reserve(m);
        std::vector<uint32_t> stack{root};
        while (!stack.empty()) {
            const uint32_t v = stack.back();
            stack.pop_back();
            order.push_back(v);
            for (int64_t c : kids[v])
                if (c >= 0) stack.push_back((uint32_t)c);
        }
        // one tree: every node reached from the root (nodes in a detached
        // cycle are not), every leaf hanging from a reached node, and no
        // branch of negative length
        std::vector<uint32_t> up(m, kRoot);
        size_t nodes = 0;
        for (uint32_t b = 0; b < m; ++b) nodes += node_parent[b] != kNotNode ? 1 : 0;
        if (order.size() != nodes) return fail(GA_EINVAL, "node parents do not form one tree");
        for (uint32_t v : order)
            for (int64_t c : kids[v])
                if (c >= 0) up[(uint32_t)c] = v;
        for (uint32_t v : order) {
            if (v != root && node_time[v] < node_time[up[v]])
                return fail(GA_EINVAL, "a node older than its parent");
            if (kids[v].empty() && std::none_of(leaf_parent, leaf_parent + n,
                                                [v](uint32_t p) { return p == v; }))
                return fail(GA_EINVAL, "a node with nothing below it");
        }
        for (uint32_t a = 0; a < n; ++a) {
            const uint32_t p = leaf_parent[a];
            if (node_parent[p] == kNotNode) return fail(GA_EINVAL, "leaf parent names no node");
            if (T < node_time[p]) return fail(GA_EINVAL, "a node younger than the leaves");
        }
        for (auto it = order.rbegin(); it != order.rend(); ++it) {
            uint32_t lv = kRoot;
            for (int64_t c : kids[*it])
                lv = std::min(lv, c >= 0 ? least[(uint32_t)c] : (uint32_t)(-1 - c));
            least[*it] = lv;
        }
        auto key = [&](int64_t c) { return c >= 0 ? least[(uint32_t)c] : (uint32_t)(-1 - c); };
        for (uint32_t v : order)
            std::sort(kids[v].begin(), kids[v].end(),
                      [&](int64_t x, int64_t y) { return key(x) < key(y); });
        // emit: a frame is (node, next child); a child's branch length is
        // its time (T for a leaf) less its parent's time
        struct Frame { uint32_t v; size_t next; };
        std::vector<Frame> frames{{root, 0}};
        out += '(';
        while (!frames.empty()) {
            Frame& f = frames.back();
            if (f.next == kids[f.v].size()) {
                out += ')';
                const uint32_t v = f.v;
                frames.pop_back();
                if (!frames.empty())
                    out += ':' + std::to_string(node_time[v] - node_time[frames.back().v]);
                continue;
            }
            const int64_t c = kids[f.v][f.next++];
            if (f.next > 1) out += ',';
            if (c < 0) {
                out += std::to_string(-1 - c) + ':' + std::to_string(T - node_time[f.v]);
            } else {
                frames.push_back({(uint32_t)c, 0});
                out += '(';
            }
        }
        out += ';';
    }
    *length = out.size();
    if (text) {
        if (cap < out.size() + 1) return fail(GA_ENOMEM, "text buffer too small");
        std::memcpy(text, out.c_str(), out.size() + 1);
    }
    return GA_OK;
}

}  // extern "C"
