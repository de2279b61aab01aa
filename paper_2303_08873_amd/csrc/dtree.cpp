// Decision-tree variant classifier -- the paper's own adaptation model
// (Sec. 3.1 model_type "dtree"; depth 2 is its default and the only model
// evaluated in Sec. 4).  Trained on the host from the profile database:
// one sample per distinct feature tuple, labelled with its fastest variant
// (median time per variant, ties to the lowest id) as Apollo labels its
// records (Sec. 2).  CART with Gini impurity: a node splits on the feature
// and threshold that maximise sum_children sum_k c_k^2 / n_child (equivalent
// to the lowest weighted Gini impurity; compared exactly as rationals),
// thresholds halfway between consecutive
// distinct values, ties to the lower feature index, then the lower
// threshold; a node stops at the maximum depth or when it is pure.  Leaves
// keep their class counts, so a masked variant can be skipped.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "internal.h"

namespace ao {

namespace {

struct Sample {
    float f[AO_MAX_FEATURES];
    int label;
};

int build(std::vector<DTree::Node>& nodes, std::vector<Sample*>& s, int depth, int max_depth,
          int num_classes) {
    DTree::Node node;
    node.counts.assign(num_classes, 0);
    for (const Sample* p : s) node.counts[p->label] += 1;
    int distinct = 0;
    for (int c : node.counts) distinct += c > 0;
    const int id = (int)nodes.size();
    nodes.push_back(node);
    if (depth >= max_depth || distinct <= 1 || s.size() < 2) return id;
    // score of a split = (sl*nr + sr*nl) / (nl*nr), compared exactly in
    // integers so that ties resolve the same way on every machine
    __int128 best_num = -1, best_den = 1;
    int best_f = -1;
    double best_t = 0.0;
    std::vector<int> left(num_classes), right(num_classes);
    for (int f = 0; f < AO_MAX_FEATURES; ++f) {
        std::sort(s.begin(), s.end(), [f](const Sample* a, const Sample* b) {
            return a->f[f] < b->f[f] || (a->f[f] == b->f[f] && a->label < b->label);
        });
        std::fill(left.begin(), left.end(), 0);
        for (int k = 0; k < num_classes; ++k) right[k] = nodes[id].counts[k];
        const size_t n = s.size();
        for (size_t q = 0; q + 1 < n; ++q) {
            left[s[q]->label] += 1;
            right[s[q]->label] -= 1;
            if (s[q]->f[f] == s[q + 1]->f[f]) continue;
            const int64_t nl = (int64_t)(q + 1), nr = (int64_t)(n - q - 1);
            int64_t sl = 0, sr = 0;
            for (int k = 0; k < num_classes; ++k) {
                sl += (int64_t)left[k] * left[k];
                sr += (int64_t)right[k] * right[k];
            }
            const __int128 num = (__int128)sl * nr + (__int128)sr * nl;
            const __int128 den = (__int128)nl * nr;
            const double thr = 0.5 * ((double)s[q]->f[f] + (double)s[q + 1]->f[f]);
            // strict: the earlier feature / lower threshold wins ties
            if (best_f < 0 || num * best_den > best_num * den) {
                best_num = num;
                best_den = den;
                best_f = f;
                best_t = thr;
            }
        }
    }
    if (best_f < 0) return id;
    std::vector<Sample*> sl, sr;
    for (Sample* p : s) ((double)p->f[best_f] <= best_t ? sl : sr).push_back(p);
    nodes[id].feature = best_f;
    nodes[id].threshold = best_t;
    const int l = build(nodes, sl, depth + 1, max_depth, num_classes);
    const int r = build(nodes, sr, depth + 1, max_depth, num_classes);
    nodes[id].left = l;
    nodes[id].right = r;
    return id;
}

}  // namespace

int DTree::predict(const float* f, int allowed_mask) const {
    if (nodes.empty()) return -1;
    int i = 0;
    while (nodes[i].feature >= 0) i = ((double)f[nodes[i].feature] <= nodes[i].threshold)
                                          ? nodes[i].left : nodes[i].right;
    const std::vector<int>& c = nodes[i].counts;
    int best = -1;
    for (int k = 0; k < (int)c.size(); ++k)
        if (((allowed_mask >> k) & 1) && c[k] > 0 && (best < 0 || c[k] > c[best])) best = k;
    return best;
}

// samples: features and label per distinct tuple (labels < num_classes)
void DTree::train(const std::vector<std::vector<float>>& feats, const std::vector<int>& labels,
                  int max_depth, int num_classes) {
    std::vector<Sample> data(feats.size());
    for (size_t q = 0; q < feats.size(); ++q) {
        memset(data[q].f, 0, sizeof(data[q].f));
        for (size_t j = 0; j < feats[q].size() && j < (size_t)AO_MAX_FEATURES; ++j)
            data[q].f[j] = feats[q][j];
        data[q].label = labels[q];
    }
    std::vector<Sample*> ptrs;
    for (Sample& d : data) ptrs.push_back(&d);
    nodes.clear();
    if (!ptrs.empty()) build(nodes, ptrs, 0, max_depth, num_classes);
}

}  // namespace ao
