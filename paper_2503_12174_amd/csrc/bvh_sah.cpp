// bvh_sah.cpp -- host construction of the binary BVH by binned surface-area heuristic
// (the scene's alternative to the GPU Morton build; its output has the same layout,
// so the leaf records, validation and the 4-wide collapse are shared).
//
// Top-down: each node's primitives are binned by centroid into 32 bins along every
// axis with a non-zero centroid extent; the split minimising
// area(left) x count(left) + area(right) x count(right) is taken, ties to the lower
// axis and bin.  Nodes whose centroids coincide are split at the middle of their range.
// Leaves are single triangles; leaf l is the triangle order[l].
#include <algorithm>
#include <cfloat>
#include <cstdint>
#include <cstring>
#include <vector>

#include "runtime.hpp"

namespace dpcs {

namespace {

struct Box {
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX};
    float hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    void grow(const Box& b) {
        for (int k = 0; k < 3; ++k) {
            lo[k] = std::min(lo[k], b.lo[k]);
            hi[k] = std::max(hi[k], b.hi[k]);
        }
    }
    double area() const {
        const double dx = std::max(0.0, (double)hi[0] - lo[0]), dy = std::max(0.0, (double)hi[1] - lo[1]),
                     dz = std::max(0.0, (double)hi[2] - lo[2]);
        return dx * dy + dy * dz + dz * dx;
    }
};

constexpr int BINS = 32;

}  // namespace

void sah_build(const float* V, const int* F, int nt, std::vector<float4>& nodes, std::vector<int>& child,
               std::vector<uint32_t>& order) {
    std::vector<Box> pb(nt);
    std::vector<float> cen(3 * (size_t)nt);
    for (int p = 0; p < nt; ++p) {
        for (int k = 0; k < 3; ++k) {
            // same float arithmetic as the device's triangle boxes and Morton centroids
            const float a = V[3 * F[3 * p] + k], b = V[3 * F[3 * p + 1] + k], c = V[3 * F[3 * p + 2] + k];
            pb[p].lo[k] = std::min(a, std::min(b, c));
            pb[p].hi[k] = std::max(a, std::max(b, c));
            cen[3 * (size_t)p + k] = (a + b + c) * (1.0f / 3.0f);
        }
    }
    const int ni = nt - 1;
    nodes.assign(4 * (size_t)ni, make_float4(0.f, 0.f, 0.f, 0.f));
    child.assign(2 * (size_t)ni, 0);
    order.resize(nt);
    for (int p = 0; p < nt; ++p) order[p] = (uint32_t)p;
    struct Task {
        int a, b, node;
    };
    std::vector<Task> tasks{{0, nt, 0}};
    int next = 1;
    auto range_box = [&](int a, int b) {
        Box r;
        for (int i = a; i < b; ++i) r.grow(pb[order[i]]);
        return r;
    };
    while (!tasks.empty()) {
        const Task t = tasks.back();
        tasks.pop_back();
        const int n = t.b - t.a;
        float cl[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, ch[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
        for (int i = t.a; i < t.b; ++i)
            for (int k = 0; k < 3; ++k) {
                cl[k] = std::min(cl[k], cen[3 * (size_t)order[i] + k]);
                ch[k] = std::max(ch[k], cen[3 * (size_t)order[i] + k]);
            }
        double best = -1.0;
        int bax = -1, bsplit = 0;
        for (int ax = 0; ax < 3; ++ax) {
            const double ext = (double)ch[ax] - cl[ax];
            if (!(ext > 0.0)) continue;
            Box bb[BINS];
            int cnt[BINS] = {0};
            const double sc = BINS / ext;
            for (int i = t.a; i < t.b; ++i) {
                const uint32_t p = order[i];
                const int bin = std::min(BINS - 1, (int)((cen[3 * (size_t)p + ax] - (double)cl[ax]) * sc));
                ++cnt[bin];
                bb[bin].grow(pb[p]);
            }
            Box suf[BINS];
            int sn[BINS];
            Box acc;
            int an = 0;
            for (int s = BINS - 1; s >= 0; --s) {
                acc.grow(bb[s]);
                an += cnt[s];
                suf[s] = acc;
                sn[s] = an;
            }
            Box pre;
            int pn = 0;
            for (int s = 1; s < BINS; ++s) {
                pre.grow(bb[s - 1]);
                pn += cnt[s - 1];
                if (pn == 0 || sn[s] == 0) continue;
                const double cost = pre.area() * pn + suf[s].area() * sn[s];
                if (best < 0.0 || cost < best) {
                    best = cost;
                    bax = ax;
                    bsplit = s;
                }
            }
        }
        int mid;
        if (bax < 0) {   // coincident centroids
            mid = t.a + n / 2;
        } else {
            const double ext = (double)ch[bax] - cl[bax], sc = BINS / ext;
            const float base = cl[bax];
            auto in_left = [&](uint32_t p) {
                return std::min(BINS - 1, (int)((cen[3 * (size_t)p + bax] - (double)base) * sc)) < bsplit;
            };
            mid = (int)(std::partition(order.begin() + t.a, order.begin() + t.b, in_left) - order.begin());
        }
        const Box lb = range_box(t.a, mid), rb = range_box(mid, t.b);
        int ref[2];
        const int lo_[2] = {t.a, mid}, hi_[2] = {mid, t.b};
        for (int k = 0; k < 2; ++k) {
            if (hi_[k] - lo_[k] == 1) {
                ref[k] = ~lo_[k];   // leaf: its position in the leaf order
            } else {
                ref[k] = next++;
                tasks.push_back({lo_[k], hi_[k], ref[k]});
            }
        }
        float4* nd = &nodes[4 * (size_t)t.node];
        nd[0] = make_float4(lb.lo[0], lb.lo[1], lb.lo[2], lb.hi[0]);
        nd[1] = make_float4(lb.hi[1], lb.hi[2], rb.lo[0], rb.lo[1]);
        nd[2] = make_float4(rb.lo[2], rb.hi[0], rb.hi[1], rb.hi[2]);
        float rf[2];
        std::memcpy(rf, ref, 8);
        nd[3] = make_float4(rf[0], rf[1], 0.f, 0.f);
        child[2 * (size_t)t.node] = ref[0];
        child[2 * (size_t)t.node + 1] = ref[1];
    }
}

}  // namespace dpcs
