// Mesher: boxes -> axis-aligned rectangles (the partition of the boundary into
// pieces I_j of section 3.1; conductors built from cuboids as in section 3.3).
//
// Edge rules (every box edge is split on its own):
//   uniform(h):  n = max(1, ceil(L/h - 1e-9)); edge k at lo + ((hi - lo) * k) / n
//   graded(h_min, growth, h_max): cells h_min, h_min*growth, ... are taken from
//     both ends while a cell is <= h_max and the run from one end stays
//     <= L/2; the middle [a, b] is split uniformly into
//     max(1, ceil((L - 2 S)/h_max - 1e-9)) cells (none when L - 2 S == 0).
// Order: boxes as given; faces -x, +x, -y, +y, -z, +z; within a face the lower
// in-plane axis is the outer loop.  All arithmetic is plain FP64 without
// contraction (this file is compiled with -ffp-contract=off).
//
// Partition rule of section 3.3 (gbem_mesh_partition), for one main net k:
// every face is split into rectangles I with |I| <= p4 where the distance d
// from I to the main net is <= p5, and |I| <= p4 p3 (d/p5)^3 beyond; p4 = p1
// on faces that face the main net and p1 p2 on faces turned away from it.
// Readings (the paper fixes only the bounds):
//   d      Euclidean distance between I and the nearest box of net k:
//          d^2 = min over those boxes of gx*gx + gy*gy + gz*gz, g the gap
//          per axis (0 where the extents overlap), d = sqrt(d^2);
//   bound  d <= p5: p4; else r = d / p5, p4 * p3 * (r * r * r);
//   facing the faces of net k itself and the faces of a box that contains
//          net k face it; any other face faces it when some box of net k
//          reaches beyond the face's plane on its outer side;
//   split  a rectangle whose area (h1 - l1) * (h2 - l2) exceeds its bound is
//          halved across its longer side (the lower in-plane axis on a tie)
//          at lo + (hi - lo) * 0.5; depth first, lower half first.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "gbem_internal.h"

namespace gbem {

static bool split_edge(double lo, double hi, const gbem_mesh_rule &r, std::vector<double> &e)
{
    e.clear();
    const double L = hi - lo;
    if (r.kind == 0) {
        double q = ceil(L / r.h - 1e-9);
        if (!(q < 1e7)) return false;
        int n = q < 1.0 ? 1 : (int)q;
        e.reserve(n + 1);
        for (int k = 0; k < n; ++k) e.push_back(lo + (L * k) / n);
        e.push_back(hi);
        return true;
    }
    std::vector<double> cells;
    const double half = 0.5 * L;
    double S = 0.0, c = r.h_min;
    while (c <= r.h_max && S + c <= half) {
        cells.push_back(c);
        S = S + c;
        c = c * r.growth;
        if (cells.size() > 100000) return false;
    }
    const double rem = L - 2.0 * S;
    int nmid = 0;
    if (rem > 0.0) {
        double q = ceil(rem / r.h_max - 1e-9);
        if (!(q < 1e7)) return false;
        nmid = q < 1.0 ? 1 : (int)q;
    }
    const int kg = (int)cells.size();
    std::vector<double> right(kg + 1);
    right[0] = hi;
    for (int k = 0; k < kg; ++k) right[k + 1] = right[k] - cells[k];
    e.push_back(lo);
    for (int k = 0; k < kg; ++k) e.push_back(e.back() + cells[k]);
    const double a = e.back(), b = right[kg];
    for (int m = 1; m < nmid; ++m) e.push_back(a + ((b - a) * m) / nmid);
    if (nmid > 0) e.push_back(b);
    for (int k = kg - 1; k >= 0; --k) e.push_back(right[k]);
    return true;
}

static bool boxes_ok(const double *blo, const double *bhi, int nb, std::string &why)
{
    for (int b = 0; b < nb; ++b)
        for (int k = 0; k < 3; ++k)
            if (!(blo[3 * b + k] < bhi[3 * b + k]) || !isfinite(blo[3 * b + k]) || !isfinite(bhi[3 * b + k])) {
                why = "box " + std::to_string(b) + " has a non-positive or non-finite extent";
                return false;
            }
    for (int a = 0; a < nb; ++a)
        for (int b = a + 1; b < nb; ++b) {
            const double *la = blo + 3 * a, *ha = bhi + 3 * a, *lb = blo + 3 * b, *hb = bhi + 3 * b;
            bool disjoint = false, a_in_b = true, b_in_a = true;
            for (int k = 0; k < 3; ++k) {
                if (ha[k] < lb[k] || hb[k] < la[k]) disjoint = true;
                if (!(lb[k] < la[k] && ha[k] < hb[k])) a_in_b = false;
                if (!(la[k] < lb[k] && hb[k] < ha[k])) b_in_a = false;
            }
            if (!disjoint && !a_in_b && !b_in_a) {
                why = "surfaces of boxes " + std::to_string(a) + " and " + std::to_string(b) +
                      " intersect or touch";
                return false;
            }
        }
    return true;
}

// Partition of one face (in-plane axes t1 < t2, normal axis nrm at plane)
// by bisection; appends to lo/hi/cond.  false when the rule asks for more
// than max_total panels or for pieces below 1e-12 of the face.
struct NetBoxes {
    std::vector<double> lo, hi;   // 3 per box of the main net
};
static double net_dist2(const NetBoxes &net, const double *l, const double *h)
{
    double best = INFINITY;
    for (size_t b = 0; b < net.lo.size() / 3; ++b) {
        double d2 = 0.0;
        for (int k = 0; k < 3; ++k) {
            double g = 0.0;
            if (net.lo[3 * b + k] > h[k]) g = net.lo[3 * b + k] - h[k];
            else if (l[k] > net.hi[3 * b + k]) g = l[k] - net.hi[3 * b + k];
            d2 = d2 + g * g;
        }
        if (d2 < best) best = d2;
    }
    return best;
}
static bool partition_face(const NetBoxes &net, double p4, const gbem_partition &r, int nrm, double plane,
                           double a0, double a1, double b0, double b1, int32_t c, std::vector<double> &lo,
                           std::vector<double> &hi, std::vector<int32_t> &cond, size_t max_total, int power = 3)
{
    const int t1 = nrm == 0 ? 1 : 0, t2 = nrm == 2 ? 1 : 2;
    const double min1 = (a1 - a0) * 1e-12, min2 = (b1 - b0) * 1e-12;
    struct Rect { double a0, a1, b0, b1; };
    std::vector<Rect> stack{{a0, a1, b0, b1}};
    while (!stack.empty()) {
        const Rect q = stack.back();
        stack.pop_back();
        double l[3], h[3];
        l[nrm] = plane;
        h[nrm] = plane;
        l[t1] = q.a0;
        h[t1] = q.a1;
        l[t2] = q.b0;
        h[t2] = q.b1;
        const double d = sqrt(net_dist2(net, l, h));
        double bound = p4;
        if (d > r.p5) {
            // power 3: conductors and outer boundary (section 3.3); power 2:
            // dielectric interfaces (section 4.1)
            const double x = d / r.p5;
            bound = p4 * r.p3 * (power == 3 ? x * x * x : x * x);
        }
        const double w1 = q.a1 - q.a0, w2 = q.b1 - q.b0;
        if (w1 * w2 <= bound) {
            if (cond.size() >= max_total) return false;
            for (int k = 0; k < 3; ++k) {
                lo.push_back(l[k]);
                hi.push_back(h[k]);
            }
            cond.push_back(c);
            continue;
        }
        if (w1 < min1 || w2 < min2) return false;
        // halves pushed upper first, so the lower half is emitted first
        if (w1 >= w2) {
            const double m = q.a0 + (q.a1 - q.a0) * 0.5;
            stack.push_back({m, q.a1, q.b0, q.b1});
            stack.push_back({q.a0, m, q.b0, q.b1});
        } else {
            const double m = q.b0 + (q.b1 - q.b0) * 0.5;
            stack.push_back({q.a0, q.a1, m, q.b1});
            stack.push_back({q.a0, q.a1, q.b0, m});
        }
    }
    return true;
}

}  // namespace gbem

using namespace gbem;

extern "C" gbem_status gbem_mesh_boxes(const double *box_lo, const double *box_hi,
                                       const int32_t *box_cond, int32_t n_boxes,
                                       const gbem_mesh_rule *rule, gbem_mesh_buf *out)
{
    if (!box_lo || !box_hi || !box_cond || !rule || !out || n_boxes <= 0) {
        set_error("gbem_mesh_boxes: null argument or no boxes");
        return GBEM_EINVAL;
    }
    if (rule->kind == 0 ? !(rule->h > 0.0)
                        : (rule->kind != 1 || !(rule->h_min > 0.0) || !(rule->growth >= 1.0) ||
                           !(rule->h_max >= rule->h_min))) {
        set_error("gbem_mesh_boxes: invalid mesh rule");
        return GBEM_EINVAL;
    }
    std::string why;
    if (!boxes_ok(box_lo, box_hi, n_boxes, why)) {
        set_error("gbem_mesh_boxes: " + why);
        return GBEM_EINVAL;
    }
    std::vector<double> E[3];
    int64_t total = 0;
    for (int b = 0; b < n_boxes; ++b) {
        int64_t n[3];
        for (int k = 0; k < 3; ++k) {
            if (!split_edge(box_lo[3 * b + k], box_hi[3 * b + k], *rule, E[k])) {
                set_error("gbem_mesh_boxes: edge split too fine");
                return GBEM_EINVAL;
            }
            n[k] = (int64_t)E[k].size() - 1;
        }
        total += 2 * (n[1] * n[2] + n[0] * n[2] + n[0] * n[1]);
    }
    if (total > INT32_MAX) {
        set_error("gbem_mesh_boxes: too many panels");
        return GBEM_EINVAL;
    }
    double *lo = (double *)malloc(sizeof(double) * 3 * total);
    double *hi = (double *)malloc(sizeof(double) * 3 * total);
    int32_t *cond = (int32_t *)malloc(sizeof(int32_t) * total);
    if (!lo || !hi || !cond) {
        free(lo);
        free(hi);
        free(cond);
        set_error("gbem_mesh_boxes: host allocation failed");
        return GBEM_ENOMEM;
    }
    int64_t p = 0;
    for (int b = 0; b < n_boxes; ++b) {
        for (int k = 0; k < 3; ++k) split_edge(box_lo[3 * b + k], box_hi[3 * b + k], *rule, E[k]);
        for (int f = 0; f < 6; ++f) {
            const int nrm = f / 2;
            const double plane = (f & 1) ? box_hi[3 * b + nrm] : box_lo[3 * b + nrm];
            const int t1 = nrm == 0 ? 1 : 0, t2 = nrm == 2 ? 1 : 2;
            const std::vector<double> &e1 = E[t1], &e2 = E[t2];
            for (size_t a = 0; a + 1 < e1.size(); ++a)
                for (size_t c = 0; c + 1 < e2.size(); ++c) {
                    double *l = lo + 3 * p, *h = hi + 3 * p;
                    l[nrm] = plane;
                    h[nrm] = plane;
                    l[t1] = e1[a];
                    h[t1] = e1[a + 1];
                    l[t2] = e2[c];
                    h[t2] = e2[c + 1];
                    cond[p] = box_cond[b];
                    ++p;
                }
        }
    }
    out->n_panels = (int32_t)total;
    out->lo = lo;
    out->hi = hi;
    out->conductor = cond;
    return GBEM_OK;
}

extern "C" void gbem_mesh_buf_free(gbem_mesh_buf *buf)
{
    if (!buf) return;
    free(buf->lo);
    free(buf->hi);
    free(buf->conductor);
    buf->lo = buf->hi = nullptr;
    buf->conductor = nullptr;
    buf->n_panels = 0;
}

extern "C" gbem_status gbem_mesh_partition(const double *box_lo, const double *box_hi,
                                           const int32_t *box_cond, int32_t n_boxes, int32_t main_net,
                                           const gbem_partition *rule, gbem_mesh_buf *out)
{
    if (!box_lo || !box_hi || !box_cond || !rule || !out || n_boxes <= 0) {
        set_error("gbem_mesh_partition: null argument or no boxes");
        return GBEM_EINVAL;
    }
    if (!(rule->p1 > 0.0) || !(rule->p2 >= 1.0) || !(rule->p3 > 0.0) || !(rule->p5 > 0.0) ||
        !isfinite(rule->p1) || !isfinite(rule->p2) || !isfinite(rule->p3) || !isfinite(rule->p5)) {
        set_error("gbem_mesh_partition: need p1 > 0, p2 >= 1, p3 > 0, p5 > 0 (finite)");
        return GBEM_EINVAL;
    }
    std::string why;
    if (!boxes_ok(box_lo, box_hi, n_boxes, why)) {
        set_error("gbem_mesh_partition: " + why);
        return GBEM_EINVAL;
    }
    // boxes of the main net: one conductor, or every conductor (GBEM_ALL_NETS)
    auto on_main = [&](int b) { return main_net == GBEM_ALL_NETS ? box_cond[b] >= 0 : box_cond[b] == main_net; };
    NetBoxes net;
    double nlo[3] = {INFINITY, INFINITY, INFINITY}, nhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < n_boxes; ++b)
        if (on_main(b))
            for (int k = 0; k < 3; ++k) {
                net.lo.push_back(box_lo[3 * b + k]);
                net.hi.push_back(box_hi[3 * b + k]);
                nlo[k] = fmin(nlo[k], box_lo[3 * b + k]);
                nhi[k] = fmax(nhi[k], box_hi[3 * b + k]);
            }
    if (net.lo.empty()) {
        set_error("gbem_mesh_partition: no box belongs to the main net");
        return GBEM_EINVAL;
    }
    const size_t max_total = (size_t)INT32_MAX / 4;
    std::vector<double> lo, hi;
    std::vector<int32_t> cond;
    for (int b = 0; b < n_boxes; ++b) {
        const double *bl = box_lo + 3 * b, *bh = box_hi + 3 * b;
        bool contains = true;   // box b strictly contains the main net's bounding box
        for (int k = 0; k < 3; ++k)
            if (!(bl[k] < nlo[k] && nhi[k] < bh[k])) contains = false;
        for (int f = 0; f < 6; ++f) {
            const int nrm = f / 2;
            const bool upper = f & 1;
            const double plane = upper ? bh[nrm] : bl[nrm];
            bool facing = on_main(b) || contains;
            if (!facing) {
                for (size_t q = 0; q < net.lo.size() / 3 && !facing; ++q)
                    facing = upper ? net.hi[3 * q + nrm] > plane : net.lo[3 * q + nrm] < plane;
            }
            const double p4 = facing ? rule->p1 : rule->p1 * rule->p2;
            const int t1 = nrm == 0 ? 1 : 0, t2 = nrm == 2 ? 1 : 2;
            if (!partition_face(net, p4, *rule, nrm, plane, bl[t1], bh[t1], bl[t2], bh[t2], box_cond[b], lo, hi,
                                cond, max_total)) {
                set_error("gbem_mesh_partition: the rule asks for too many or too small panels");
                return GBEM_EINVAL;
            }
        }
    }
    const size_t n = cond.size();
    double *plo = (double *)malloc(sizeof(double) * 3 * n);
    double *phi = (double *)malloc(sizeof(double) * 3 * n);
    int32_t *pc = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!plo || !phi || !pc) {
        free(plo);
        free(phi);
        free(pc);
        set_error("gbem_mesh_partition: host allocation failed");
        return GBEM_ENOMEM;
    }
    memcpy(plo, lo.data(), sizeof(double) * 3 * n);
    memcpy(phi, hi.data(), sizeof(double) * 3 * n);
    memcpy(pc, cond.data(), sizeof(int32_t) * n);
    out->n_panels = (int32_t)n;
    out->lo = plo;
    out->hi = phi;
    out->conductor = pc;
    return GBEM_OK;
}

// ------------------------------------------------------------------------
// Layered multi-dielectric layouts (section 4): per-main-net meshes
// ------------------------------------------------------------------------
extern "C" void gbem_dmesh_buf_free(gbem_dmesh_buf *buf)
{
    if (!buf) return;
    free(buf->lo);
    free(buf->hi);
    free(buf->kind);
    free(buf->conductor);
    free(buf->region_plus);
    free(buf->region_minus);
    memset(buf, 0, sizeof(*buf));
}

extern "C" gbem_status gbem_mesh_dielectric_partition(const gbem_dlayout *L, int32_t main_net,
                                                      const gbem_partition *rule, gbem_dmesh_buf *out)
{
    if (!L || !rule || !out || !L->box_lo || !L->box_hi || !L->box_net || !L->z_layer || L->n_boxes <= 0 ||
        L->n_layers <= 0 || L->n_conductors <= 0) {
        set_error("gbem_mesh_dielectric_partition: null argument, no boxes or no layers");
        return GBEM_EINVAL;
    }
    if (!(rule->p1 > 0.0) || !(rule->p2 >= 1.0) || !(rule->p3 > 0.0) || !(rule->p5 > 0.0) ||
        !isfinite(rule->p1) || !isfinite(rule->p2) || !isfinite(rule->p3) || !isfinite(rule->p5)) {
        set_error("gbem_mesh_dielectric_partition: need p1 > 0, p2 >= 1, p3 > 0, p5 > 0 (finite)");
        return GBEM_EINVAL;
    }
    const int nb = L->n_boxes, nl = L->n_layers;
    const double *dlo = L->domain_lo, *dhi = L->domain_hi, *z = L->z_layer;
    for (int k = 0; k < 3; ++k)
        if (!(dlo[k] < dhi[k])) {
            set_error("gbem_mesh_dielectric_partition: empty domain");
            return GBEM_EINVAL;
        }
    if (z[0] != dlo[2] || z[nl] != dhi[2]) {
        set_error("gbem_mesh_dielectric_partition: z_layer must run from domain_lo[2] to domain_hi[2]");
        return GBEM_EINVAL;
    }
    for (int a = 0; a < nl; ++a)
        if (!(z[a] < z[a + 1])) {
            set_error("gbem_mesh_dielectric_partition: z_layer must increase");
            return GBEM_EINVAL;
        }
    for (int kd : {L->bottom_kind, L->top_kind, L->side_kind})
        if (kd != GBEM_PANEL_DIRICHLET && kd != GBEM_PANEL_NEUMANN) {
            set_error("gbem_mesh_dielectric_partition: outer faces must be GBEM_PANEL_DIRICHLET or GBEM_PANEL_NEUMANN");
            return GBEM_EINVAL;
        }
    std::string why;
    if (!boxes_ok(L->box_lo, L->box_hi, nb, why)) {
        set_error("gbem_mesh_dielectric_partition: " + why);
        return GBEM_EINVAL;
    }
    // layer of each box: strictly inside one layer and inside the domain
    std::vector<int> layer(nb, -1);
    for (int b = 0; b < nb; ++b) {
        const double *bl = L->box_lo + 3 * b, *bh = L->box_hi + 3 * b;
        bool inside = L->box_net[b] >= 0 && L->box_net[b] < L->n_conductors;
        for (int k = 0; k < 3; ++k) inside = inside && dlo[k] < bl[k] && bh[k] < dhi[k];
        for (int a = 0; a < nl && inside; ++a)
            if (z[a] < bl[2] && bh[2] < z[a + 1]) layer[b] = a;
        if (layer[b] < 0) {
            set_error("gbem_mesh_dielectric_partition: box " + std::to_string(b) +
                      " is not strictly inside one layer of the domain, or its net is out of range");
            return GBEM_EINVAL;
        }
    }
    NetBoxes net;
    for (int b = 0; b < nb; ++b)
        if (L->box_net[b] == main_net)
            for (int k = 0; k < 3; ++k) {
                net.lo.push_back(L->box_lo[3 * b + k]);
                net.hi.push_back(L->box_hi[3 * b + k]);
            }
    if (net.lo.empty()) {
        set_error("gbem_mesh_dielectric_partition: no box belongs to the main net");
        return GBEM_EINVAL;
    }
    const size_t max_total = (size_t)INT32_MAX / 4;
    std::vector<double> lo, hi;
    std::vector<int32_t> cond, kind, rp, rm;
    // append the panels a face produced since `from`, with their kind and regions
    auto tag = [&](size_t from, int32_t kd, int32_t plus, int32_t minus) {
        for (size_t i = from; i < cond.size(); ++i) {
            kind.push_back(kd);
            rp.push_back(plus);
            rm.push_back(minus);
        }
    };
    auto fail = [&]() {
        set_error("gbem_mesh_dielectric_partition: the rule asks for too many or too small panels");
        return GBEM_EINVAL;
    };
    // conductor faces: the section 3.3 rule, facing / back as for boxes
    for (int b = 0; b < nb; ++b) {
        const double *bl = L->box_lo + 3 * b, *bh = L->box_hi + 3 * b;
        for (int f = 0; f < 6; ++f) {
            const int nrm = f / 2;
            const bool upper = f & 1;
            const double plane = upper ? bh[nrm] : bl[nrm];
            bool facing = L->box_net[b] == main_net;
            for (size_t q = 0; q < net.lo.size() / 3 && !facing; ++q)
                facing = upper ? net.hi[3 * q + nrm] > plane : net.lo[3 * q + nrm] < plane;
            const double p4 = facing ? rule->p1 : rule->p1 * rule->p2;
            const int t1 = nrm == 0 ? 1 : 0, t2 = nrm == 2 ? 1 : 2;
            const size_t from = cond.size();
            if (!partition_face(net, p4, *rule, nrm, plane, bl[t1], bh[t1], bl[t2], bh[t2], L->box_net[b], lo, hi,
                                cond, max_total))
                return fail();
            // the dielectric lies outside the box: on the - side of a lower face
            tag(from, GBEM_PANEL_CONDUCTOR, upper ? layer[b] : -1, upper ? -1 : layer[b]);
        }
    }
    // outer boundary (section 3.3 rule; it encloses the main net, so every
    // face counts as facing): bottom, top, and the side walls per layer
    {
        size_t from = cond.size();
        if (!partition_face(net, rule->p1, *rule, 2, dlo[2], dlo[0], dhi[0], dlo[1], dhi[1], -1, lo, hi, cond,
                            max_total))
            return fail();
        tag(from, L->bottom_kind, 0, -1);
        from = cond.size();
        if (!partition_face(net, rule->p1, *rule, 2, dhi[2], dlo[0], dhi[0], dlo[1], dhi[1], -1, lo, hi, cond,
                            max_total))
            return fail();
        tag(from, L->top_kind, -1, nl - 1);
        for (int a = 0; a < nl; ++a)
            for (int nrm = 0; nrm < 2; ++nrm)
                for (int upper = 0; upper < 2; ++upper) {
                    const int t = 1 - nrm;   // the other horizontal axis (in-plane axes t < 2)
                    from = cond.size();
                    const double plane = upper ? dhi[nrm] : dlo[nrm];
                    if (!partition_face(net, rule->p1, *rule, nrm, plane, dlo[t], dhi[t], z[a], z[a + 1], -1, lo, hi,
                                        cond, max_total))
                        return fail();
                    tag(from, L->side_kind, upper ? -1 : a, upper ? a : -1);
                }
    }
    // interfaces between layers: the section 4.1 rule (growth with d^2)
    for (int a = 1; a < nl; ++a) {
        const size_t from = cond.size();
        if (!partition_face(net, rule->p1, *rule, 2, z[a], dlo[0], dhi[0], dlo[1], dhi[1], -1, lo, hi, cond,
                            max_total, 2))
            return fail();
        tag(from, GBEM_PANEL_INTERFACE, a, a - 1);
    }
    const size_t n = cond.size();
    gbem_dmesh_buf r{};
    r.lo = (double *)malloc(sizeof(double) * 3 * n);
    r.hi = (double *)malloc(sizeof(double) * 3 * n);
    r.kind = (int32_t *)malloc(sizeof(int32_t) * n);
    r.conductor = (int32_t *)malloc(sizeof(int32_t) * n);
    r.region_plus = (int32_t *)malloc(sizeof(int32_t) * n);
    r.region_minus = (int32_t *)malloc(sizeof(int32_t) * n);
    if (!r.lo || !r.hi || !r.kind || !r.conductor || !r.region_plus || !r.region_minus) {
        gbem_dmesh_buf_free(&r);
        set_error("gbem_mesh_dielectric_partition: host allocation failed");
        return GBEM_ENOMEM;
    }
    memcpy(r.lo, lo.data(), sizeof(double) * 3 * n);
    memcpy(r.hi, hi.data(), sizeof(double) * 3 * n);
    memcpy(r.kind, kind.data(), sizeof(int32_t) * n);
    memcpy(r.conductor, cond.data(), sizeof(int32_t) * n);
    memcpy(r.region_plus, rp.data(), sizeof(int32_t) * n);
    memcpy(r.region_minus, rm.data(), sizeof(int32_t) * n);
    r.n_panels = (int32_t)n;
    *out = r;
    return GBEM_OK;
}
