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
