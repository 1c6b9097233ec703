// Host-side fuzz driver for the library's meshers and tuning-cache parser,
// built by tests/test_host_sanitizers.py with g++ and the address and
// undefined-behaviour sanitizers (host code only; no device code is built).
// Seeded random valid and invalid inputs; every call must either succeed
// with a consistent result or fail with an error message.  Exit status 0 on
// success, 1 on an inconsistent result (the sanitizers abort on their own).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <random>
#include <string>
#include <vector>

#include "gbem.h"

namespace gbem {
static std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }
}  // namespace gbem

static int fails = 0;
#define CHECK(c, what)                                              \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "inconsistent: %s (%s)\n", what, #c);   \
            ++fails;                                                \
        }                                                           \
    } while (0)

static double area_of(const double *lo, const double *hi)
{
    double a = 1.0;
    for (int k = 0; k < 3; ++k)
        if (hi[k] > lo[k]) a *= hi[k] - lo[k];
    return a;
}

int main(int argc, char **argv)
{
    const int rounds = argc > 1 ? atoi(argv[1]) : 200;
    std::mt19937_64 rng(20221203);
    std::uniform_real_distribution<double> U(0.0, 1.0);
    for (int it = 0; it < rounds; ++it) {
        // ---- random boxes (sometimes overlapping or degenerate) ----
        const int nb = 1 + (int)(U(rng) * 4);
        std::vector<double> lo(3 * nb), hi(3 * nb);
        std::vector<int32_t> cond(nb);
        double surface = 0.0;
        for (int b = 0; b < nb; ++b) {
            for (int k = 0; k < 3; ++k) {
                lo[3 * b + k] = 3.0 * b + U(rng) * 2.0 * (k == 0);
                hi[3 * b + k] = lo[3 * b + k] + (U(rng) < 0.05 ? 0.0 : 0.2 + U(rng));
            }
            cond[b] = U(rng) < 0.1 ? -1 : b % 3;
            const double e0 = hi[3 * b] - lo[3 * b], e1 = hi[3 * b + 1] - lo[3 * b + 1], e2 = hi[3 * b + 2] - lo[3 * b + 2];
            surface += 2.0 * (e0 * e1 + e0 * e2 + e1 * e2);
        }
        gbem_mesh_rule rule{};
        rule.kind = U(rng) < 0.5 ? 0 : 1;
        rule.h = U(rng) < 0.05 ? -1.0 : 0.05 + 0.3 * U(rng);
        rule.h_min = 0.01 + 0.05 * U(rng);
        rule.growth = 1.0 + U(rng);
        rule.h_max = rule.h_min * (1.0 + 5.0 * U(rng));
        gbem_mesh_buf mb{};
        if (gbem_mesh_boxes(lo.data(), hi.data(), cond.data(), nb, &rule, &mb) == GBEM_OK) {
            double a = 0.0;
            for (int i = 0; i < mb.n_panels; ++i) a += area_of(mb.lo + 3 * i, mb.hi + 3 * i);
            CHECK(fabs(a - surface) <= 1e-9 * surface, "gbem_mesh_boxes tiles the surfaces");
            gbem_mesh_buf_free(&mb);
        }
        gbem_partition pr{};
        pr.p1 = U(rng) < 0.05 ? 0.0 : 0.01 + 0.2 * U(rng);
        pr.p2 = 1.0 + 3.0 * U(rng);
        pr.p3 = 0.2 + U(rng);
        pr.p5 = 0.2 + U(rng);
        const int main_net = U(rng) < 0.1 ? GBEM_ALL_NETS : (int)(U(rng) * 3);
        if (gbem_mesh_partition(lo.data(), hi.data(), cond.data(), nb, main_net, &pr, &mb) == GBEM_OK) {
            double a = 0.0;
            for (int i = 0; i < mb.n_panels; ++i) a += area_of(mb.lo + 3 * i, mb.hi + 3 * i);
            CHECK(fabs(a - surface) <= 1e-9 * surface, "gbem_mesh_partition tiles the surfaces");
            gbem_mesh_buf_free(&mb);
        }

        // ---- layered dielectric layouts (sometimes invalid) ----
        const int nl = 1 + (int)(U(rng) * 3);
        std::vector<double> z(nl + 1), eps(nl);
        z[0] = 0.0;
        for (int a = 0; a < nl; ++a) {
            z[a + 1] = z[a] + 0.8 + U(rng);
            eps[a] = 1.0 + 5.0 * U(rng);
        }
        const double W = 3.0 + 2.0 * U(rng);
        const int nw = 1 + (int)(U(rng) * 3);
        std::vector<double> blo, bhi;
        std::vector<int32_t> bnet;
        for (int w = 0; w < nw; ++w) {
            const int a = (int)(U(rng) * nl);
            const double y0 = 0.5 + w * (W - 1.0) / nw;
            const double zz = z[a] + 0.2 * (z[a + 1] - z[a]) + (U(rng) < 0.05 ? -1.0 : 0.0);
            blo.insert(blo.end(), {0.5, y0, zz});
            bhi.insert(bhi.end(), {W - 0.5, y0 + 0.3 * (W - 1.0) / nw, zz + 0.5 * (z[a + 1] - z[a])});
            bnet.push_back(w);
        }
        gbem_dlayout L{};
        L.n_boxes = nw;
        L.box_lo = blo.data();
        L.box_hi = bhi.data();
        L.box_net = bnet.data();
        L.n_conductors = nw;
        L.domain_lo[0] = L.domain_lo[1] = 0.0;
        L.domain_lo[2] = z[0];
        L.domain_hi[0] = L.domain_hi[1] = W;
        L.domain_hi[2] = z[nl];
        L.n_layers = nl;
        L.z_layer = z.data();
        L.eps_r = eps.data();
        L.bottom_kind = GBEM_PANEL_DIRICHLET;
        L.top_kind = U(rng) < 0.05 ? 7 : GBEM_PANEL_DIRICHLET;
        L.side_kind = GBEM_PANEL_NEUMANN;
        L.length_unit_m = 1e-6;
        gbem_partition dr{};
        dr.p1 = 0.05 + 0.3 * U(rng);
        dr.p2 = 1.0 + 3.0 * U(rng);
        dr.p3 = 0.3 + U(rng);
        dr.p5 = 0.3 + U(rng);
        gbem_dmesh_buf db{};
        if (gbem_mesh_dielectric_partition(&L, (int)(U(rng) * nw), &dr, &db) == GBEM_OK) {
            // every region's boundary closes: outward area vectors sum to zero
            for (int a = 0; a < nl; ++a) {
                double v[3] = {0, 0, 0};
                for (int i = 0; i < db.n_panels; ++i) {
                    if (db.region_plus[i] != a && db.region_minus[i] != a) continue;
                    int n = 0;
                    for (int k = 0; k < 3; ++k)
                        if (db.hi[3 * i + k] == db.lo[3 * i + k]) n = k;
                    v[n] += (db.region_plus[i] == a ? -1.0 : 1.0) * area_of(db.lo + 3 * i, db.hi + 3 * i);
                }
                CHECK(fabs(v[0]) + fabs(v[1]) + fabs(v[2]) <= 1e-9 * W * W, "region boundary closes");
            }
            gbem_dmesh_buf_free(&db);
        }
    }

    // ---- tuning cache parser: valid, truncated and corrupted files ----
    const char *good =
        "{\"entries\": [{\"factor\": \"16bit\", \"npad_min\": 0, \"npad_max\": 4096, \"outer_width\": 256, "
        "\"super_panels\": 2, \"ms\": {\"256x2\": 1.0}}, {\"factor\": \"f64\", \"npad_min\": 0, \"npad_max\": 1000000, "
        "\"outer_width\": 512}]}";
    char path[] = "/tmp/gbem_fuzz_tuneXXXXXX";
    const int fd = mkstemp(path);
    if (fd < 0) return 1;
    close(fd);
    const std::string g(good);
    for (int it = 0; it < 400; ++it) {
        std::string t = g;
        if (it > 0) {
            const int kind = it % 3;
            const size_t pos = (size_t)(U(rng) * t.size());
            if (kind == 0) t = t.substr(0, pos);                              // truncated
            else if (kind == 1) t[pos] = (char)(32 + (int)(U(rng) * 95));     // one character changed
            else t.insert(pos, std::string(1 + (int)(U(rng) * 40), '{'));      // nesting
        }
        FILE *f = fopen(path, "wb");
        fwrite(t.data(), 1, t.size(), f);
        fclose(f);
        const gbem_status s = gbem_load_tuning(path);
        CHECK(it > 0 || s == GBEM_OK, "the valid cache loads");
    }
    (void)gbem_load_tuning(nullptr);
    remove(path);
    printf("host fuzz: %d rounds, %d inconsistencies\n", rounds, fails);
    return fails ? 1 : 0;
}
