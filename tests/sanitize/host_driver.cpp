// Drives the host-only paths of libart (argument validation, the block-
// wavefront schedule, handle lifetime, SHA-256) in a build whose host code has
// AddressSanitizer and UndefinedBehaviorSanitizer.  No call here reaches the
// device, so it runs without a GPU.  Exit status 0 when every call returned
// the expected code.
#include <cstdio>
#include <cstring>
#include <vector>

#include "art.h"
#include "art_point.h"
#include "art_surrogate.h"

#define CHECK(cond, what)                                   \
    do {                                                    \
        if (!(cond)) {                                      \
            std::fprintf(stderr, "FAIL: %s (%s)\n", what, art_last_error()); \
            return 1;                                       \
        }                                                   \
    } while (0)

int main()
{
    art_mesh *m = nullptr;
    CHECK(art_create_mesh(0, 4, 4, 1.0, &m) == ART_E_INVAL, "zero side");
    CHECK(art_create_mesh(4, 4, 4, -1.0, &m) == ART_E_INVAL, "negative cell size");
    CHECK(art_create_mesh(5000, 4, 4, 1.0, &m) == ART_E_INVAL, "side above 4096");
    CHECK(art_create_mesh(4, 4, 4, 1.0, nullptr) == ART_E_INVAL, "null out");
    CHECK(art_create_mesh(9, 7, 5, 0.5, &m) == ART_OK && m, "create");
    art_tuning t{6, 1, 1, 3};
    CHECK(art_set_tuning(m, &t) == ART_OK, "set tuning");
    art_tuning bad{0, 1, 1, 3};
    CHECK(art_set_tuning(m, &bad) == ART_E_INVAL, "bad tuning");
    art_tuning bigk{6, 1, 1, 5};
    CHECK(art_set_tuning(m, &bigk) == ART_E_INVAL, "five directions per wave");
    art_tuning got{};
    CHECK(art_get_tuning(m, &got) == ART_OK && got.depth == 6, "get tuning");
    art_outputs out{};
    CHECK(art_sweep(m, 2, nullptr, 0.0f, &out, nullptr) == ART_E_STATE, "sweep before fields");
    CHECK(art_sweep_range(m, 2, 0, 3, 0.0f, nullptr, nullptr, nullptr) == ART_E_STATE, "range before fields");
    CHECK(art_set_fields(m, 1, nullptr, nullptr, 0, nullptr) == ART_E_INVAL, "null fields");
    float f = 0.0f;
    CHECK(art_set_fields(m, 5, &f, &f, 0, nullptr) == ART_E_UNSUPPORTED, "too many bins");
    CHECK(art_set_heating(m, &f, &f) == ART_E_STATE, "heating before fields");
    long long segs = 0;
    CHECK(art_sweep_stats(m, &segs, nullptr, nullptr) == ART_E_STATE, "stats before a sweep");
    CHECK(art_point_sources(m, 0, nullptr, nullptr, nullptr, &f, &f, nullptr, nullptr, nullptr) == ART_E_STATE,
          "point sources before fields");
    CHECK(art_ndirs(8) == 768 && art_ndirs(0) == ART_E_INVAL && art_ndirs(65) == ART_E_INVAL, "ndirs");
    for (int depth : {1, 3, 6, 12})
        for (int subsets : {1, 2, 5}) {
            art_tuning ts{depth, subsets, 1, 2};
            long long n = 0;
            int nw = 0;
            CHECK(art_schedule(9, 7, 5, &ts, nullptr, 0, &n, &nw) == ART_OK && n > 0, "schedule count");
            std::vector<int> items((size_t)n * 3);
            CHECK(art_schedule(9, 7, 5, &ts, items.data(), n - 1, &n, &nw) == ART_E_INVAL, "schedule cap");
            CHECK(art_schedule(9, 7, 5, &ts, items.data(), n, &n, &nw) == ART_OK, "schedule items");
            for (long long q = 0; q < n; ++q)
                CHECK(items[3 * q] >= 0 && items[3 * q] < nw, "wavefront in range");
        }
    CHECK(art_destroy_mesh(m) == ART_OK, "destroy");
    CHECK(art_destroy_mesh(nullptr) == ART_OK, "destroy NULL");
    art_batch *b = nullptr;
    CHECK(art_batch_create(nullptr, nullptr, 0, nullptr, 0.0f, nullptr, 1, &b, nullptr) == ART_E_INVAL,
          "batch without meshes");
    CHECK(art_batch_launch(nullptr, nullptr) == ART_E_INVAL, "launch NULL batch");
    CHECK(art_batch_destroy(nullptr) == ART_OK, "destroy NULL batch");
    art_surrogate *s = nullptr;
    CHECK(art_surrogate_create(33, 8, 8, 1, &s) == ART_E_INVAL, "surrogate width not a multiple of 32");
    CHECK(art_surrogate_destroy(nullptr) == ART_OK, "destroy NULL surrogate");
    unsigned char dg[32];
    const char *msg = "abc";
    CHECK(art_sha256(msg, 3, dg) == ART_OK && dg[0] == 0xba && dg[31] == 0xad, "sha256 of abc");
    std::vector<unsigned char> big1(1000003, 0x61);
    CHECK(art_sha256(big1.data(), big1.size(), dg) == ART_OK, "sha256 of 1 MB");
    std::printf("host driver: ok\n");
    return 0;
}
