// Host-only check of the autotuner's JSON cache format: write, read back,
// reject malformed input.  Built and run by tests/test_tune_format.py.
#include <cstdio>
#include <string>
#include <vector>

#include "tune.hpp"

using bdm::TuneEntry;

static int fails = 0;
#define CHECK(c)                                                   \
    do {                                                           \
        if (!(c)) {                                                \
            std::printf("FAIL %s:%d %s\n", __FILE__, __LINE__, #c); \
            ++fails;                                               \
        }                                                          \
    } while (0)

int main() {
    std::vector<TuneEntry> in(2);
    in[0].device = "gfx950";
    in[0].family = "stencil";
    in[0].cls = "mesh 8x8x8 \"q\"\\";
    in[0].choice = 3;
    in[0].ms = {0.5, 0.25, -1, 0.125, 1e-3};
    in[1].device = "gfx950";
    in[1].family = "syrk";
    in[1].cls = "f32 interior nsub=8 ne<=686 n<=1458";
    in[1].choice = 0;
    const std::string js = bdm::tune_to_json(in);
    std::vector<TuneEntry> out;
    CHECK(bdm::tune_from_json(js, out).empty());
    CHECK(out.size() == 2);
    if (out.size() == 2) {
        CHECK(out[0].device == "gfx950" && out[0].family == "stencil" && out[0].cls == in[0].cls);
        CHECK(out[0].choice == 3 && out[0].ms.size() == 5 && out[0].ms[1] == 0.25 && out[0].ms[2] == -1);
        CHECK(out[1].cls == in[1].cls && out[1].choice == 0 && out[1].ms.empty());
        CHECK(out[0].cached && out[1].cached);
    }
    // whitespace and key order are free
    CHECK(bdm::tune_from_json(" {\n \"entries\" : [ { \"ms\":[1,2], \"choice\" : 1, \"class\":\"c\", \"family\":\"f\","
                              " \"device\":\"d\"} ], \"format\":\"bidomain-tune-1\" } ", out).empty());
    CHECK(out.size() == 1 && out[0].choice == 1 && out[0].family == "f");
    // malformed inputs are rejected
    const char* bad[] = {"", "{", "[]", "{\"format\": \"other\", \"entries\": []}",
                         "{\"format\": \"bidomain-tune-1\"}",
                         "{\"format\": \"bidomain-tune-1\", \"entries\": [{\"device\": \"d\"}]}",
                         "{\"format\": \"bidomain-tune-1\", \"entries\": [{\"device\": \"d\", \"family\": \"f\", "
                         "\"class\": \"c\", \"choice\": 1.5}]}",
                         "{\"format\": \"bidomain-tune-1\", \"entries\": []} x"};
    for (const char* b : bad) {
        std::vector<TuneEntry> o;
        CHECK(!bdm::tune_from_json(b, o).empty());
    }
    // the tuner takes a cached choice without timing, times otherwise
    bdm::Tuner t;
    t.device = "gfx950";
    t.entries = out;
    t.entries[0].device = "gfx950";
    int calls = 0;
    CHECK(t.pick("f", "c", 4, [&](int) { ++calls; return 1.0; }) == 1 && calls == 0 && !t.dirty);
    CHECK(t.pick("f", "c2", 3, [&](int v) { ++calls; return v == 2 ? 0.5 : (v == 0 ? -1.0 : 2.0); }) == 2);
    CHECK(calls == 3 && t.dirty);
    CHECK(t.pick("f", "c", 1, [&](int) { ++calls; return 1.0; }) == 0 && calls == 4);   // cached choice out of range
    // within 1% of the fastest is a tie, taken by the lowest index; a failed
    // timing (negative) never wins
    const double tt[5] = {-1.0, 1.2, 1.009, 1.0, 1.005};
    CHECK(t.pick("f", "tie", 5, [&](int v) { return tt[v]; }) == 2);
    const double tu[3] = {1.02, 1.011, 1.0};
    CHECK(t.pick("f", "notie", 3, [&](int v) { return tu[v]; }) == 2);
    std::vector<TuneEntry> rep;
    CHECK(bdm::tune_from_json(t.report(), rep).empty() && rep.size() == 5);
    std::printf(fails ? "FAILED\n" : "OK\n");
    return fails ? 1 : 0;
}
