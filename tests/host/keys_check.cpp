// Host check of the partition's iteration-stamped key arithmetic
// (paper_1612_09368_amd/csrc/cm_keys.h), built with hipcc as host code and
// run by tests/test_keys.py: keys fall strictly with (iteration, round) up to
// the largest stamp a handle can use, never wrap, and matched_before accepts
// exactly the earlier rounds of the same iteration.
#include <cstdio>
#include <cstdlib>

#include "../../paper_1612_09368_amd/csrc/cm_keys.h"

using namespace cm;

static int fails = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            std::printf("FAIL line %d: %s\n", __LINE__, #c);             \
            if (++fails > 20) std::exit(1);                              \
        }                                                                \
    } while (0)

static void window(int rounds, int32_t ep_lo, int32_t ep_hi) {
    unsigned long long prev = ~0ull;  // the cleared claim value: every key must beat it
    for (int32_t ep = ep_lo; ep <= ep_hi; ++ep) {
        for (int r = 0; r < rounds; ++r) {
            const unsigned long long k = claim_hi(ep, rounds, r) | 0xFFFFFFFFull;  // largest key of the round
            CHECK(k < prev);
            CHECK((claim_hi(ep, rounds, r) >> 32) != 0xFFFFFFFFull);  // never the cleared high word
            prev = claim_hi(ep, rounds, r);                            // smallest key of the round
            const uint32_t m = matched_stamp(ep, rounds, r);
            CHECK(m != 0u);
            for (int rr = 0; rr < rounds; ++rr) {
                CHECK(matched_before(m, ep, rounds, rr) == (r < rr));  // a match counts in later rounds only
                if (ep > ep_lo) CHECK(!matched_before(matched_stamp(ep - 1, rounds, rr), ep, rounds, r));
                CHECK(!matched_before(0u, ep, rounds, rr));  // the cleared value never counts
            }
        }
    }
}

int main() {
    for (int rounds = 1; rounds <= MAX_ROUNDS; ++rounds) {
        window(rounds, 1, 64);                            // after a restart
        window(rounds, EPOCH_REWIND - 64, EPOCH_REWIND);  // up to the largest stamp in use
        // the largest round number of the largest stamp still fits in 32 bits
        CHECK((unsigned long long)EPOCH_REWIND * rounds + rounds - 1 < (1ull << 32));
    }
    std::printf(fails ? "keys: %d failures\n" : "keys: ok\n", fails);
    return fails ? 1 : 0;
}
