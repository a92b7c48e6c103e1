// Unit tests of the native server's admission and grouping policy
// (csrc/admission.hpp), host only, meant to run under AddressSanitizer and
// UndefinedBehaviorSanitizer.  The fake engine below models what a slot's
// device buffers really hold: a build asks for a random split of at most
// its group's footprint over a fixed set of buffers, each buffer grows to
// the exact size asked for and keeps it, and a trimmed slot holds nothing.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "admission.hpp"

using cleora::Admission;
using cleora::AdmitDecision;

static int failures = 0;
#define CHECK(cond)                                                                 \
    do {                                                                            \
        if (!(cond)) {                                                              \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                             \
        }                                                                           \
    } while (0)

static void budget_edges()
{
    {
        Admission a(2, 100, 4);
        a.push(100, 10);
        CHECK(a.can_admit());  // exactly the budget fits
        AdmitDecision d = a.admit();
        CHECK(d.count == 1 && d.footprint == 100 && d.trim.empty());
        CHECK(a.used() == 100 && a.peak() == 100);
        a.push(1, 1);
        CHECK(!a.can_admit());  // nothing left while it builds
        CHECK(a.built(d.slot, 60));
        CHECK(a.used() == 60);
        CHECK(!a.can_admit() || a.room() >= 1);
    }
    {
        Admission a(1, 99, 4);
        a.push(100, 10);
        CHECK(!a.can_admit());  // one byte over: never
    }
    {
        Admission a(3, 0, 4);
        a.push(0, 1);  // a zero charge fits a zero budget
        CHECK(a.can_admit());
    }
}

static void max_group_and_order()
{
    Admission a(8, 1000, 4);
    for (int i = 0; i < 10; ++i) a.push(10, 5);
    std::vector<int> sizes;
    while (a.can_admit()) sizes.push_back(a.admit().count);
    CHECK(sizes.size() == 3 && sizes[0] == 4 && sizes[1] == 4 && sizes[2] == 2);
    CHECK(a.used() == 100 && a.groups() == 3);

    // no overtaking: a request that does not fit blocks the ones behind it
    Admission b(4, 100, 4);
    b.push(60, 1);
    AdmitDecision d = b.admit();
    b.push(50, 1);
    b.push(1, 1);
    CHECK(!b.can_admit());
    CHECK(b.built(d.slot, 0));
    b.release(d.slot);
    CHECK(b.can_admit());
    AdmitDecision e = b.admit();
    CHECK(e.count == 2 && e.footprint == 51);

    // the group stops at the first request that does not fit
    Admission c(4, 100, 8);
    c.push(40, 1);
    c.push(40, 1);
    c.push(40, 1);
    c.push(1, 1);
    AdmitDecision f = c.admit();
    CHECK(f.count == 2 && f.footprint == 80 && c.waiting() == 2);
}

static void node_limit()
{
    Admission a(4, 1 << 30, 8);
    const int64_t half = int64_t(1) << 30;
    a.push(1, half);
    a.push(1, half);       // 2^31 nodes together: above the int32 range
    a.push(1, half - 1);
    AdmitDecision d = a.admit();
    CHECK(d.count == 1);
    AdmitDecision e = a.admit();
    CHECK(e.count == 2);   // 2^30 + 2^30 - 1 = 2^31 - 1 is allowed
    Admission b(1, 100, 8);
    b.push(1, Admission::kMaxNodes);  // one request may use the whole range
    CHECK(b.admit().count == 1);
}

static void trimming()
{
    Admission a(3, 1000, 1);
    // three slots each end up holding 300
    std::vector<int> slots;
    for (int i = 0; i < 3; ++i) {
        a.push(300, 1);
        AdmitDecision d = a.admit();
        CHECK(d.trim.empty());
        CHECK(a.built(d.slot, 300));
        slots.push_back(d.slot);
    }
    for (int s : slots) a.release(s);
    CHECK(a.used() == 900);
    // a 700-byte group: the build slot keeps its 300 (charged 300 + 700)
    // only if the other two are trimmed: 1000 <= budget
    a.push(700, 1);
    CHECK(a.can_admit());
    AdmitDecision d = a.admit();
    CHECK(d.trim.size() == 2);
    for (int t : d.trim) CHECK(t != d.slot);
    CHECK(a.used() == 1000 && a.used() <= a.budget());
    for (int t : d.trim) a.trimmed(t);
    CHECK(a.built(d.slot, 700));
    CHECK(a.used() == 700);
    a.release(d.slot);
    // a 1000-byte group needs the build slot itself trimmed
    a.push(1000, 1);
    AdmitDecision e = a.admit();
    CHECK(e.slot == d.slot);  // the largest holding is chosen
    CHECK(e.trim.size() == 1 && e.trim[0] == e.slot);
    CHECK(a.used() == 1000);
}

static void misuse_is_rejected()
{
    Admission a(1, 10, 1);
    bool threw = false;
    try {
        a.admit();
    } catch (const std::logic_error &) {
        threw = true;
    }
    CHECK(threw);
    threw = false;
    try {
        a.release(0);  // idle, not running
    } catch (const std::logic_error &) {
        threw = true;
    }
    CHECK(threw);
    threw = false;
    try {
        a.push(1, 0);
    } catch (const std::invalid_argument &) {
        threw = true;
    }
    CHECK(threw);
    threw = false;
    try {
        Admission b(0, 10, 1);
    } catch (const std::invalid_argument &) {
        threw = true;
    }
    CHECK(threw);
}

// Random arrivals and completions against the fake engine: the bytes the
// slots really hold never exceed the charges, the charges never exceed the
// budget, every build stays within its charge, groups keep arrival order,
// and every request is served.
static void simulation(uint64_t seed, int slots, int64_t budget, int32_t max_group, int n_req)
{
    std::mt19937_64 rng(seed);
    const int NB = 6;  // buffers per slot
    std::vector<std::vector<int64_t>> caps((size_t)slots, std::vector<int64_t>(NB, 0));
    auto held = [&](int s) {
        int64_t b = 0;
        for (int64_t c : caps[(size_t)s]) b += c;
        return b;
    };
    Admission a(slots, budget, max_group);
    std::uniform_int_distribution<int64_t> fp_d(1, budget / 3);
    std::vector<int64_t> fps;
    int next = 0, served = 0, admitted = 0;
    struct Run {
        int slot;
        int64_t fp;
        int left;
        bool built;
    };
    std::vector<Run> running;
    int guard = 0;
    while (served < n_req && ++guard < 1000000) {
        // arrivals
        if (next < n_req && rng() % 3 == 0) {
            fps.push_back(fp_d(rng));
            a.push(fps.back(), 1 + (int64_t)(rng() % 1000));
            ++next;
        }
        // admissions
        if (a.can_admit() && rng() % 2 == 0) {
            AdmitDecision d = a.admit();
            int64_t sum = 0;
            for (int i = 0; i < d.count; ++i) sum += fps[(size_t)admitted + i];
            CHECK(sum == d.footprint);  // the first waiting requests, in order
            admitted += d.count;
            for (int t : d.trim) {
                for (int64_t &c : caps[(size_t)t]) c = 0;
                if (t != d.slot) a.trimmed(t);
            }
            running.push_back({d.slot, d.footprint, d.count, false});
        }
        // builds end: ask for a random split of at most the footprint
        for (Run &r : running) {
            if (r.built || rng() % 2) continue;
            int64_t left = r.fp;
            for (int b = 0; b < NB && left > 0; ++b) {
                const int64_t ask = b + 1 == NB ? left : (int64_t)(rng() % (uint64_t)(left + 1));
                left -= ask;
                int64_t &c = caps[(size_t)r.slot][(size_t)b];
                c = std::max(c, ask);  // exact growth, kept afterwards
            }
            CHECK(a.built(r.slot, held(r.slot)));
            r.built = true;
        }
        // the real holdings never exceed the charges
        int64_t total = 0;
        for (int s = 0; s < slots; ++s) total += held(s);
        CHECK(total <= a.used());
        CHECK(a.used() <= budget);
        // groups finish
        for (size_t i = 0; i < running.size();) {
            if (running[i].built && rng() % 4 == 0) {
                served += running[i].left;
                a.release(running[i].slot);
                running[i] = running.back();
                running.pop_back();
            } else {
                ++i;
            }
        }
    }
    CHECK(served == n_req);
    CHECK(a.peak() <= budget);
    CHECK(a.waiting() == 0);
}

int main()
{
    budget_edges();
    max_group_and_order();
    node_limit();
    trimming();
    misuse_is_rejected();
    for (uint64_t seed = 1; seed <= 20; ++seed)
        simulation(seed, 1 + (int)(seed % 6), 10000 + 997 * (int64_t)seed, 1 + (int32_t)(seed % 8),
                   300);
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("admission ok\n");
    return 0;
}
