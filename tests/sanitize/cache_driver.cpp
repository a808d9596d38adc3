// Host-side check of the autotune cache parser under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_sanitizers.py, no GPU):
// malformed, truncated, overlong and out-of-range lines must be skipped or
// read without touching memory outside their buffers, and the last valid
// entry for a key wins.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "kc_internal.h"

// The parser maps a cached depth to a compiled one through the kernel table,
// which this host-only build does not link; the depths used here are compiled.
namespace kc {
int stream_depth_at_most(int t, int) { return t; }
} // namespace kc

static int fails = 0;
#define CHECK(c)                                                                                 \
    do {                                                                                         \
        if (!(c)) {                                                                              \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);                         \
            ++fails;                                                                             \
        }                                                                                        \
    } while (0)

int main(int argc, char **argv)
{
    if (argc < 2)
        return 2;
    const char *path = argv[1];
    setenv("KC_AUTOTUNE_CACHE", path, 1);
    FILE *f = fopen(path, "w");
    if (!f)
        return 2;
    const char *key = "gfx950:sramecc+:xnack-|128x128|fp32|receptor";
    std::string longline(3000, 'x');
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": 2, \"rows\": 8, \"prefetch\": 2, \"gcell_s\": 3.5}\n", key);
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": 9, \"rows\": 8, \"prefetch\": 2}\n", key);   // bad depth
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": 4, \"rows\": -1, \"prefetch\": 2}\n", key);  // bad rows
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": 4, \"rows\": 8, \"prefetch\": 3}\n", key);   // bad pf
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": 4, \"rows\": 8, \"prefetch\": 4, \"waves\": 7}\n", key);
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": \n", key);                                    // truncated
    fprintf(f, "{\"key\": \"%s\", %s}\n", key, longline.c_str());                          // overlong
    fprintf(f, "{\"key\": \"%s|rk2\", \"tsteps\": 3, \"rows\": 16, \"prefetch\": 4}\n", key);
    fprintf(f, "garbage \"key\": \"\" \"tsteps\": 99999999999999999999 \"rows\":\n");
    fprintf(f, "{\"key\": \"%s\", \"tsteps\": 99999999999999999999, \"rows\": 8, \"prefetch\": 2}\n", key);
    fprintf(f, "%s", "{\"key\": \"no newline at end\"");
    fclose(f);

    kc::Tuning t;
    double g = -1.0;
    CHECK(kc::cache_lookup(key, 0, &t, &g));
    CHECK(t.tsteps == 2 && t.rows == 8 && t.prefetch == 2 && t.waves == 1 && g == 3.5);
    std::string rk = std::string(key) + "|rk2";
    CHECK(kc::cache_lookup(rk.c_str(), 1, &t, &g));
    CHECK(t.tsteps == 3 && t.rows == 16 && t.prefetch == 4 && g == 0.0);
    CHECK(!kc::cache_lookup("gfx950|nothing", 0, &t, nullptr));

    // a stored entry is appended and wins over the earlier one
    kc::Tuning s;
    s.tsteps = 4;
    s.rows = 35;
    s.prefetch = 4;
    s.waves = 2;
    kc::cache_store(key, s, 812.25);
    CHECK(kc::cache_lookup(key, 0, &t, &g));
    CHECK(t.tsteps == 4 && t.rows == 35 && t.prefetch == 4 && t.waves == 2 && g == 812.25);

    // no cache path: nothing read or written
    unsetenv("KC_AUTOTUNE_CACHE");
    CHECK(!kc::cache_lookup(key, 0, &t, &g));
    kc::cache_store(key, s, 1.0);
    printf("cache driver: %d failed checks\n", fails);
    return fails ? 1 : 0;
}
