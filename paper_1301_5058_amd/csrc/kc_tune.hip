// kc_tune.hip -- autotuner cache (host side).
//
// Cache file: one JSON object per line,
//   {"key": "<arch>|<nx>x<ny>|fp32|receptor", "tsteps": T, "rows": R, "prefetch": P,
//    "waves": W, "gcell_s": G}
// (an entry without "waves" has one wavefront per strip)
// The path comes from the environment variable KC_AUTOTUNE_CACHE; without it
// nothing is read or written.  A later line with the same key wins.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>

#include "kc_internal.h"

namespace kc {

int device_key(char *buf, size_t n, int nx, int ny, int precision, int chi_law, int integrator,
               bool noise)
{
    int dev = 0;
    hipDeviceProp_t prop;
    const char *arch = "unknown";
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    char a[64];
    snprintf(a, sizeof a, "%s", arch);
    for (char *p = a; *p; ++p)
        if (*p == '"' || *p == '|' || *p == ' ')
            *p = '_';
    // forward-Euler keys carry no integrator field; Runge-Kutta keys add "|rk2",
    // per-step noise "|noise"
    return snprintf(buf, n, "%s|%dx%d|%s|%s%s%s", a, nx, ny, precision == 0 ? "fp32" : "fp64",
                    chi_law == 0 ? "receptor" : "constant", integrator == 0 ? "" : "|rk2",
                    noise ? "|noise" : "");
}

static const char *cache_path() { return getenv("KC_AUTOTUNE_CACHE"); }

bool cache_lookup(const char *key, int integrator, Tuning *t, double *gcells)
{
    const char *path = cache_path();
    if (!path || !*path)
        return false;
    FILE *f = fopen(path, "r");
    if (!f)
        return false;
    char line[512];
    bool found = false;
    const std::string want = std::string("\"key\": \"") + key + "\"";
    while (fgets(line, sizeof line, f)) {
        if (!strstr(line, want.c_str()))
            continue;
        int T = 0, R = 0, P = 0, W = 1;
        const char *pt = strstr(line, "\"tsteps\":");
        const char *pr = strstr(line, "\"rows\":");
        const char *pp = strstr(line, "\"prefetch\":");
        const char *pw = strstr(line, "\"waves\":");
        if (pw && sscanf(pw, "\"waves\": %d", &W) != 1)
            W = 1;
        if (pt && pr && pp && sscanf(pt, "\"tsteps\": %d", &T) == 1 &&
            sscanf(pr, "\"rows\": %d", &R) == 1 && sscanf(pp, "\"prefetch\": %d", &P) == 1 &&
            T >= 1 && T <= 8 && R >= 1 && (P == 2 || P == 4) && (W == 1 || W == 2)) {
            t->tsteps = stream_depth_at_most(T, integrator);
            t->rows = R;
            t->prefetch = P;
            t->waves = W;
            double g = 0.0;
            const char *pg = strstr(line, "\"gcell_s\":");
            if (pg && sscanf(pg, "\"gcell_s\": %lf", &g) != 1)
                g = 0.0;
            if (gcells)
                *gcells = g;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *key, const Tuning &t, double gcells)
{
    const char *path = cache_path();
    if (!path || !*path)
        return;
    FILE *f = fopen(path, "a");
    if (!f)
        return;
    fprintf(f,
            "{\"key\": \"%s\", \"tsteps\": %d, \"rows\": %d, \"prefetch\": %d, \"waves\": %d, "
            "\"gcell_s\": %.3f}\n",
            key, t.tsteps, t.rows, t.prefetch, t.waves, gcells);
    fclose(f);
}

} // namespace kc
