// Autotuner for the kernel variants of a context (tile shapes of the stencil
// kernel, output tile and inner chunk of the batched rank-k update).  Each
// tuned family is timed once per size class on the device, and the fastest
// variant is kept; results can be cached in a JSON file so that later
// contexts with the same device and size class reuse them without timing.
//
// Cache format (one object per tuned family and size class):
//   {"format": "bidomain-tune-1",
//    "entries": [{"device": "gfx950", "family": "stencil", "class": "...",
//                 "choice": 0, "ms": [0.12, 0.13]}, ...]}
#pragma once
#include <functional>
#include <string>
#include <vector>

namespace bdm {

struct TuneEntry {
    std::string device, family, cls;
    int choice = 0;
    std::vector<double> ms;     // time of each variant (ms; negative: not run)
    bool cached = false;        // taken from the cache file, not timed here
};

class Tuner {
public:
    std::string device;               // device name the entries are keyed by
    std::vector<TuneEntry> entries;   // cache contents plus this context's results
    std::vector<int> used;            // entries this context chose from
    bool dirty = false;               // new results not yet saved

    // Read a cache file; a missing file is not an error.  Returns an empty
    // string on success, else a message (the cache is then ignored).
    std::string load(const std::string& path);
    // Write every entry to path (atomically: temporary file, then rename).
    std::string save(const std::string& path) const;
    // Variant for (family, cls): the cached choice when there is one (and it
    // is < nvar), else the fastest of time_ms(0..nvar-1) (time_ms returns
    // milliseconds, or a negative value for a variant that cannot run).
    int pick(const std::string& family, const std::string& cls, int nvar,
             const std::function<double(int)>& time_ms);
    // JSON of the entries this context used.
    std::string report() const;
};

// JSON helpers shared by load/report (exposed for tests of the format).
std::string tune_to_json(const std::vector<TuneEntry>& e);
std::string tune_from_json(const std::string& text, std::vector<TuneEntry>& out);

}  // namespace bdm
