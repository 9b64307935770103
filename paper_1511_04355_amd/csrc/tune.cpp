// Autotuning table: (device, kernel, size, variant) -> chosen candidate, with
// the times measured for every candidate kept for the report.
#include "tune.hpp"

#include <map>
#include <mutex>
#include <sstream>
#include <tuple>

namespace afsbem {

namespace {

struct Entry {
    int choice = 0;
    std::vector<std::pair<int, float>> times;  // candidate, ms per run
};

std::mutex g_mu;
bool g_enabled = true;
std::map<std::tuple<int, std::string, int64_t, int>, Entry> g_table;

}  // namespace

void autotune_set_enabled(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_enabled = on;
}

int autotune(const char *kernel, int64_t n, int variant, const std::vector<int> &cands, hipStream_t st,
             const std::function<void(int)> &run, int fallback, int reps) {
    int dev = 0;
    AFS_HIP(hipGetDevice(&dev));
    const auto key = std::make_tuple(dev, std::string(kernel), n, variant);
    {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_table.find(key);
        if (it != g_table.end())
            return it->second.choice;
        if (!g_enabled || cands.empty())
            return fallback;
    }
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    AFS_HIP(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone)
        return fallback;
    hipEvent_t e0, e1;
    AFS_HIP(hipEventCreate(&e0));
    AFS_HIP(hipEventCreate(&e1));
    Entry ent;
    float best = 0.f;
    try {
        for (int c : cands) {
            run(c);
            AFS_HIP(hipEventRecord(e0, st));
            for (int r = 0; r < reps; ++r)
                run(c);
            AFS_HIP(hipEventRecord(e1, st));
            AFS_HIP(hipEventSynchronize(e1));
            float ms = 0.f;
            AFS_HIP(hipEventElapsedTime(&ms, e0, e1));
            ms /= (float)reps;
            ent.times.push_back({c, ms});
            if (ent.times.size() == 1 || ms < best) {
                best = ms;
                ent.choice = c;
            }
        }
    } catch (...) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        throw;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    std::lock_guard<std::mutex> lk(g_mu);
    g_table[key] = ent;
    return ent.choice;
}

std::string autotune_report() {
    std::lock_guard<std::mutex> lk(g_mu);
    std::ostringstream os;
    for (const auto &kv : g_table) {
        os << "device " << std::get<0>(kv.first) << " " << std::get<1>(kv.first) << " n=" << std::get<2>(kv.first)
           << " variant=" << std::get<3>(kv.first) << " -> " << kv.second.choice << " |";
        for (const auto &t : kv.second.times)
            os << " " << t.first << ":" << t.second << "ms";
        os << "\n";
    }
    return os.str();
}

}  // namespace afsbem
