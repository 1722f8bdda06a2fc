// Diagnostic per-kernel timing shared by plans and batch plans: HIP event
// pairs recorded around kernel launches on the launch stream.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "lens_api.h"

// Event pairs around kernel launches of one plan (diagnostic timing).
struct KernelTimer {
    static constexpr int kMaxRecords = 65536;
    bool enabled = false;
    bool capturing = false;
    std::vector<hipEvent_t> ev[LENS_NUM_KERNEL_SLOTS];
    int used[LENS_NUM_KERNEL_SLOTS] = {0};
    int64_t count[LENS_NUM_KERNEL_SLOTS] = {0};

    hipEvent_t take(int slot) {
        auto& v = ev[slot];
        if (used[slot] >= (int)v.size()) {
            if ((int)v.size() >= 2 * kMaxRecords) return nullptr;
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            v.push_back(e);
        }
        return v[used[slot]++];
    }
    // Totals per slot since the last read (synchronises on the events), then reset.
    lens_status read(double* h_ms, int64_t* h_count) {
        lens_status st = LENS_OK;
        for (int k = 0; k < LENS_NUM_KERNEL_SLOTS; ++k) {
            double tot = 0.0;
            for (int r = 0; r + 1 < used[k]; r += 2) {
                if (hipEventSynchronize(ev[k][r + 1]) != hipSuccess) return LENS_EHIP;
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[k][r], ev[k][r + 1]) != hipSuccess) return LENS_EHIP;
                tot += ms;
            }
            if (count[k] * 2 > used[k]) st = LENS_EUNSUPPORTED;
            h_ms[k] = tot;
            h_count[k] = count[k];
            used[k] = 0;
            count[k] = 0;
        }
        return st;
    }
    void release() {
        for (auto& v : ev)
            for (auto e : v) (void)hipEventDestroy(e);
        for (auto& v : ev) v.clear();
    }
};

// Records start/stop events around one launch when timing is enabled.
struct TimedLaunch {
    KernelTimer* t;
    int slot;
    hipStream_t st;
    hipEvent_t stop = nullptr;
    TimedLaunch(KernelTimer* t_, int slot_, hipStream_t st_) : t(t_), slot(slot_), st(st_) {
        if (!t->enabled || t->capturing) return;
        t->count[slot]++;
        hipEvent_t start = t->take(slot);
        stop = start ? t->take(slot) : nullptr;
        if (start && stop) (void)hipEventRecord(start, st);
        else stop = nullptr;
    }
    ~TimedLaunch() {
        if (stop) (void)hipEventRecord(stop, st);
    }
};

