// batched_copy.h -- the label copies that close a batched fit whose
// instances ran as several work items (restart groups, km_schedule::
// restart_group): the kept restart's labels, written by its item into a
// workspace buffer, go to the caller's labels_out.  Internal to
// libkmeans_mi355x.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace km {

struct BCopy {
    const int32_t* src;  // device, n labels
    int32_t* dst;        // device, n labels
    int64_t n;
};

// Copies every entry of tab[0..n) (device); one launch.
hipError_t launch_batched_copy_labels(const BCopy* tab, int n, hipStream_t s);

}  // namespace km
