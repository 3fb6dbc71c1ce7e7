// Internal batch hooks used by the serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fitnll.h"

namespace fn {
hipStream_t batch_stream(fn_batch* b);
int batch_params(fn_batch* b);
int batch_slots(fn_batch* b);
void batch_set_slot_async(fn_batch* b, int slot, const double* ev, int64_t n, const double* theta0);
void batch_steps(fn_batch* b, int k);
void batch_poll(fn_batch* b, int* stat_host);
void batch_read_rows(fn_batch* b, const int* slots, int n, double* rows_host);
}  // namespace fn
