// Internal batch hooks used by the serving loop.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/fitnll.h"
#include "batch.hpp"

namespace fn {
hipStream_t batch_stream(fn_batch* b);
int batch_params(fn_batch* b);
int batch_slots(fn_batch* b);
void batch_admit_async(fn_batch* b, const AdmitRec* recs_host, int n, int64_t gen_blocks, double lo, double hi,
                       unsigned int* n_unresolved);
void batch_steps(fn_batch* b, int k);
void batch_poll(fn_batch* b, int* stat_host);
void batch_read_rows(fn_batch* b, const int* slots, int n, double* rows_host);
}  // namespace fn
