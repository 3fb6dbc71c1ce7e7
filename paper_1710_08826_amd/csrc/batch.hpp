// Batched fits: per-fit minimizer state and the device buffers of a batch.
#pragma once
#include "kernels.hpp"
#include "bfgs_device.hpp"
#include "mix1d_device.hpp"

namespace fn {

constexpr int kBatchMaxP = 24;      // parameters per batched fit
constexpr int kGenMaxAttempts = 64; // redraws per generated event

using BfgsState = BfgsStateT<kBatchMaxP>;

// Device pointers of a batch (n_fits slots).
struct BatchDev {
  BfgsState* st;
  Mix1dTable* tabs;
  const double** ev;       // event pointer per slot
  int64_t* nev;            // events per slot
  int64_t* item_base;      // n_fits + 1
  int64_t* part_base;      // first partial row of each slot
  double* part;            // partial rows
  double* out;             // per slot [NLL, grad(P), I, dI(P)]
  int* n_running;
  int* stat;               // per slot status, mirrored every step
  double* rres;            // per slot result row, written when the fit retires (3 + 2P)
};

void batch_launch_step(const BatchDev& b, const Mix1dConst& mc, int n_fits, int P, int chunk, int eval_grid,
                       double tol, int max_iter, hipStream_t s);
int batch_eval_blocks_per_cu(const Mix1dConst& mc);
void batch_launch_gen_mix1d(uint32_t k0, uint32_t k1, uint32_t word, int64_t n, const double* theta_gen, double lo,
                            double hi, double* x, unsigned int* n_unresolved, hipStream_t s);

}  // namespace fn
