/*
 * mlp.h — C ABI of the learned closure of the DIG synthetic equations.
 *
 * A multilayer perceptron predicts the higher-order terms (HoT) of the
 * macroscopic equations (the quantities eq. hot_extraction_ch3 defines as
 * the DSMC stress and heat flux minus their NSF values) from local
 * gradients, so that the coupling step (Algorithm 1) can take a smooth
 * prediction where the sampled HoT is noisy.  This closure is an addition
 * of this library, not part of the paper's method; the plain sampled HoT
 * stays the fallback and the test every prediction must pass
 * (dig_set_closure).
 *
 * Network: 13 inputs -> 128 -> 128 -> 128 -> 9 outputs, SiLU on the hidden
 * layers.  Inputs per cell, nondimensional: lambda du_i/dx_j / sqrt(RT)
 * (i, j = x, y, z, row-major, 9 values), lambda dT/dx_j / T (3 values) and
 * Kn_Delta (eq. cell_kn_stability), with lambda the local mean free path
 * (Kn_Delta times the cell diameter d_c).  Outputs: HoT stresses over p
 * (xx, yy, zz, xy, xz, yz) and HoT heat fluxes over p sqrt(RT) (x, y, z).
 *
 * Parameters: one FP32 vector of 35,977 values, for each layer l = 1..4 the
 * weights W_l[in][out] row-major followed by the biases b_l[out].
 *
 * Arithmetic: products on the BF16 matrix cores with FP32 accumulation
 * (inputs, weights, hidden activations and pre-activation gradients are
 * rounded to bfloat16, nearest even); biases, SiLU, the loss, its bias
 * gradients and the Adam optimiser in FP32 on FP32 master weights.
 * Loss: mean squared error over all n x 9 outputs.
 *
 * Conventions of dsmc.h: status codes, host arrays unless stated, calls
 * synchronise the network's stream, dsmc_mlp_last_error() explains a failure.
 */
#ifndef DSMC_MLP_H
#define DSMC_MLP_H

#include "dsmc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DSMC_MLP_INPUTS 13
#define DSMC_MLP_OUTPUTS 9
#define DSMC_MLP_PARAMS 35977

typedef struct dsmc_mlp_s* dsmc_mlp;

typedef struct {
    int32_t steps;   /* optimiser steps */
    int32_t batch;   /* rows per step; >= n (or 0) uses the whole set every step */
    float lr;        /* Adam step size */
    float beta1, beta2, eps;
    uint64_t seed;   /* minibatch draws: generator purpose 8, keyed by (seed, 0) */
} dsmc_mlp_train_params;

typedef struct {
    int32_t steps;
    double loss_first;  /* loss of the first minibatch */
    double loss_last;   /* loss of the last minibatch (before its update) */
} dsmc_mlp_train_report;

/* New network with zero weights on a HIP stream (NULL: null stream); device
 * memory through the allocator (NULL: hipMalloc).  The Adam moments start at
 * zero and persist across dsmc_mlp_train calls (reset by set_weights). */
dsmc_status dsmc_mlp_create(dsmc_mlp* out, void* hip_stream, const dsmc_allocator* allocator);
dsmc_status dsmc_mlp_set_weights(dsmc_mlp net, const float* params);
/* Random initial weights, uniform in (-1, 1) / sqrt(fan_in), zero biases
 * (generator purpose 8 keyed by (seed, 1), subject = parameter index). */
dsmc_status dsmc_mlp_init_weights(dsmc_mlp net, uint64_t seed);
dsmc_status dsmc_mlp_get_weights(dsmc_mlp net, float* params);

/* y[n][9] = network(x[n][13]); x and y are device pointers if on_device. */
dsmc_status dsmc_mlp_forward(dsmc_mlp net, const float* x, int64_t n, float* y, int32_t on_device);

/* Gradient of the mean squared error over the n rows of (x, t[n][9]):
 * grad[35977] (layout of the parameters) and *loss. */
dsmc_status dsmc_mlp_backward(dsmc_mlp net, const float* x, const float* t, int64_t n, float* grad, double* loss);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * gradient of dsmc_mlp_backward with every array in device memory and no
 * allocation, host synchronisation or host copy.  x[rows][13], t[rows][9]
 * (inputs), grad[35977] and *loss (the mean squared error, outputs) are
 * device pointers the caller owns; rows must be between 1 and
 * DSMC_MLP_NOALLOC_MAX_ROWS (DSMC_E_INVALID otherwise).  The work is
 * enqueued on the network's stream and the call returns at once.  Its
 * per-block partials live in a fixed scratch array of the library
 * (DSMC_MLP_NOALLOC_MAX_ROWS / 32 blocks of 35,977 floats, 18.4 MB, held on
 * each device that creates a network until the process ends) shared by
 * every call on that device: calls that overlap on one device race, so the
 * caller orders them (one stream, or events).  Results equal
 * dsmc_mlp_backward's on the same rows. */
#define DSMC_MLP_NOALLOC_MAX_ROWS 4096
dsmc_status dsmc_mlp_backward_noalloc(dsmc_mlp net, const float* x, const float* t, int64_t rows, float* grad,
                                      double* loss);

/* One Adam step with a caller-given gradient grad[35977]. */
dsmc_status dsmc_mlp_adam_step(dsmc_mlp net, const float* grad, float lr, float beta1, float beta2, float eps);

/* Minibatch Adam on the set (x[n][13], t[n][9]) copied to the device. */
dsmc_status dsmc_mlp_train(dsmc_mlp net, const float* x, const float* t, int64_t n,
                           const dsmc_mlp_train_params* params, dsmc_mlp_train_report* report);

const char* dsmc_mlp_last_error(dsmc_mlp net);
void dsmc_mlp_destroy(dsmc_mlp net);

/* Closure of the coupling step (dig_couple): with a network, every cell with
 * samples gets the network's HoT when its distance to the sampled HoT is at
 * most gate_tol times max(sqrt(s^2 + 14.5 / n), 1e-3), with s =
 * |(sigma/p, q/(p sqrt(RT)))| of the samples and n the particle samples of
 * the moving average (mean particles per step x min(samples taken, n_a)):
 * 14.5 / n is the expected squared sampling error of that vector in an
 * equilibrium gas, so a network within a few noise widths of the window's
 * own HoT is accepted; otherwise (or with net NULL) the sampled HoT.  The network
 * must stay alive while it is attached.  The report of dig_couple counts
 * the cells that took the network (n_closure) and fell back (n_fallback). */
dsmc_status dig_set_closure(dsmc_ctx ctx, dsmc_mlp net, double gate_tol);

/* The closure's training pairs of the last dig_couple in caller cell order:
 * x[n_tets][13] inputs, t[n_tets][9] nondimensional sampled HoT, valid[n_tets]
 * (1 where the cell had samples). */
dsmc_status dig_closure_data(dsmc_ctx ctx, float* x, float* t, uint8_t* valid);

#ifdef __cplusplus
}
#endif
#endif /* DSMC_MLP_H */
