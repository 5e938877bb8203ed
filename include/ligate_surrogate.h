/*
 * ligate_surrogate.h - C ABI of the learned pre-filter of the docking screen.
 *
 * The operation (paper §3.5, machine-learning engines; §2, the AI engine fed by data the
 * workflow generates in silico): a cheap model, trained on docking scores produced by the
 * screen itself, predicts each ligand's best score so that only the most promising fraction
 * of a library is docked.
 *
 * Model: per-ligand features (512 FP32: 16 rows of 32 = per-type atom count, 30-bin histogram
 * of distances from that type's atoms to every other atom, rotatable-bond count; log1p; z-score),
 * then y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3 with widths d_in -> h1 -> h2 -> 1.  Weights are
 * BF16 copies of FP32 master weights, the input and hidden layers are stored in BF16, all sums
 * are FP32 on the matrix cores.  Training: mean squared error, Adam.
 *
 * Conventions are those of ligate_dock.h: device pointers d_*, caller-owned memory, workspaces
 * sized by a query (d_ws == NULL), asynchronous on `stream`, capture-safe, synchronous argument
 * errors (DOCK_ERR_* codes).
 */
#ifndef LIGATE_SURROGATE_H
#define LIGATE_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SURR_FEATURES 512 /* 16 rows x 32 slots */
#define SURR_MAX_TYPES 16

/*
 * A model.  All pointers are device memory owned by the caller.
 * d_master: FP32 master weights, flat [W1 (h1 x d_in, row-major), b1 (h1), W2 (h2 x h1), b2 (h2),
 *           w3 (h2), b3 (1)]; d_grad, d_adam_m, d_adam_v: the same layout.
 * d_bf16:   BF16 copies [W1, W2, w3] (bit patterns as uint16), refreshed by surr_cast / surr_adam.
 * d_in, h1 and h2 must be multiples of 64.
 */
typedef struct {
    int32_t d_in, h1, h2;
    float *d_master;
    uint16_t *d_bf16;
    float *d_grad;
    float *d_adam_m, *d_adam_v;
} surr_model;

/* Number of FP32 master values and of BF16 weight values of a model. */
int surr_param_count(int32_t d_in, int32_t h1, int32_t h2, int64_t *n_master, int64_t *n_bf16);

/*
 * Features of every ligand of a packed library (dock_pack_ligands), from the input CSR
 * coordinates and types (the same arrays given to the packer).  Row t: slot 0 = number of
 * type-t atoms, slots 1..30 = ordered-pair counts of distances from type-t atoms to every other
 * atom in 0.5 A bins on [1.25, 16.25) A (ends folded in; the bin is decided on the FP32 squared
 * distance against the exact squared edges), slot 31 = rotatable-bond count; then log1p.  If
 * d_mean and d_istd are given, (f - mean) * istd.  Ligands whose status is not OK get zeros,
 * and so does a ligand holding an atom type >= 16 (a pack built with more types than the
 * features have rows).  The bin of a pair within about 1e-6 A of an inner edge is decided by
 * FP32 rounding and may be either neighbour.
 * Outputs (either may be NULL): d_feat [n_lig][512] FP32, d_feat_bf16 [n_lig][512] BF16 bits.
 * Requires n_types <= 16.
 */
int surr_features(const int32_t *d_atom_off, const float *d_xyz, const uint8_t *d_type, const void *d_pack,
                  int32_t n_lig, int64_t n_atoms_total, int32_t n_types, const float *d_mean, const float *d_istd,
                  float *d_feat, uint16_t *d_feat_bf16, void *stream);

/* Per-column mean and 1/std (population std; 1 where std is 0) of d_feat [n_rows][512]. */
int surr_feature_stats(const float *d_feat, int64_t n_rows, float *d_mean, float *d_istd, void *d_ws,
                       size_t *ws_bytes, void *stream);

/* Refreshes the BF16 weight copies from the FP32 master weights (round to nearest even). */
int surr_cast(const surr_model *m, void *stream);

/* Predictions d_y [batch] for inputs d_x [batch][d_in] (BF16 bits).  batch >= 1. */
int surr_forward(const surr_model *m, const uint16_t *d_x, int32_t batch, float *d_y, void *d_ws,
                 size_t *ws_bytes, void *stream);

/*
 * Forward and backward pass of the mean squared error against targets d_t [batch]: writes the
 * gradient of every master value to m->d_grad and the loss to d_loss [1].  batch must be a
 * multiple of 32.
 */
int surr_backward(const surr_model *m, const uint16_t *d_x, const float *d_t, int32_t batch, float *d_loss,
                  void *d_ws, size_t *ws_bytes, void *stream);

/*
 * One Adam step (Kingma and Ba, 2015; bias-corrected, no weight decay) on the master weights
 * from m->d_grad, step = 1, 2, ...; then refreshes the BF16 copies.
 */
int surr_adam(const surr_model *m, float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/*
 * Minibatch assembly: rows d_idx[i] of d_x [*][row] (BF16 bits) and of d_t [*] go to row i of
 * d_x_out and d_t_out.  Either pair may be NULL.  Indices must be valid rows of the inputs.
 */
int surr_gather(const uint16_t *d_x, const float *d_t, const int32_t *d_idx, int64_t n_idx, int32_t row,
                uint16_t *d_x_out, float *d_t_out, void *stream);

/*
 * Ensemble prediction (paper §3.5: the cheap model here is an ensemble of networks): d_out[i] =
 * (d_y[0][i] + d_y[1][i] + ... + d_y[n_members-1][i]) / n_members, summed in member order in
 * FP32.  d_y is [n_members][n] (each member's surr_forward output, rows contiguous).
 * 1 <= n_members <= 64, n >= 0.
 */
int surr_average(const float *d_y, int32_t n_members, int64_t n, float *d_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LIGATE_SURROGATE_H */
