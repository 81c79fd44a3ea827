/*
 * poredvm_unet: the learned warm start of the iteration of poredvm.h.
 *
 * The iteration (Sec. 3.1, Algorithm 1) takes its initial density and velocity
 * fields as input and leaves them open (the paper starts from given initial
 * conditions). This network predicts them from the solid mask and Kn. It is a
 * 4-level U-Net (32, 64, 128, 256 channels; two 3x3 convolutions with ReLU per
 * level; 2x2 max pooling; nearest upsampling with skip concatenation; a 1x1
 * head to 3 outputs), trained on fields that the iteration itself converged.
 * The iteration stays unchanged, so a poor guess costs iterations, never
 * correctness; callers compare the guess against rest and keep the better one.
 *
 * Arithmetic: bfloat16 weights and activations (round to nearest even),
 * FP32 accumulation on the matrix cores, FP32 biases, master weights and
 * Adam state. Padding is circular along x1 (the periodic flow axis) and zero
 * along x2.
 *
 * Inputs per voxel: solid (0/1) and f = ln(Kn * N1 / 256) / 3, where Kn is
 * referenced to the sample's x1 length N1 (as in poredvm.h), so f uses a fixed
 * 256-voxel reference.
 * Outputs (normalised, zero on solid voxels), with g = 256 J / N1 (J = the
 * pressure jump) and sigma = 10 K / (1 + 10 K), K = Kn N1 / 256:
 *   t0 = (rho + J (x1 - 1/2) - its fluid mean) / g,   x1 = (i + 1/2) / N1,
 *   t1, t2 = 10 sigma u_j / g.
 * Predicted physical fields take mean density 0 (the density level is a free
 * constant of the problem).
 *
 * Parameter vector (FP32, pdvm_unet_num_params() values): for each layer in
 * the order enc1a, enc1b, enc2a, enc2b, enc3a, enc3b, bott_a, bott_b, dec3a,
 * dec3b, dec2a, dec2b, dec1a, dec1b, head: weights [Cout][taps][Cin] then
 * biases [Cout]. Cin of enc1a is 8 (solid, f, six zero channels); a decoder's
 * first layer reads [upsampled deeper features, skip features] in that order.
 *
 * Status codes are those of poredvm.h. Device work runs on the stream given
 * at creation; calls that return host data synchronise it.
 */
#ifndef POREDVM_UNET_H
#define POREDVM_UNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdvm_unet pdvm_unet;

/* Number of FP32 parameters of the network. */
int64_t pdvm_unet_num_params(void);

/* A network instance for images of n2 x n1 voxels (each a multiple of 8),
 * batches of up to batch_max (<= 32) and a device-resident training set of
 * up to dataset_max samples. hip_stream: a hipStream_t or NULL (private
 * stream). Parameters start at zero: set them before use. */
int pdvm_unet_create(int32_t n1, int32_t n2, int32_t batch_max, int32_t dataset_max, void *hip_stream,
                     pdvm_unet **out);

/* Host FP32 parameter vectors in the layout above (n must equal
 * pdvm_unet_num_params()). set_params also resets the Adam state. */
int pdvm_unet_set_params(pdvm_unet *net, const float *params, int64_t n);
int pdvm_unet_get_params(pdvm_unet *net, float *params, int64_t n);

/* Store training sample `slot` (0 <= slot < dataset_max): the solid mask
 * (n1*n2 bytes, x1 fastest), Kn, J and the converged fields rho (N doubles)
 * and u (2N doubles, component-major) of the iteration; the normalised targets
 * are computed on the device. */
int pdvm_unet_set_sample(pdvm_unet *net, int32_t slot, const uint8_t *solid, double kn, double jump,
                         const double *rho, const double *u);

/* One training step over the samples slots[0..batch): forward pass, loss
 * L = mean over the batch of (1 / (3 n_fluid)) sum over fluid voxels and the
 * three outputs of (prediction - target)^2, backward pass (gradients of L in
 * FP32), then, if update != 0, one Adam step (beta1 0.9, beta2 0.999,
 * eps 1e-8, learning rate lr). *loss receives L (may be NULL). */
int pdvm_unet_train_step(pdvm_unet *net, const int32_t *slots, int32_t batch, float lr, int32_t update,
                         double *loss);

/* Gradients of the last train_step, same layout as the parameters. */
int pdvm_unet_get_grads(pdvm_unet *net, float *grads, int64_t n);

/* Forward pass only: normalised outputs of slots[0..batch) into out
 * (batch * n2 * n1 * 4 floats: per voxel t0, t1, t2, 0). */
int pdvm_unet_forward(pdvm_unet *net, const int32_t *slots, int32_t batch, float *out);

/* Warm-start fields for one image of the instance's size: rho (N doubles)
 * and u (2N doubles, component-major), physical units of poredvm.h, zero on
 * solid voxels. */
int pdvm_unet_predict(pdvm_unet *net, const uint8_t *solid, double kn, double jump, double *rho, double *u);

/* Average milliseconds of the forward pass and of one training step (forward,
 * backward, Adam) over `reps` repetitions on slots[0..batch), the matrix-core
 * FLOP of each, and the share of the time spent in the MFMA kernels. */
typedef struct {
  double forward_ms, step_ms;
  double forward_flop, step_flop;
  double mfma_ms_per_step;  /* summed durations of the MFMA kernels of one step */
} pdvm_unet_timing;
int pdvm_unet_time(pdvm_unet *net, const int32_t *slots, int32_t batch, int32_t reps, pdvm_unet_timing *out);

void pdvm_unet_destroy(pdvm_unet *net);
const char *pdvm_unet_last_error(const pdvm_unet *net);

#ifdef __cplusplus
}
#endif
#endif /* POREDVM_UNET_H */
