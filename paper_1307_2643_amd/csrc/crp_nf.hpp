// Neural-field (Fourier-feature MLP) part of libcrp: interface between the
// host runtime and the neural-field kernels.
#pragma once

#include <string>

#include "../../include/crp.h"
#include "crp_internal.hpp"

struct crp_ctx;

namespace crp {

struct NeuralField;

NeuralField* nf_create(hipStream_t s);
void nf_destroy(NeuralField* nf);
crp_status nf_load(NeuralField* nf, const int32_t* freq, const float* params, double b_scale,
                   std::string& err);
crp_status nf_get(NeuralField* nf, float* params, std::string& err);
crp_status nf_eval(NeuralField* nf, const GridView& g, int64_t n, const double* dpos, double* dB,
                   hipStream_t s);
crp_status nf_loss_grad(NeuralField* nf, const GridView& g, int64_t n, const double* pos,
                        const float* target, float* out, float* grad, double* loss,
                        std::string& err);
crp_status nf_train(NeuralField* nf, const GridView& g, int64_t steps, int64_t batch, double lr0,
                    double lr1, uint64_t seed, float* loss_out, std::string& err);
crp_status nf_adam_step(NeuralField* nf, const float* grad, double lr, std::string& err);
void nf_prop_params(const NeuralField* nf, const GridView& g, NFProp* p);

}  // namespace crp
