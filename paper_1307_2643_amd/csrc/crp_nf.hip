// Neural-field kernels of libcrp (placeholder until the MFMA kernels land):
// every entry point reports that the neural field is unavailable.
#include "crp_nf.hpp"

namespace crp {

struct NeuralField {
    hipStream_t stream;
};

NeuralField* nf_create(hipStream_t s) { return new NeuralField{s}; }
void nf_destroy(NeuralField* nf) { delete nf; }

static crp_status unavailable(std::string& err)
{
    err = "neural field: not available in this build";
    return CRP_ESTATE;
}

crp_status nf_load(NeuralField*, const int32_t*, const float*, double, std::string& err)
{
    return unavailable(err);
}
crp_status nf_get(NeuralField*, float*, std::string& err) { return unavailable(err); }
crp_status nf_eval(NeuralField*, const GridView&, int64_t, const double*, double*, hipStream_t)
{
    return CRP_ESTATE;
}
crp_status nf_loss_grad(NeuralField*, const GridView&, int64_t, const double*, const float*,
                        float*, float*, double*, std::string& err)
{
    return unavailable(err);
}
crp_status nf_train(NeuralField*, const GridView&, int64_t, int64_t, double, double, uint64_t,
                    float*, std::string& err)
{
    return unavailable(err);
}
crp_status nf_propagate(NeuralField*, crp_ctx*, int64_t, DevCounters*) { return CRP_ESTATE; }

}  // namespace crp
