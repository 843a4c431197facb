// Host build of the GPU generator's per-ray code (the same __host__ __device__
// functions the kernel runs), with a per-thread sample cache of K entries
// (K = 0: none; 0 < K < samples: the fallback that samples the volume again).
#include "vdi_generate.hip"

#include <cstdio>
#include <vector>

namespace vdi {
int set_error(int code, const char *fmt, ...)
{
    fprintf(stderr, "vdi_generate host build: %s\n", fmt);
    return code;
}
int hip_error(hipError_t, const char *) { return VDI_ERR_HIP; }
hipError_t library_pool(int, hipMemPool_t *) { return hipErrorNotSupported; }
}  // namespace vdi

extern "C" int host_generate(const vdi_volume *vol, const vdi_gen_params *p, uint8_t *count, float *depth, float *rgba,
                             double *gamma_out, int K)
{
    vdi::GenParams G;
    const int rc = vdi::make_gen_params(vol, p, G);
    if (rc) return rc;
#pragma omp parallel
    {
        std::vector<double2> buf(K > 0 ? K : 1);
        const vdi::SampleCache C = {buf.data(), K, 1};
#pragma omp for schedule(dynamic, 1)
        for (int py = 0; py < p->height; ++py)
            for (int px = 0; px < p->width; ++px)
                vdi::gen_ray(G, C, px, py, count, reinterpret_cast<float2 *>(depth), reinterpret_cast<float4 *>(rgba),
                             gamma_out);
    }
    return 0;
}
