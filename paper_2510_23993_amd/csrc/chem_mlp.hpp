// Surrogate network shared between translation units: parameter layout,
// device weight views and the host-side launchers of the inference kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chem {
namespace mlp {

// 12 -> 256 -> 256 -> 256 -> 10, GELU after the hidden layers
constexpr int NIN = 12, NH = 256, NOUT = 10, NOUT_PAD = 32;
// flat FP32 parameter vector: W1 [NH][NIN], b1, W2 [NH][NH], b2, W3 [NH][NH], b3, W4 [NOUT][NH], b4
constexpr int64_t OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
                  OB3 = OW3 + NH * NH, OW4 = OB3 + NH, OB4 = OW4 + NOUT * NH, NPARAM = OB4 + NOUT;
static_assert(NPARAM == 137482, "parameter count");

// BF16 copies of the dense layers for the MFMA inference kernel (W4 padded
// to 32 output rows with zeros); element counts
// (and the first layer, K = 12 padded to 16, as high and low BF16 parts)
constexpr int64_t NW2H = NH * NH, NW3H = NH * NH, NW4H = NOUT_PAD * NH, NW1H = 2 * NH * 16,
                  NBF16 = NW2H + NW3H + NW4H + NW1H;

struct MlpDev {
    const float* p;          // FP32 parameters (W1, biases read from here)
    const uint16_t* w2h;     // BF16 [NH][NH]
    const uint16_t* w3h;     // BF16 [NH][NH]
    const uint16_t* w4h;     // BF16 [NOUT_PAD][NH]
    const uint16_t* w1h;     // BF16 hi then lo parts of W1, fragments of [NH][16]
};

// Convert the FP32 dense weights to the BF16 copies (round to nearest even).
int convert_bf16(hipStream_t s, const float* params, uint16_t* bf16);
// out[r][10] = network(X[r][12]) for r < *rows_dev (or rows_host when
// rows_dev is NULL); BF16 MFMA with FP32 accumulation.
int launch_infer(hipStream_t s, const MlpDev& w, int64_t rows_host, const int* rows_dev, int64_t max_rows,
                 const float* X, float* out, int ncu);

}  // namespace mlp
}  // namespace chem
