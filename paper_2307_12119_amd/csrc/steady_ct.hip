// Row passes of the FP32 steady solve with compensated twiddles (the option
// varsim_options.compensated_twiddles): the same kernel template as steady.hip, instantiated
// with CT = true for the fixed-point modes only, in a translation unit of its own so that the
// two sets compile in parallel.
#include "rowpass.hpp"

namespace vs {

namespace {

template <int N>
hipError_t row_ct_mode(int mode, const PassArgs& a, hipStream_t s) {
  using Cfg = RowCfg<N>;
  if (a.ny < 2 * Cfg::FFTS || a.ny % (2 * Cfg::FFTS)) return hipErrorInvalidValue;
  if (!a.tw.tw32lo || !a.tw.qw32lo) return hipErrorInvalidValue;
  const dim3 grid((a.ny / 2) / Cfg::FFTS, a.n_maps), block(Cfg::THREADS);
  const Cx<float>*tw = a.tw.tw32, *qw = a.tw.qw32, *twl = a.tw.tw32lo, *qwl = a.tw.qw32lo;
  switch (mode) {
    case ROW_HEAD:
      hipLaunchKernelGGL((row_pass_kernel<float, float, N, ROW_HEAD, true>), grid, block, 0, s, a, tw, qw, twl, qwl);
      break;
    case ROW_MERGED:
      hipLaunchKernelGGL((row_pass_kernel<float, float, N, ROW_MERGED, true>), grid, block, 0, s, a, tw, qw, twl, qwl);
      break;
    case ROW_LAST:
      hipLaunchKernelGGL((row_pass_kernel<float, float, N, ROW_LAST, true>), grid, block, 0, s, a, tw, qw, twl, qwl);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_pass_ct(int mode, const PassArgs& a, hipStream_t stream) {
  switch (a.n) {
    case 16: return row_ct_mode<16>(mode, a, stream);
    case 32: return row_ct_mode<32>(mode, a, stream);
    case 64: return row_ct_mode<64>(mode, a, stream);
    case 128: return row_ct_mode<128>(mode, a, stream);
    case 256: return row_ct_mode<256>(mode, a, stream);
    case 512: return row_ct_mode<512>(mode, a, stream);
    case 1024: return row_ct_mode<1024>(mode, a, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace vs
