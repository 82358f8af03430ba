// Internal interface between the solver and the warm-start network.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "mgwr.h"

namespace mgwr {
// Forward pass of one instance (batch 1, fine-grid spacing h) on the
// network's buffers; *y points at the output [c_L][H][W].
int net_infer(mgwr_net* net, const float* x, int H, int W, double h, const float** y);
int net_signal_channels(const mgwr_net* net);
int net_input_channels(const mgwr_net* net);
int net_out_channels(const mgwr_net* net);
long long net_capacity(const mgwr_net* net);
hipStream_t net_stream(const mgwr_net* net);
// Solver predictions from several threads (batches solved side by side) take
// this lock around gather, inference and interpolation: they share the
// network's buffers and stream.  The input is staged in a network-owned
// buffer so that the captured inference graph always reads one address.
std::mutex& net_mutex(mgwr_net* net);
float* net_input_stage(mgwr_net* net);
// shape checks and the master weights (for loading a weight blob)
bool net_same_shape(const mgwr_net* net, int layers, const int* channels, int nsignal);
bool net_is_bound(const mgwr_net* net);
float* net_params(mgwr_net* net);
size_t net_param_count(const mgwr_net* net);
// split: b (gather) / u (interpolation) in the solver's colour-split storage
// of 2D grids; the network's arrays are in natural order.
hipError_t launch_gather_slices(const double* b, const int* rows, int nslices, long long N, double scale,
                                float alpha, float rdiv, float* x, bool split, hipStream_t s);
hipError_t launch_time_interp(const float* y, const int* rows, int nslices, const double* t, const double* g,
                              long long M, long long N, double scale, double* u, bool split, hipStream_t s);
void set_last_error(const std::string& msg);
}  // namespace mgwr
