// Arguments of one step of the learned predictor (shared by the predictor's
// own four-launch step and by the predictive persistent frames).
#pragma once

#include <stdint.h>

namespace rtcm {

// One predictor step: modes m = P s + (P D) c and their
// history window; with a full window the network (layer 1 with GELU, layer 2)
// and the forecast change d = y std + mean, else d = 0; the feed-forward
// slopes s_out = s + P^T d / gain.  Matrices are float32 rows padded with zeros
// to a multiple of 4 elements (16-byte aligned rows); network weights are the
// bfloat16 copies, inputs rounded to bfloat16 as they are read.
struct PredStepArgs {
  const float *P;        // [n_modes][ldp]
  int64_t ldp;
  const float *PD;       // [n_modes][ldd]
  int64_t ldd;
  const float *PT;       // [n_slopes][ldt]
  int64_t ldt;
  const float *s;        // [n_slopes] measured slopes
  const float *c;        // [n_act] previous commands
  int n_slopes, n_act, n_modes, history, n_in, n_hid;
  int push;              // a previous frame exists (the window takes a change)
  int full;              // the window holds `history` changes (the network runs)
  float *hist;           // [2 history][n_modes] ring of normalised changes: a change goes to slots
                         // pos and pos + history, so slots pos + 1 .. pos + history are the window
  int pos;               // ring slot of this frame's change
  float *m, *m_prev;     // [n_modes]
  const float *mean, *std_, *inv_std;
  const uint16_t *W1;    // [n_hid][n_in]
  const float *b1;
  const uint16_t *W2;    // [n_modes][n_hid]
  const float *b2;
  float *h;              // [n_hid] hidden activations
  float *d;              // [n_modes] forecast change
  float *modes_out;      // nullable [2 n_modes]: m, then m + d
  float *s_out;          // [n_slopes]
  float inv_gain;
};

}  // namespace rtcm
