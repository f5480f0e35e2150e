// cx_spec.h -- station spec validation, tree compilation and sampling tables.
#pragma once

#include <string>
#include <vector>

#include "cx_internal.h"

namespace cx {

// Owning copy of a cx_station_spec (the caller's arrays are copied at create).
struct SpecCopy {
  cx_station_spec s;
  std::vector<int32_t> node_parent, port_parent;
  std::vector<double> node_limit, node_eta, port_pmax, port_eta;
  std::vector<double> arrival_rate, price_table;  // empty: the default curves
  std::vector<double> port_pdis;                  // discharge maxima (port maxima if not given)
  std::vector<double> price_days;                 // [n_price_days][steps] (empty: none)
  std::vector<double> car_models;                 // [n_car_models][4] (empty: none)
  std::vector<int32_t> port_dc;                   // [n_ports] (all 0 if not given)
};

// The capacity tree in the kernels' layout.  Aligned layout: every node owns an
// aligned block of 2^b slots; children are placed in port order, each aligned to
// its own block size, so the slot order of ports equals their port order and a
// subtree sum is a butterfly over its block.  Dense layout (chosen when the
// aligned one would pad and every level below the root has at most 4 nodes):
// port i sits in slot i, and a slot's 8-bit level field holds 0x80 | m for the
// level's node m that covers it (0 if none); each node's sum is then a station
// sum of the slots it covers.  Level 0 is the deepest node level, level D-1 the
// root.
struct Compiled {
  int N = 0, S = 0, D = 0;
  std::vector<int32_t> slot_port;   // [S], -1 = padding
  std::vector<int32_t> port_slot;   // [N]
  std::vector<uint32_t> slot_lb;    // [S], 8 bits per level: log2 block size (aligned) or 0x80 | node (dense)
  uint32_t dense_nodes = 0;         // dense layout: nodes per level below the root (8 bits each), 0 = aligned
  std::vector<float> slot_cap;      // [D][S]
  std::vector<float> slot_pmax, slot_inv_pmax, slot_inv_eta;
  std::vector<float> slot_pdis, slot_eta;  // discharge maxima and efficiencies (V2G)
  bool uniform_eta = true;
  float inv_eta_uniform = 1.f;
  bool v2g = false, battery = false;       // ports discharge / a station battery
  bool users = false;                      // some users are charge-sensitive (u = 1)
  int n_days = 0;                          // exploring starts: price days (0: none)
  int n_models = 0;                        // car models (0: none)
  std::vector<uint32_t> model_thresh;      // [8] cumulative thresholds (0xFFFFFFFF past the last)
  std::vector<float> model_data;           // [8][3]: capacity, AC rate, DC rate
  std::vector<int32_t> slot_dc;            // [S] 1 = DC charger
  int day_obs = 0;                         // observation offset of [day / n_days, weekend]
  uint32_t cs_thresh = 0;                  // u = 1 iff the user word <= cs_thresh
  int n_act = 0, obs_dim = 0;              // action bytes and observation floats per env
  int user_obs = 0;                        // observation offset of the user flags
  bool extended() const { return v2g || battery || users || n_days > 0 || n_models > 0; }  // extended kernels
};

struct Tables {
  std::vector<uint32_t> tpois;      // [steps][24] as defined
  std::vector<uint32_t> tpois_dev;  // [steps][32] padded with 0xFFFFFFFF
  std::vector<uint32_t> tdwell;     // [dwell_max], entry 0 unused
  std::vector<uint32_t> tdwell_dev; // [2^dwell_log2]: entries 1.. of tdwell, then 0xFFFFFFFF
  int dwell_log2 = 1;
  std::vector<float> glob;          // [steps][4]
  std::vector<float> price_days;    // [n_days][steps] (exploring starts)
};

bool copy_spec(const cx_station_spec &in, SpecCopy *out, std::string *err);
bool compile_spec(const SpecCopy &sc, Compiled *c, std::string *err);
void build_tables(const SpecCopy &sc, Tables *t);
bool tables_monotone(const Tables &t);

}  // namespace cx
