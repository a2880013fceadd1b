// Device-side setup phase (Sec. 4.4 of Li, arXiv:1710.04985, the paper's
// LEV_GPU / DEP_GPU route of Table 1): levels, level-ordered layout and level
// pointers computed on the GPU from the caller's device pattern, without
// copying it to the host.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <vector>

namespace sptrsv {

// Device arrays of one analysed triangle (owned by the caller after success;
// free with free_device_analysis).  Same meaning as the HostPlan fields.
struct DeviceAnalysis {
  int n = 0;
  int nlev = 0;
  int64_t noff = 0;
  int max_row_len = 0;
  int* level = nullptr;     // [n]
  int* depcnt = nullptr;    // [n]
  int* jlev = nullptr;      // [n] rows by (level, row)
  int* pos_row = nullptr;   // [n]
  int* off_ptr = nullptr;   // [n+1]
  int* off_col = nullptr;   // [noff]
  int* off_pos = nullptr;   // [noff]
  int* off_src = nullptr;   // [noff]
  int* diag_src = nullptr;  // [n]
  std::vector<int> ilev;    // host: level pointers [nlev+1]
  std::vector<int> off_ptr_h;   // host copy of off_ptr
};

// Analyses the triangle (row_ptr, col) held in device memory.  Returns kOk,
// or kErrNotSupported when the pattern is not one the device path takes
// (an invalid pattern, columns not strictly increasing inside a row, n or
// nnz beyond its limits): the caller then runs the host analysis, which also
// produces the exact validation error.  Other errors: kErrHip, kErrOom,
// kErrTimeout (level kernel spin limit; cannot happen on a valid pattern).
// Blocking: synchronises `stream`.
int device_analysis(int n, int64_t nnz, const int* row_ptr, const int* col, bool upper,
                    bool unit_diag, int num_cu, hipStream_t stream, DeviceAnalysis& out);

void free_device_analysis(DeviceAnalysis& a);

// Pattern of T^T in CSR, on the device: rows of T^T are the columns of T,
// each with its columns (rows of T) strictly increasing; srcT[t] is the entry
// of T that entry t of T^T came from.  The three arrays are allocated here
// (hipFree them).  Blocking.
int device_transpose(int n, int64_t nnz, const int* row_ptr, const int* col, hipStream_t stream,
                     int** rpT, int** colT, int** srcT);

// Rewrites the value sources of an analysis t of T^T (built from the pattern
// of device_transpose, whose sources index T^T's entries) to index the
// forward plan's value buffer instead: off-diagonal o of the forward plan
// holds T's entry off_src_f[o], position k's diagonal entry diag_src_f[k] at
// noff_f + k.  Blocking.
int device_value_sources(int n, int64_t noff_f, const int* off_src_f, const int* diag_src_f,
                         int64_t nnz, const int* srcT, DeviceAnalysis& t, hipStream_t stream);

// One system of a batch: device pattern and values.
struct ConcatSystem {
  const int* row_ptr;
  const int* col;
  const void* vals;
  int n;
  int nnz;
};

// Block-diagonal concatenation of the systems into rp_cat [sum n + 1],
// col_cat [sum nnz] and vals_cat [sum nnz values of vb bytes], on the
// device.  kErrNotSupported if a system's row pointers do not run from 0 to
// its nnz or a column lies outside its own system (the host route then names
// the error).  Blocking.
int device_concat(const std::vector<ConcatSystem>& systems, int vb, int* rp_cat, int* col_cat,
                  void* vals_cat, hipStream_t stream);

}  // namespace sptrsv
