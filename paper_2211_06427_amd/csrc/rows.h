// Launchers of the assembly kernels (each defined in its own translation unit).
#pragma once

#include "rules.h"

template <typename T>
void launch_rows(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s);
void launch_rows_bf16x3(const wq_rules* H, uint32_t which, const float* kappa, float* vm, float* vk, hipStream_t s);
// buf == nullptr: scratch from the handle's pool; else the caller's device buffer of cap bytes
template <typename T>
int launch_cut(const wq_rules* H, uint32_t which, uint32_t parts, const T* kappa, T* vm, T* vk, hipStream_t s,
               void* buf = nullptr, size_t cap = 0);
template <typename T>
int launch_adjoint(const wq_rules* H, uint32_t which, const T* gm, const T* gk, T* dk, hipStream_t s);
template <typename T>
int launch_gauss(const wq_rules* H, uint32_t which, const T* kg, const T* kappa, T* vm, T* vk, hipStream_t s);
int launch_gauss_coords(const wq_rules* H, double* xyz, hipStream_t s);
template <typename T>
int launch_tensor(const wq_rules* H, const T* C, T* vk, hipStream_t s);   // tensor.hip
// fused assembly (wq_assemble): rows split over two streams (rows.hip); the cut part's element
// work and remainder on two streams, then the gather (cut.hip)
template <typename T>
void launch_rows_split(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s_int, hipStream_t s_cut);
template <typename T>
size_t cut_fused_scratch_bytes(const wq_rules* H);
template <typename T>
int launch_cut_prep(const wq_rules* H, uint32_t which, const T* kappa, T* vm, T* vk, hipStream_t s_rem, hipStream_t s_oct,
                    void* scratch);
template <typename T>
void launch_cut_finish(const wq_rules* H, uint32_t which, const void* scratch, T* vm, T* vk, hipStream_t s);
template <typename T>
int launch_tensor_cut(const wq_rules* H, const T* C, T* vk, hipStream_t s);   // cut.hip: cut elements, moment form

// L2 projection (projection.hip)
int projection_load_vector(const wq_rules* H, const double* f, double* b, hipStream_t s);
int projection_build_extension(const wq_rules* H, hipStream_t s, wq_extension** out);
int projection_info(const wq_extension* X, wq_extension_info* out);
void projection_free(wq_extension* X);
const wq_rules* projection_owner(const wq_extension* X);
int projection_solve(const wq_rules* H, const wq_extension* X, const double* M, const double* b, double* u,
                     double tol, int32_t max_iter, int32_t* iters, double* relres, hipStream_t s);
int projection_error(const wq_rules* H, const double* u, const double* fg, const double* f, double* out,
                     hipStream_t s);
