// Exception-to-status translation at the C ABI boundary.
#pragma once

#include <new>

#include "internal.h"

#define HH_API_BEGIN(ctx)                                           \
  if (!(ctx)) return HH_ERR_INVALID_ARG;                            \
  try {                                                             \
    (void)hipSetDevice((ctx)->device);

#define HH_API_END(ctx)                                             \
  }                                                                 \
  catch (const hh_error& e_) {                                      \
    (ctx)->last_error = e_.msg;                                     \
    return e_.st;                                                   \
  }                                                                 \
  catch (const std::bad_alloc&) {                                   \
    (ctx)->last_error = "host allocation failed";                   \
    return HH_ERR_OUT_OF_MEMORY;                                    \
  }                                                                 \
  catch (...) {                                                     \
    (ctx)->last_error = "unexpected internal error";                \
    return HH_ERR_HIP;                                              \
  }                                                                 \
  (ctx)->last_error.clear();                                        \
  return HH_OK;
