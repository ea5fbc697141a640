// ssg_internal.h -- declarations shared by the library's translation units
// (not part of the public C ABI).
#pragma once

// Records msg as the calling thread's last error (what ssg_last_error()
// returns) and returns code.
__attribute__((visibility("hidden"))) int ssg_internal_fail(int code, const char* msg);
// Clears the calling thread's last error.
__attribute__((visibility("hidden"))) void ssg_internal_clear_error();
