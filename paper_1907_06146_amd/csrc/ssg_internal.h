// ssg_internal.h -- declarations shared by the library's translation units
// (not part of the public C ABI).
#pragma once

// Records msg as the calling thread's last error (what ssg_last_error()
// returns) and returns code.
__attribute__((visibility("hidden"))) int ssg_internal_fail(int code, const char* msg);
// Clears the calling thread's last error.
__attribute__((visibility("hidden"))) void ssg_internal_clear_error();

// Search kernel with several queries per wavefront (ssg_groups.hip): dtype,
// 16-byte chunks per vector, pool registers per lane, lanes per query,
// persistent (batched) form. Null when no compiled shape fits. The kernel
// takes the search's argument block (ssg_search_common.h) by value.
namespace ssgk {
struct Args;
}
__attribute__((visibility("hidden"))) void (*ssg_internal_group_kernel(int dtype, int dc, int preg,
                                                                        int lanes,
                                                                        bool batched))(ssgk::Args);
