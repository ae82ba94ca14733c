#pragma once
#include "coarse.hpp"
namespace pr { struct AsyncWork { int dummy; }; }
